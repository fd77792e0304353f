// exx_kernels.hip -- HIP kernels (gfx950) of the pair-Poisson exact-exchange
// path of Ko et al., arXiv:1911.10630, Sec. III.C Steps III-V.
//
//   k_solve   persistent: one work-group owns one pair at a time, pulled from a
//             queue; gather + pair density + multipoles (Eq. mepole), shell
//             potential (Eq. me), boundary-charge right-hand side
//             (Eq. pe_mat_red), conjugate gradient on the 19-point stencil
//             (Eq. d2_1), pair energy (Eq. exx_omega).  Every reduction is a
//             fixed-order work-group tree, so results are bitwise
//             reproducible whatever the scheduling.
//   k_dxx     owner-computes accumulation of D^k = sum_j v_kj phi_j over the
//             pairs of each orbital, in pair order (Eq. Dxx_mlwf_omega);
//             no atomics.
//   k_energy  E_xx = -sum w_ij e_ij in pair order, one work-group.
#include "exx_internal.h"

namespace exx {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int wrap_n(int v, int n)
{
    v = v < 0 ? v + n : v;
    return v >= n ? v - n : v;
}

__device__ __forceinline__ double load_phi(const void *phi, int f32, long long idx)
{
    return f32 ? (double)(static_cast<const float *>(phi)[idx]) : static_cast<const double *>(phi)[idx];
}

// Unnormalized real regular solid harmonics U_lm(x, y, z), index l*l + l + m:
//   U_l,+m = Pi_l^m(z, r^2) Re (x + i y)^m,  U_l,-m = Pi_l^m Im (x + i y)^m,
// with Pi_m^m = (2m-1)!!, Pi_{m+1}^m = (2m+1) z Pi_m^m and
//   (l - m) Pi_l^m = (2l-1) z Pi_{l-1}^m - (l+m-1) r^2 Pi_{l-2}^m,
// i.e. r^l times the associated Legendre functions without the
// Condon-Shortley phase.  R_lm = norm_lm U_lm are orthonormal solid
// harmonics, r^l S_lm(rhat); sum_m Q_lm R_lm equals the complex-form
// sum of Eqs. me / mepole by the addition theorem.
__device__ __forceinline__ void solid_u(double x, double y, double z, double *U)
{
    const double r2 = x * x + y * y + z * z;
    double A[LMAX + 1], B[LMAX + 1];
    A[0] = 1.0;
    B[0] = 0.0;
#pragma unroll
    for (int m = 1; m <= LMAX; ++m) {
        A[m] = x * A[m - 1] - y * B[m - 1];
        B[m] = x * B[m - 1] + y * A[m - 1];
    }
    constexpr double dfact[LMAX + 1] = {1.0, 1.0, 3.0, 15.0, 105.0, 945.0, 10395.0};
#pragma unroll
    for (int m = 0; m <= LMAX; ++m) {
        double p2 = 0.0, p1 = dfact[m];
        U[m * m + 2 * m] = p1 * A[m];
        if (m > 0) U[m * m] = p1 * B[m];
#pragma unroll
        for (int l = m + 1; l <= LMAX; ++l) {
            const double pl = ((2 * l - 1) * z * p1 - (l + m - 1) * r2 * p2) * (1.0 / (l - m));
            p2 = p1;
            p1 = pl;
            U[l * l + l + m] = pl * A[m];
            if (m > 0) U[l * l + l - m] = pl * B[m];
        }
    }
}

template <int BLOCK>
__device__ __forceinline__ double block_sum(double v, double *red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < BLOCK / 64; ++k) s += red[k];
    __syncthreads();
    return s;
}

// PE packed index of offset (x, y, z), or -1 if outside PE.
__device__ __forceinline__ int pe_index(const ClassDev &g, int x, int y, int z)
{
    const int zz = z - g.pzlo, yy = y - g.pylo;
    if ((unsigned)zz >= (unsigned)g.pnz || (unsigned)yy >= (unsigned)g.pny) return -1;
    const int4 r = g.pe_rows[zz * g.pny + yy];
    if (x < r.y || x > r.z) return -1;
    return r.x + x - r.y;
}

// Shell packed index of an offset known to lie in ME but not in PE.
__device__ __forceinline__ int sh_index(const ClassDev &g, int x, int y, int z)
{
    const int row = (z - g.mzlo) * g.mny + (y - g.mylo);
    const int4 a = g.me_rows[2 * row];
    const int4 b = g.me_rows[2 * row + 1];
    return a.w + (x < a.y ? x - b.x : (a.y - b.x) + (x - a.z - 1));
}

// (A u)_q for packed PE vector u, A = -(discrete Laplacian restricted to PE).
__device__ __forceinline__ double apply_A_flat(const ClassDev &g, const double *u, int q, int x, int y, int z,
                                               const double (&w)[3][4])
{
    double c = (w[0][0] + w[1][0] + w[2][0]) * u[q];
    const int4 row = g.pe_rows[(z - g.pzlo) * g.pny + (y - g.pylo)];
#pragma unroll
    for (int s = 1; s <= FD_N; ++s) {
        if (x - s >= row.y) c += w[0][s] * u[q - s];
        if (x + s <= row.z) c += w[0][s] * u[q + s];
    }
#pragma unroll
    for (int s = 1; s <= FD_N; ++s) {
#pragma unroll
        for (int sg = -1; sg <= 1; sg += 2) {
            int k = pe_index(g, x, y + sg * s, z);
            if (k >= 0) c += w[1][s] * u[k];
            k = pe_index(g, x, y, z + sg * s);
            if (k >= 0) c += w[2][s] * u[k];
        }
    }
    return -c;
}

// ---------------------------------------------------------------------------
// pair preparation: one work-group per pair of the wave
// ---------------------------------------------------------------------------

__device__ __forceinline__ void fd_weights(const SolveArgs &a, double (&w)[3][4])
{
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        w[0][s] = a.wfd[s] / (a.h[0] * a.h[0]);
        w[1][s] = a.wfd[s] / (a.h[1] * a.h[1]);
        w[2][s] = a.wfd[s] / (a.h[2] * a.h[2]);
    }
}

__device__ __forceinline__ long long grid_index(const SolveArgs &a, const int4 &pg, int x, int y, int z)
{
    const int gx = wrap_n(pg.x + x, a.nx), gy = wrap_n(pg.y + y, a.ny), gz = wrap_n(pg.z + z, a.nz);
    return ((long long)gz * a.ny + gy) * a.nx + gx;
}

constexpr int PREP_BLOCK = 256;

// Gather of phi_i, phi_j on PE and the pair density rho_ij (Step III, Eq. l2g),
// moments Q_lm (Eq. mepole), far-field potential on the shell (Eq. me) and the
// boundary-charge right-hand side b = 4 pi rho + sum_shell w v / h^2
// (Eq. pe_mat_red).  b is first used to hold rho (same thread, same index).
__global__ __launch_bounds__(PREP_BLOCK) void k_prep(SolveArgs a)
{
    __shared__ double red[PREP_BLOCK / 64][NLM];
    __shared__ double qs[NLM];
    const int tid = threadIdx.x;
    const int pair = a.wave_begin + blockIdx.x;
    const int4 pg = a.pair_gc[pair];
    const int2 ij = a.pair_ij[pair];
    const ClassDev g = pg.w ? a.cls[1] : a.cls[0];
    double *v_sh = a.vout + a.out_off[pair] + g.n_pe;
    double *bv = a.rhs + (long long)blockIdx.x * a.slot_n;
    double *keep = a.rho_keep ? a.rho_keep + (long long)pair * a.slot_n : nullptr;
    const double hx = a.h[0], hy = a.h[1], hz = a.h[2];
    const long long oi = (long long)ij.x * a.ngrid, oj = (long long)ij.y * a.ngrid;
    double w[3][4];
    fd_weights(a, w);

    double acc[NLM];
#pragma unroll
    for (int k = 0; k < NLM; ++k) acc[k] = 0.0;
    for (int q = tid; q < g.n_pe; q += PREP_BLOCK) {
        int x, y, z;
        unpack_xyz(g.pe_xyz[q], x, y, z);
        const long long gi = grid_index(a, pg, x, y, z);
        const double rv = load_phi(a.phi, a.phi_f32, oi + gi) * load_phi(a.phi, a.phi_f32, oj + gi);
        bv[q] = rv;
        if (keep) keep[q] = rv;
        double U[NLM];
        solid_u(x * hx, y * hy, z * hz, U);
#pragma unroll
        for (int k = 0; k < NLM; ++k) acc[k] += rv * U[k];
    }
    {
        const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
        for (int k = 0; k < NLM; ++k) {
            double v = acc[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) red[wv][k] = v;
        }
        __syncthreads();
        if (tid < NLM) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < PREP_BLOCK / 64; ++k) s += red[k][tid];
            int l = 0;
            while ((l + 1) * (l + 1) <= tid) ++l;
            const double Q = s * (hx * hy * hz) * a.ylm_norm[tid];
            a.q_out[(long long)pair * NLM + tid] = Q;
            qs[tid] = Q * a.ylm_norm[tid] * (4.0 * M_PI / (2 * l + 1));
        }
        __syncthreads();
    }
    for (int s = tid; s < g.n_sh; s += PREP_BLOCK) {
        int x, y, z;
        unpack_xyz(g.sh_xyz[s], x, y, z);
        const double X = x * hx, Y = y * hy, Z = z * hz;
        const double r2 = X * X + Y * Y + Z * Z;
        double U[NLM];
        solid_u(X, Y, Z, U);
        const double inv_r2 = 1.0 / r2;
        double f = 1.0 / sqrt(r2);
        double v = 0.0;
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) {
            double t = 0.0;
#pragma unroll
            for (int m = -l; m <= l; ++m) t += qs[l * l + l + m] * U[l * l + l + m];
            v += f * t;
            f *= inv_r2;
        }
        v_sh[s] = v;
    }
    __syncthreads();
    for (int q = tid; q < g.n_pe; q += PREP_BLOCK) {
        int x, y, z;
        unpack_xyz(g.pe_xyz[q], x, y, z);
        double bq = 4.0 * M_PI * bv[q];
#pragma unroll
        for (int s = 1; s <= FD_N; ++s) {
#pragma unroll
            for (int sg = -1; sg <= 1; sg += 2) {
                const int d = sg * s;
                if (pe_index(g, x + d, y, z) < 0) bq += w[0][s] * v_sh[sh_index(g, x + d, y, z)];
                if (pe_index(g, x, y + d, z) < 0) bq += w[1][s] * v_sh[sh_index(g, x, y + d, z)];
                if (pe_index(g, x, y, z + d) < 0) bq += w[2][s] * v_sh[sh_index(g, x, y, z + d)];
            }
        }
        bv[q] = bq;
    }
}

// ---------------------------------------------------------------------------
// conjugate gradient: persistent, one work-group per pair (Step IV)
// ---------------------------------------------------------------------------

template <int BLOCK>
__device__ void cg_one_pair(const SolveArgs &a, int pair, long long slot, double *red)
{
    const int tid = threadIdx.x;
    const int4 pg = a.pair_gc[pair];
    const int2 ij = a.pair_ij[pair];
    const ClassDev g = pg.w ? a.cls[1] : a.cls[0];
    double *xv = a.vout + a.out_off[pair];
    const double *bv = a.rhs + (long long)(pair - a.wave_begin) * a.slot_n;
    double *r = a.scratch + slot * 3 * a.slot_n;
    double *p = r + a.slot_n;
    double *ap = p + a.slot_n;
    double w[3][4];
    fd_weights(a, w);
    const int n = g.n_pe;

    double bb = 0.0;
    for (int q = tid; q < n; q += BLOCK) {
        const double bq = bv[q];
        r[q] = bq;
        p[q] = bq;
        xv[q] = 0.0;
        bb += bq * bq;
    }
    bb = block_sum<BLOCK>(bb, red);

    double rr = bb;
    const double stop = a.tol * a.tol * bb;
    int k = 0, conv = 0;
    for (;;) {
        if (rr <= stop) { conv = 1; break; }
        if (k >= a.maxit) break;
        double pap = 0.0;
        for (int q = tid; q < n; q += BLOCK) {
            int x, y, z;
            unpack_xyz(g.pe_xyz[q], x, y, z);
            const double t = apply_A_flat(g, p, q, x, y, z, w);
            ap[q] = t;
            pap += p[q] * t;
        }
        pap = block_sum<BLOCK>(pap, red);
        const double alpha = rr / pap;
        double rn = 0.0;
        for (int q = tid; q < n; q += BLOCK) {
            xv[q] += alpha * p[q];
            const double t = r[q] - alpha * ap[q];
            r[q] = t;
            rn += t * t;
        }
        rn = block_sum<BLOCK>(rn, red);
        const double beta = rn / rr;
        rr = rn;
        for (int q = tid; q < n; q += BLOCK) p[q] = r[q] + beta * p[q];
        __syncthreads();
        ++k;
    }

    // pair energy with the re-gathered density (Step V, Eq. exx_omega) and the
    // true residual ||b - A x|| / ||b||
    const long long oi = (long long)ij.x * a.ngrid, oj = (long long)ij.y * a.ngrid;
    double e = 0.0, res = 0.0;
    for (int q = tid; q < n; q += BLOCK) {
        int x, y, z;
        unpack_xyz(g.pe_xyz[q], x, y, z);
        const long long gi = grid_index(a, pg, x, y, z);
        const double rv = load_phi(a.phi, a.phi_f32, oi + gi) * load_phi(a.phi, a.phi_f32, oj + gi);
        e += rv * xv[q];
        const double d = bv[q] - apply_A_flat(g, xv, q, x, y, z, w);
        res += d * d;
    }
    e = block_sum<BLOCK>(e, red);
    res = block_sum<BLOCK>(res, red);
    if (tid == 0) {
        a.e_out[pair] = e * (a.h[0] * a.h[1] * a.h[2]);
        a.iters_out[pair] = k;
        a.conv_out[pair] = conv;
        a.relres_out[pair] = bb > 0.0 ? sqrt(res / bb) : 0.0;
    }
    __syncthreads();
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_solve(SolveArgs a)
{
    __shared__ double red[BLOCK / 64];
    __shared__ int s_pair;
    for (int it = 0;; ++it) {
        int k;
        if (a.static_sched) {
            k = blockIdx.x + it * gridDim.x;
        } else {
            if (threadIdx.x == 0) s_pair = atomicAdd(a.counter, 1);
            __syncthreads();
            k = s_pair;
            __syncthreads();
        }
        if (k >= a.wave_n) break;
        cg_one_pair<BLOCK>(a, a.wave_begin + k, blockIdx.x, red);
    }
}

// ---------------------------------------------------------------------------
// D accumulation: owner computes, pair order, no atomics
// ---------------------------------------------------------------------------

constexpr int DXX_BLOCK = 256;
constexpr int DXX_PER_THREAD = 4;
constexpr int DXX_TILE = DXX_BLOCK * DXX_PER_THREAD;

template <typename TO>
__global__ __launch_bounds__(DXX_BLOCK) void k_dxx(DxxArgs a)
{
    const int k = blockIdx.y;
    const long long t0 = (long long)blockIdx.x * DXX_TILE;
    double acc[DXX_PER_THREAD];
    int gx[DXX_PER_THREAD], gy[DXX_PER_THREAD], gz[DXX_PER_THREAD];
    bool ok[DXX_PER_THREAD];
#pragma unroll
    for (int e = 0; e < DXX_PER_THREAD; ++e) {
        const long long gi = t0 + e * DXX_BLOCK + threadIdx.x;
        ok[e] = gi < a.ngrid;
        const long long gl = ok[e] ? gi : 0;
        gx[e] = (int)(gl % a.nx);
        gy[e] = (int)((gl / a.nx) % a.ny);
        gz[e] = (int)(gl / ((long long)a.nx * a.ny));
        acc[e] = 0.0;
    }
    const int pb = a.orb_ptr[k], pe = a.orb_ptr[k + 1];
    for (int pp = pb; pp < pe; ++pp) {
        const int pair = a.orb_pairs[pp];
        const int4 pg = a.pair_gc[pair];
        const int2 ij = a.pair_ij[pair];
        const int other = ij.x == k ? ij.y : ij.x;
        const ClassDev g = pg.w ? a.cls[1] : a.cls[0];
        const double *v = a.vout + a.out_off[pair];
        const long long oo = (long long)other * a.ngrid;
#pragma unroll
        for (int e = 0; e < DXX_PER_THREAD; ++e) {
            if (!ok[e]) continue;
            int tx = gx[e] - pg.x - g.mxlo, ty = gy[e] - pg.y - g.mylo, tz = gz[e] - pg.z - g.mzlo;
            tx = wrap_n(tx, a.nx);
            ty = wrap_n(ty, a.ny);
            tz = wrap_n(tz, a.nz);
            if (tx >= g.mnx || ty >= g.mny || tz >= g.mnz) continue;
            const int row = tz * g.mny + ty;
            const int4 r0 = g.me_rows[2 * row];
            const int4 r1 = g.me_rows[2 * row + 1];
            const int ox = tx + g.mxlo;
            if (ox < r1.x || ox > r1.y) continue;
            double vv;
            if (ox >= r0.y && ox <= r0.z)
                vv = v[r0.x + ox - r0.y];
            else
                vv = v[g.n_pe + r0.w + (ox < r0.y ? ox - r1.x : (r0.y - r1.x) + (ox - r0.z - 1))];
            const long long gi = t0 + e * DXX_BLOCK + threadIdx.x;
            acc[e] += vv * load_phi(a.phi, a.f32, oo + gi);
        }
    }
    TO *out = static_cast<TO *>(a.dxx) + (long long)k * a.ngrid;
#pragma unroll
    for (int e = 0; e < DXX_PER_THREAD; ++e) {
        const long long gi = t0 + e * DXX_BLOCK + threadIdx.x;
        if (ok[e]) out[gi] = (TO)acc[e];
    }
}

// ---------------------------------------------------------------------------
// E reduction and small utilities
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(1024) void k_energy(const double *e, const int2 *ij, int n, double *out)
{
    __shared__ double red[16];
    double s = 0.0;
    for (int p = threadIdx.x; p < n; p += 1024) {
        const int2 q = ij[p];
        s += (q.x == q.y ? 1.0 : 2.0) * e[p];
    }
    s = block_sum<1024>(s, red);
    if (threadIdx.x == 0) out[0] = -s;
}

__global__ void k_zero_int(int *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static const int kBlocks[] = {256, 512};

int solve_block_sizes(int *out, int max_n)
{
    int n = 0;
    for (int b : kBlocks)
        if (n < max_n) out[n++] = b;
    return n;
}

hipError_t solve_occupancy(int block, int *blocks_per_cu)
{
    switch (block) {
    case 256: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_solve<256>, 256, 0);
    case 512: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_solve<512>, 512, 0);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_prep(const SolveArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_prep, dim3(a.wave_n), dim3(PREP_BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_solve(const SolveArgs &a, int grid, int block, hipStream_t s)
{
    switch (block) {
    case 256: hipLaunchKernelGGL(k_solve<256>, dim3(grid), dim3(256), 0, s, a); break;
    case 512: hipLaunchKernelGGL(k_solve<512>, dim3(grid), dim3(512), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dxx(const DxxArgs &a, int n_orb, hipStream_t s)
{
    const dim3 grid((unsigned)((a.ngrid + DXX_TILE - 1) / DXX_TILE), (unsigned)n_orb);
    if (a.f32)
        hipLaunchKernelGGL(k_dxx<float>, grid, dim3(DXX_BLOCK), 0, s, a);
    else
        hipLaunchKernelGGL(k_dxx<double>, grid, dim3(DXX_BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_energy(const double *e, const int2 *ij, int n_pairs, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(1024), 0, s, e, ij, n_pairs, out);
    return hipGetLastError();
}

hipError_t launch_zero_int(int *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_int, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace exx
