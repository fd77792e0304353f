// exx_kernels.hip -- HIP kernels (gfx950) of the pair-Poisson exact-exchange
// path of Ko et al., arXiv:1911.10630, Sec. III.C Steps III-V (the D
// accumulation of Step V is in exx_dxx.hip).
//
//   k_prep        one work-group per pair: gather and pair density (Eq. l2g),
//                 multipoles (Eq. mepole), shell potential (Eq. me) and the
//                 boundary-charge right-hand side (Eq. pe_mat_red).
//   k_cg_zmarch   persistent: one work-group owns one pair at a time, pulled
//                 from a queue; conjugate gradient on the 19-point stencil
//                 (Eq. d2_1) marching z planes with a register queue (FP64,
//                 FP32 with FP64 reliable updates, or multigrid-preconditioned),
//                 then the true residual.  k_solve is the flat form for
//                 spheres whose planes do not fit the LDS.
//   k_pair_energy e_ij = h^3 sum_PE rho_ij v_ij (Eq. exx_omega), one
//                 work-group per pair.
//   k_energy      E_xx = -sum w_ij e_ij in pair order, one work-group.
// Every reduction is a fixed-order work-group tree, so results are bitwise
// reproducible whatever the scheduling.
#include "exx_internal.h"

#include <algorithm>
#include <type_traits>

namespace exx {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Unnormalized real regular solid harmonics U_lm(x, y, z), index l*l + l + m:
//   U_l,+m = Pi_l^m(z, r^2) Re (x + i y)^m,  U_l,-m = Pi_l^m Im (x + i y)^m,
// with Pi_m^m = (2m-1)!!, Pi_{m+1}^m = (2m+1) z Pi_m^m and
//   (l - m) Pi_l^m = (2l-1) z Pi_{l-1}^m - (l+m-1) r^2 Pi_{l-2}^m,
// i.e. r^l times the associated Legendre functions without the
// Condon-Shortley phase.  R_lm = norm_lm U_lm are orthonormal solid
// harmonics, r^l S_lm(rhat); sum_m Q_lm R_lm equals the complex-form
// sum of Eqs. me / mepole by the addition theorem.
// Each value is handed to use(l, index, U) as soon as it is formed (m-major
// order), so a caller that folds it into a sum never holds all 49.
template <class Use>
__device__ __forceinline__ void solid_u(double x, double y, double z, Use &&use)
{
    const double r2 = x * x + y * y + z * z;
    double A = 1.0, B = 0.0;
    constexpr double dfact[LMAX + 1] = {1.0, 1.0, 3.0, 15.0, 105.0, 945.0, 10395.0};
#pragma unroll
    for (int m = 0; m <= LMAX; ++m) {
        if (m > 0) {
            const double An = x * A - y * B;
            B = x * B + y * A;
            A = An;
        }
        double p2 = 0.0, p1 = dfact[m];
        use(m, m * m + 2 * m, p1 * A);
        if (m > 0) use(m, m * m, p1 * B);
#pragma unroll
        for (int l = m + 1; l <= LMAX; ++l) {
            const double pl = ((2 * l - 1) * z * p1 - (l + m - 1) * r2 * p2) * (1.0 / (l - m));
            p2 = p1;
            p1 = pl;
            use(l, l * l + l + m, pl * A);
            if (m > 0) use(l, l * l + l - m, pl * B);
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

// rho_ij at offset (x, y, z) from the pair origin (Eq. l2g): the two
// orbitals read from their boxes at the wrapped grid point.
__device__ __forceinline__ double pair_rho(const SolveArgs &a, const int4 &pg, long long oi, long long oj, int4 org_i,
                                           int4 org_j, int x, int y, int z)
{
    const int gx = wrap_n(pg.x + x, a.nx), gy = wrap_n(pg.y + y, a.ny), gz = wrap_n(pg.z + z, a.nz);
    return load_orb(a.phi, a.phi_f32, a.box, oi, org_i, gx, gy, gz, a.nx, a.ny, a.nz) *
           load_orb(a.phi, a.phi_f32, a.box, oj, org_j, gx, gy, gz, a.nx, a.ny, a.nz);
}

constexpr int PREP_BLOCK = 256;

// Gather of phi_i, phi_j on PE and the pair density rho_ij (Step III, Eq. l2g),
// moments Q_lm (Eq. mepole), far-field potential on the shell (Eq. me) and the
// boundary-charge right-hand side b = 4 pi rho + sum_shell w v / h^2
// (Eq. pe_mat_red).  b first holds 4 pi rho; the shell term is then added
// to the PE points of the class's coupling list only, in stencil order.
__global__ __launch_bounds__(PREP_BLOCK) void k_prep(SolveArgs a)
{
    __shared__ double red[PREP_BLOCK / 64][NLM];
    __shared__ double qs[NLM];
    __shared__ double wsh[3 * FD_N];   // stencil weight of axis a, distance s at a * 3 + s - 1
    const int tid = threadIdx.x;
    const int pair = a.wave_begin + blockIdx.x;
    const int4 pg = a.pair_gc[pair];
    const int2 ij = a.pair_ij[pair];
    const ClassDev g = a.cls[pg.w];
    double *v_sh = a.vout + a.out_off[pair] + g.n_pe;
    double *bv = a.rhs + a.rhs_off[pair];
    double *keep = a.rho_keep ? a.rho_keep + (long long)pair * a.slot_n : nullptr;
    const double hx = a.h[0], hy = a.h[1], hz = a.h[2];
    const long long oi = (long long)ij.x * a.box.vol, oj = (long long)ij.y * a.box.vol;
    const int4 org_i = a.box.org[ij.x], org_j = a.box.org[ij.y];
    if (tid < 3 * FD_N) wsh[tid] = a.wfd[tid % FD_N + 1] / (a.h[tid / FD_N] * a.h[tid / FD_N]);

    double acc[NLM];
#pragma unroll
    for (int k = 0; k < NLM; ++k) acc[k] = 0.0;
    for (int q = tid; q < g.n_pe; q += PREP_BLOCK) {
        int x, y, z;
        unpack_xyz(g.pe_xyz[q], x, y, z);
        const double rv = pair_rho(a, pg, oi, oj, org_i, org_j, x, y, z);
        bv[q] = 4.0 * M_PI * rv;
        if (keep) keep[q] = rv;
        solid_u(x * hx, y * hy, z * hz, [&](int, int k, double u) { acc[k] += rv * u; });
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
        double t[LMAX + 1];
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) t[l] = 0.0;
        solid_u(X, Y, Z, [&](int l, int k, double u) { t[l] += qs[k] * u; });
        const double inv_r2 = 1.0 / r2;
        double f = 1.0 / sqrt(r2);
        double v = 0.0;
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) {
            v += f * t[l];
            f *= inv_r2;
        }
        v_sh[s] = v;
    }
    __syncthreads();
    // boundary charge: only the PE points next to the shell receive any
    for (int t = tid; t < g.n_bnd; t += PREP_BLOCK) {
        const int q = g.bnd_q[t];
        double bq = bv[q];
        for (int e = g.bnd_ptr[t]; e < g.bnd_ptr[t + 1]; ++e) {
            const int ent = g.bnd_ent[e];
            bq += wsh[ent & 15] * v_sh[ent >> 4];
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
    const ClassDev g = a.cls[pg.w];
    double *xv = a.vout + a.out_off[pair];
    const double *bv = a.rhs + a.rhs_off[pair];
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

    // true residual ||b - A x|| / ||b|| (the pair energy is k_pair_energy's)
    double res = 0.0;
    for (int q = tid; q < n; q += BLOCK) {
        int x, y, z;
        unpack_xyz(g.pe_xyz[q], x, y, z);
        const double d = bv[q] - apply_A_flat(g, xv, q, x, y, z, w);
        res += d * d;
    }
    res = block_sum<BLOCK>(res, red);
    if (tid == 0) {
        a.iters_out[pair] = k;
        a.outer_out[pair] = 0;
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
    if (a.clock && threadIdx.x == 0) atomicMin(&a.clock[0], (unsigned long long)wall_clock64());
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
        cg_one_pair<BLOCK>(a, a.queue ? a.queue[a.wave_begin + k] : a.wave_begin + k, blockIdx.x, red);
    }
    if (a.clock && threadIdx.x == 0) atomicMax(&a.clock[1], (unsigned long long)wall_clock64());
}

// ---------------------------------------------------------------------------
// z-marching CG: one work-group per pair, register queue along z
// ---------------------------------------------------------------------------
//
// Each thread owns xy columns of the PE sphere (up to K per band) and marches
// through the planes z.  For every owned column it keeps the seven planes
// z-3..z+3 of the stencil operand in registers; the current plane is written
// to an LDS plane (zero-padded by 3 on every side) so the x and y neighbours
// come from LDS.  Every vector element is therefore read from memory once
// per pass.  Columns are split into y bands when they do not fit K per
// thread; a band also loads the current plane of its 3 halo rows on each
// side.  Loads of the next plane are issued before the LDS barrier, which
// waits on LDS traffic only, so they overlap the stencil arithmetic.
//
// A CG iteration is two passes:
//   direction  u = r + beta p_old (p_old and p_new in two buffers, so a later
//              band's halo still sees p_old), store p_new, accumulate p.Ap;
//   update     u = p, x += alpha p at load time, r -= alpha Ap at output
//              time, accumulate r.r.
// The final pass recomputes the true residual b - A x (the pair energy is
// k_pair_energy's).

__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Packed index of PE element (x, pylo + ry, z), or -1 when outside PE.
__device__ __forceinline__ int zaddr(const ClassDev &g, int z, int ry, int x)
{
    const int zz = z - g.pzlo;
    if ((unsigned)zz >= (unsigned)g.pnz) return -1;
    const int4 r = g.pe_rows[zz * g.pny + ry];
    return (x >= r.y && x <= r.z) ? r.x + x - r.y : -1;
}

template <typename R>
struct StencilW {
    R c, x[4], y[4], z[4];
};

template <typename R>
__device__ __forceinline__ StencilW<R> stencil_w(const SolveArgs &a)
{
    StencilW<R> w;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        w.x[s] = (R)(a.wfd[s] / (a.h[0] * a.h[0]));
        w.y[s] = (R)(a.wfd[s] / (a.h[1] * a.h[1]));
        w.z[s] = (R)(a.wfd[s] / (a.h[2] * a.h[2]));
    }
    w.c = (R)(a.wfd[0] / (a.h[0] * a.h[0]) + a.wfd[0] / (a.h[1] * a.h[1]) + a.wfd[0] / (a.h[2] * a.h[2]));
    return w;
}

// The march is written without divergent branches: invalid columns load from
// index 0 and select zero, store through a pointer redirected to a sink, and
// write their LDS value to a sink slot.  Divergent branches around loads make
// the compiler wait for every outstanding load (the next plane's prefetch
// included) at each join.
// Load from a (or from index 0 when a < 0: always valid memory); the caller
// discards the value of invalid lanes when it consumes it, one plane later,
// so the load stays in flight until then.
template <typename T>
__device__ __forceinline__ T raw_load(const T *p, int a)
{
    return p[a >= 0 ? a : 0];
}

// policies that declare kXYZ receive each point's local offsets
template <class P, class = void>
struct wants_xyz : std::false_type {};
template <class P>
struct wants_xyz<P, std::void_t<decltype(P::kXYZ)>> : std::true_type {};

template <typename T>
__device__ __forceinline__ T *sel_ptr(T *p, int a, T *sink)
{
    return a >= 0 ? p + a : sink;
}

// Planes of loads in flight.  A policy holds its loaded values in kSlots
// slots: with one slot the loads of the plane the next step consumes are
// issued one step ahead; with two, two steps ahead (the z loop is unrolled
// by two so each slot index is a constant), which hides twice the memory
// latency at the register cost of a second copy of the loaded values.
template <typename R, int T, int K, int KH, class P>
__device__ __forceinline__ void zmarch_band(const ClassDev &g, int bi, double *lds, int &par, P &pol,
                                            const StencilW<R> &w, const int4 &pg, int nx, int ny, int nz)
{
    constexpr int PF = P::kSlots;
    static_assert(PF == 1 || PF == 2, "one or two planes of loads in flight");
    const int tid = threadIdx.x;
    constexpr bool F32 = sizeof(R) == 4;
    const int *bd = (F32 ? g.bands32 : g.bands) + 12 * bi;
    const int plane = F32 ? g.lds_plane32 : g.lds_plane;
    const int c0 = bd[0], c1 = bd[1], h0 = bd[2], h1 = bd[3], h2 = bd[4], h3 = bd[5], zlo = bd[6], zhi = bd[7];
    const int ya = bd[8];
    const int W = g.lds_w;
    const int *tbl = reinterpret_cast<const int *>(lds);
    R *planes = reinterpret_cast<R *>(lds + g.tbl_ints / 2);
    R *lsink = planes + 2 * plane;
    // the plane buffers are band-relative: clear them (positions outside this
    // band's projection must read as zero)
    __syncthreads();
    for (int t = tid; t < 2 * plane + 2; t += T) planes[t] = (R)0;
    __syncthreads();

    // own columns: x, table row, LDS offset, z range (empty range when unused)
    int cxr[K], clo[K], czr[K];
    bool cok[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int c = c0 + k * T + tid;
        cok[k] = c < c1;
        int x = g.pxlo, y = ya, z;
        unpack_xyz(g.cols[cok[k] ? c : c0], x, y, z);
        czr[k] = cok[k] ? g.colz[cok[k] ? c : c0] : 1023;
        cxr[k] = (x + 512) | ((y - g.pylo) << 16);
        clo[k] = (y - ya + 3) * W + (x - g.pxlo + 3);
    }
    const int nh0 = h1 - h0, nh = nh0 + (h3 - h2);
    int hxr[KH], hlo[KH], hzr[KH];
    bool hok[KH];
#pragma unroll
    for (int j = 0; j < KH; ++j) {
        const int t = j * T + tid;
        hok[j] = t < nh;
        const int c = hok[j] ? (t < nh0 ? h0 + t : h2 + (t - nh0)) : c0;
        int x, y, z;
        unpack_xyz(g.cols[c], x, y, z);
        hzr[j] = hok[j] ? g.colz[c] : 1023;
        hxr[j] = (x + 512) | ((y - g.pylo) << 16);
        hlo[j] = (y - ya + 3) * W + (x - g.pxlo + 3);
    }
    // packed index of a column at plane z, or -1 (branch-free)
    auto addr = [&](int z, int xr, int zr) __attribute__((always_inline)) -> int {
        const int zl = (zr & 0xffff) - 512, zh = (zr >> 16) - 512;
        const int zc = min(max(z, g.pzlo), g.pzlo + g.pnz - 1);
        const int idx = tbl[(zc - g.pzlo) * g.pny + (xr >> 16)] + (xr & 0xffff) - 512;
        return (unsigned)(z - zl) <= (unsigned)(zh - zl) ? idx : -1;
    };
    // slot arguments are std::integral_constant, so every index into the
    // policy's arrays is a constant and they stay in registers
    auto fetch_own = [&](auto sc, int zl) __attribute__((always_inline)) {
        constexpr int s = decltype(sc)::value;
        int ad[K];
#pragma unroll
        for (int k = 0; k < K; ++k) ad[k] = addr(zl, cxr[k], czr[k]);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if constexpr (wants_xyz<P>::value)
                pol.fetch_own_at(s, k, ad[k], (cxr[k] & 0xffff) - 512, g.pylo + (cxr[k] >> 16), zl);
            else
                pol.fetch_own(s, k, ad[k]);
        }
    };
    auto fetch_halo = [&](auto sc, int z) __attribute__((always_inline)) {
        constexpr int s = decltype(sc)::value;
        int ad[KH];
#pragma unroll
        for (int j = 0; j < KH; ++j) ad[j] = addr(z, hxr[j], hzr[j]);
#pragma unroll
        for (int j = 0; j < KH; ++j) {
            if constexpr (wants_xyz<P>::value)
                pol.fetch_halo_at(s, j, ad[j], (hxr[j] & 0xffff) - 512, g.pylo + (hxr[j] >> 16), z);
            else
                pol.fetch_halo(s, j, ad[j]);
        }
    };
    auto fetch_out = [&](auto sc, int z) __attribute__((always_inline)) {
        constexpr int s = decltype(sc)::value;
        int ad[K];
#pragma unroll
        for (int k = 0; k < K; ++k) ad[k] = addr(z, cxr[k], czr[k]);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if constexpr (wants_xyz<P>::value)
                pol.fetch_out_at(s, k, ad[k], (cxr[k] & 0xffff) - 512, g.pylo + (cxr[k] >> 16), z);
            else
                pol.fetch_out(s, k, ad[k]);
        }
    };

    R q[K][7];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int j = 0; j < 7; ++j) q[k][j] = (R)0;
    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, 1>;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        fetch_own(S0{}, zlo + j);
#pragma unroll
        for (int k = 0; k < K; ++k) q[k][4 + j] = pol.fin_own(0, k);
    }
    // in flight: own planes zlo+3 .. zlo+2+PF, halo and output planes zlo .. zlo+PF-1
    fetch_own(S0{}, zlo + 3);
    fetch_halo(S0{}, zlo);
    fetch_out(S0{}, zlo);
    if constexpr (PF == 2) {
        fetch_own(S1{}, zlo + 4);
        fetch_halo(S1{}, zlo + 1);
        fetch_out(S1{}, zlo + 1);
    }
    // one output plane zo, from slot s (a constant after unrolling)
    auto step = [&](auto slot, int zo) __attribute__((always_inline)) {
        constexpr int s = decltype(slot)::value;
        R un[K], uh[KH];
#pragma unroll
        for (int k = 0; k < K; ++k) un[k] = pol.fin_own(s, k);
#pragma unroll
        for (int j = 0; j < KH; ++j) uh[j] = pol.fin_halo(s, j);
        fetch_own(slot, zo + 3 + PF);
        fetch_halo(slot, zo + PF);
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
            for (int j = 0; j < 6; ++j) q[k][j] = q[k][j + 1];
            q[k][6] = un[k];
        }
        // the plane buffer alternates every step; the empty asm keeps the
        // compiler from precomputing each column's stencil addresses into
        // both buffers ahead of the loop (registers it does not have)
        int boff = (par & 1) * plane;
        asm volatile("" : "+v"(boff));
        R *buf = planes + boff;
        ++par;
#pragma unroll
        for (int k = 0; k < K; ++k) *(cok[k] ? buf + clo[k] : lsink) = q[k][3];
#pragma unroll
        for (int j = 0; j < KH; ++j) *(hok[j] ? buf + hlo[j] : lsink) = uh[j];
        lds_barrier();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const R *c = buf + clo[k];
            R sm = w.c * q[k][3];
            sm += w.z[1] * (q[k][2] + q[k][4]) + w.z[2] * (q[k][1] + q[k][5]) + w.z[3] * (q[k][0] + q[k][6]);
            sm += w.x[1] * (c[-1] + c[1]) + w.x[2] * (c[-2] + c[2]) + w.x[3] * (c[-3] + c[3]);
            sm += w.y[1] * (c[-W] + c[W]) + w.y[2] * (c[-2 * W] + c[2 * W]) + w.y[3] * (c[-3 * W] + c[3 * W]);
            pol.output(s, k, q[k][3], -sm);
        }
        fetch_out(slot, zo + PF);
    };
    if constexpr (PF == 1) {
        for (int zo = zlo; zo <= zhi; ++zo) step(S0{}, zo);
    } else {
        int zo = zlo;
        for (; zo + 1 <= zhi; zo += 2) {
            step(S0{}, zo);
            step(S1{}, zo + 1);
        }
        if (zo <= zhi) step(S0{}, zo);
    }
}

template <typename R, int T, int K, int KH, class P>
__device__ __forceinline__ void zmarch(const ClassDev &g, double *lds, int &par, P &pol, const StencilW<R> &w,
                                       const int4 &pg, int nx, int ny, int nz)
{
    const int nb = sizeof(R) == 4 ? g.n_bands32 : g.n_bands;
    for (int bi = 0; bi < nb; ++bi) zmarch_band<R, T, K, KH>(g, bi, lds, par, pol, w, pg, nx, ny, nz);
}

// direction pass: u = r + beta p_old, p_new <- u; sum p.Ap (and b.b when r is b)
template <typename R, int K, int KH, int S = 1>
struct PDir {
    static constexpr int kSlots = S;
    const R *rsrc, *pold;
    R *pnew, *sink;
    R beta;
    bool load_p, acc_bb;
    double pap = 0.0, bb = 0.0;
    R fr[S][K], fp[S][K];
    int fa[S][K];
    R hr[S][KH], hp[S][KH];
    int ha[S][KH];
    __device__ __forceinline__ void fetch_own(int s, int k, int a)
    {
        fa[s][k] = a;
        fr[s][k] = raw_load(rsrc, a);
        fp[s][k] = load_p ? raw_load(pold, a) : (R)0;
    }
    __device__ __forceinline__ R fin_own(int s, int k)
    {
        const bool ok = fa[s][k] >= 0;
        const R r = ok ? fr[s][k] : (R)0;
        const R u = ok ? fr[s][k] + beta * fp[s][k] : (R)0;
        *sel_ptr(pnew, fa[s][k], sink) = u;
        if (acc_bb) bb += (double)r * (double)r;
        return u;
    }
    __device__ __forceinline__ void fetch_halo(int s, int j, int a)
    {
        ha[s][j] = a;
        hr[s][j] = raw_load(rsrc, a);
        hp[s][j] = load_p ? raw_load(pold, a) : (R)0;
    }
    __device__ __forceinline__ R fin_halo(int s, int j) { return ha[s][j] >= 0 ? hr[s][j] + beta * hp[s][j] : (R)0; }
    __device__ __forceinline__ void fetch_out(int, int, int) {}
    __device__ __forceinline__ void output(int, int, R u, R Au) { pap += (double)u * (double)Au; }
};

// update pass: u = p, r = rsrc - alpha Ap (output time), sum r.r; and the
// iterate at load time, by mode XM:
//   XM_STEP  x += alpha p                      (every iteration)
//   XM_SKIP  x untouched: alpha p is owed      (first of two iterations)
//   XM_PAIR  x += alpha2 q + alpha p           (second: q = the previous p)
// Pairing the iterate updates reads and writes x every other iteration:
// 7.5 vector passes per CG iteration instead of 8.
enum { XM_STEP = 0, XM_SKIP = 1, XM_PAIR = 2 };
template <typename R, int K, int KH, int XM = XM_STEP, int S = 1>
struct PUpd {
    static constexpr int kSlots = S;
    const R *p, *rsrc;
    R *x, *r, *sink;
    R alpha;
    bool load_x;
    const R *q = nullptr;       // XM_PAIR: the previous direction
    R alpha2 = (R)0;
    double rr = 0.0;
    R fp[S][K], fx[S][K], fq[S][K];
    int fa[S][K];
    R hp[S][KH];
    int ha[S][KH];
    R orr[S][K];
    int oa[S][K];
    __device__ __forceinline__ void fetch_own(int s, int k, int a)
    {
        fa[s][k] = a;
        fp[s][k] = raw_load(p, a);
        if constexpr (XM != XM_SKIP) fx[s][k] = load_x ? raw_load(x, a) : (R)0;
        if constexpr (XM == XM_PAIR) fq[s][k] = raw_load(q, a);
    }
    __device__ __forceinline__ R fin_own(int s, int k)
    {
        const R pv = fa[s][k] >= 0 ? fp[s][k] : (R)0;
        if constexpr (XM == XM_STEP) *sel_ptr(x, fa[s][k], sink) = fx[s][k] + alpha * pv;
        if constexpr (XM == XM_PAIR) *sel_ptr(x, fa[s][k], sink) = fx[s][k] + alpha2 * fq[s][k] + alpha * pv;
        return pv;
    }
    __device__ __forceinline__ void fetch_halo(int s, int j, int a)
    {
        ha[s][j] = a;
        hp[s][j] = raw_load(p, a);
    }
    __device__ __forceinline__ R fin_halo(int s, int j) { return ha[s][j] >= 0 ? hp[s][j] : (R)0; }
    __device__ __forceinline__ void fetch_out(int s, int k, int a)
    {
        oa[s][k] = a;
        orr[s][k] = raw_load(rsrc, a);
    }
    __device__ __forceinline__ void output(int s, int k, R, R Au)
    {
        const R t = oa[s][k] >= 0 ? orr[s][k] - alpha * Au : (R)0;
        *sel_ptr(r, oa[s][k], sink) = t;
        rr += (double)t * (double)t;
    }
};

// FP64 residual pass: u = x (+ dscale d), r = b - A u; sums r.r and b.b
// (unscaled); the residual is stored times oscale in RT (double, or float
// for the FP32 iterations).  x is not written here (a later band's halo
// still needs the old x); the caller adds d to x afterwards.
template <int K, int KH, typename DT, typename RT, int S = 1>
struct PRes {
    static constexpr int kSlots = S;
    const double *x;
    const DT *d;
    const double *b;
    RT *r, *sink;
    bool add_d;
    double dscale;              // u = x + dscale * d
    double oscale = 1.0;        // stored residual = oscale (b - A u)
    double rr = 0.0, bb = 0.0;
    double fx[S][K];
    DT fd[S][K];
    int fa[S][K];
    double hx[S][KH];
    DT hd[S][KH];
    int ha[S][KH];
    double ob[S][K];
    int oa[S][K];
    __device__ __forceinline__ void fetch_own(int s, int k, int a)
    {
        fa[s][k] = a;
        fx[s][k] = raw_load(x, a);
        fd[s][k] = add_d ? raw_load(d, a) : (DT)0;
    }
    __device__ __forceinline__ double fin_own(int s, int k)
    {
        return fa[s][k] >= 0 ? fx[s][k] + dscale * (double)fd[s][k] : 0.0;
    }
    __device__ __forceinline__ void fetch_halo(int s, int j, int a)
    {
        ha[s][j] = a;
        hx[s][j] = raw_load(x, a);
        hd[s][j] = add_d ? raw_load(d, a) : (DT)0;
    }
    __device__ __forceinline__ double fin_halo(int s, int j)
    {
        return ha[s][j] >= 0 ? hx[s][j] + dscale * (double)hd[s][j] : 0.0;
    }
    __device__ __forceinline__ void fetch_out(int s, int k, int a)
    {
        oa[s][k] = a;
        ob[s][k] = raw_load(b, a);
    }
    __device__ __forceinline__ void output(int s, int k, double, double Au)
    {
        const bool ok = oa[s][k] >= 0;
        const double bv = ok ? ob[s][k] : 0.0;
        const double t = ok ? bv - Au : 0.0;
        *sel_ptr(r, oa[s][k], sink) = (RT)(t * oscale);
        rr += t * t;
        bb += bv * bv;
    }
};

// final pass: true residual b - A x
template <int K, int KH, int S = 1>
struct PFin {
    static constexpr int kSlots = S;
    const double *x, *b;
    double res = 0.0;
    double fx[S][K];
    int fa[S][K];
    double hx[S][KH];
    int ha[S][KH];
    double ob[S][K];
    int oa[S][K];
    __device__ __forceinline__ void fetch_own(int s, int k, int a)
    {
        fa[s][k] = a;
        fx[s][k] = raw_load(x, a);
    }
    __device__ __forceinline__ double fin_own(int s, int k) { return fa[s][k] >= 0 ? fx[s][k] : 0.0; }
    __device__ __forceinline__ void fetch_halo(int s, int j, int a)
    {
        ha[s][j] = a;
        hx[s][j] = raw_load(x, a);
    }
    __device__ __forceinline__ double fin_halo(int s, int j) { return ha[s][j] >= 0 ? hx[s][j] : 0.0; }
    __device__ __forceinline__ void fetch_out(int s, int k, int a)
    {
        oa[s][k] = a;
        ob[s][k] = raw_load(b, a);
    }
    __device__ __forceinline__ void output(int s, int k, double, double Au)
    {
        const double t = oa[s][k] >= 0 ? ob[s][k] - Au : 0.0;
        res += t * t;
    }
};


// ---------------------------------------------------------------------------
// multigrid preconditioner (symmetric V-cycle; not in the paper, which
// uses plain CG: the preconditioned iteration stops on the same residual)
// ---------------------------------------------------------------------------
//
// z = M r with M = S + (I - S A) P C R (I - A S): S = (omega / diag A) I is
// one damped Jacobi step of the fine operator A on the z-march, R averages a
// fine 2x2x2 block onto its level-1 cell, P injects a cell's value back
// (R = P^T / 8), and C is a V-cycle on masked dense boxes with the 7-point
// Laplacian at spacing 2^l h (Dirichlet zero outside the mask) and one damped
// Jacobi sweep before and after each coarsening, several on the coarsest
// box.  Every part is symmetric, so M is too and plain PCG applies.

// Storage of the FP64 preconditioned iteration: r and x in FP64; the dense
// residual, z and the directions p in FP32, scaled by a power of two sigma
// (the RMS of the residual rounded down to 2^k, so scaling is exact and the
// values stay inside the FP32 range as the residual falls).  p is rounded
// before the direction pass applies A, and the update pass recomputes Ap from
// the stored p, so x and r stay consistent in FP64; the rounding of z and p
// only perturbs M, like an inexact preconditioner.
// The FP32 form (FP32_REFINE) keeps r in FP32 too, scaled, and computes the
// fine passes and the V-cycle in FP32; x stays FP64 and the residual is
// replaced by the true FP64 b - A x whenever the recursive one has fallen by
// a fixed factor, so rounding never accumulates into the result.
__device__ __forceinline__ double pow2_scale(double rr, double n)
{
    int e;
    (void)frexp(sqrt(rr / n), &e);
    return ldexp(1.0, e - 1);
}

// fine passes on the z-march (each takes each point's offsets), in the
// arithmetic R of the iteration (double, or float for the FP32 form):
//   MG_PRE:  t = r - c A r on PE, stored / sigma in the dense, even-padded
//            PE box (the residual left by the smoothing step S r)
//   MG_POST: u = c r + e_1(cell of the point) (S r plus the prolonged coarse
//            correction), z = u + c (r - A u) on PE stored / sigma,
//            rho += r . z (of the stored z).  r at the output plane is not
//            read again: in FP64 it is recovered as (u - e_1) / c from the
//            cell's correction (cached), in FP32 kept in a four-plane
//            register queue (the recovery would cancel digits FP32 lacks).
enum { MG_PRE = 0, MG_POST = 1 };
template <typename R, int K, int KH, int MODE, int S = 1>
struct PMg {
    static constexpr int kSlots = S;
    static constexpr bool kXYZ = true;
    static constexpr bool kQueue = sizeof(R) == 4 && MODE == MG_POST;
    const R *r;                         // the vector M is applied to
    const R *e1;                        // level-1 correction (MG_POST)
    float *out, *sink;                  // MG_PRE: dense box; MG_POST: z (packed)
    double c, sigma, inv_sigma;
    int pxlo, pylo, pzlo;
    int dnx, dnxy;                      // dense box pitches (MG_PRE)
    int nx1, nxy1;                      // level-1 pitches (MG_POST)
    double rho = 0.0;
    R fr[S][K], fe[S][K];
    int fa[S][K];
    R hr[S][KH], he[S][KH];
    int ha[S][KH];
    R oe[S][K];                         // MG_POST, FP64: e_1 at the output point
    int oa[S][K];
    R rq[K][4];                         // MG_POST, FP32: r at the planes zo .. zo+3
    __device__ __forceinline__ int cell(int a, int x, int y, int z) const
    {
        return a >= 0 ? ((z - pzlo) >> 1) * nxy1 + ((y - pylo) >> 1) * nx1 + ((x - pxlo) >> 1) : 0;
    }
    __device__ __forceinline__ void fetch_own_at(int s, int k, int a, int x, int y, int z)
    {
        fa[s][k] = a;
        fr[s][k] = raw_load(r, a);
        if constexpr (MODE == MG_POST) fe[s][k] = e1[cell(a, x, y, z)];
    }
    __device__ __forceinline__ R fin_own(int s, int k)
    {
        const bool ok = fa[s][k] >= 0;
        if constexpr (kQueue) {
#pragma unroll
            for (int j = 0; j < 3; ++j) rq[k][j] = rq[k][j + 1];
            rq[k][3] = ok ? fr[s][k] : (R)0;
        }
        if constexpr (MODE == MG_POST) return ok ? (R)c * fr[s][k] + fe[s][k] : (R)0;
        return ok ? fr[s][k] : (R)0;
    }
    __device__ __forceinline__ void fetch_halo_at(int s, int j, int a, int x, int y, int z)
    {
        ha[s][j] = a;
        hr[s][j] = raw_load(r, a);
        if constexpr (MODE == MG_POST) he[s][j] = e1[cell(a, x, y, z)];
    }
    __device__ __forceinline__ R fin_halo(int s, int j)
    {
        if constexpr (MODE == MG_POST) return ha[s][j] >= 0 ? (R)c * hr[s][j] + he[s][j] : (R)0;
        return ha[s][j] >= 0 ? hr[s][j] : (R)0;
    }
    __device__ __forceinline__ void fetch_out_at(int s, int k, int a, int x, int y, int z)
    {
        if constexpr (MODE == MG_POST) {
            oa[s][k] = a;
            if constexpr (!kQueue) oe[s][k] = e1[cell(a, x, y, z)];
        } else {
            oa[s][k] = a >= 0 ? ((z - pzlo) * dnxy + (y - pylo) * dnx + (x - pxlo)) : -1;
        }
    }
    __device__ __forceinline__ void output(int s, int k, R uu, R Au)
    {
        if constexpr (MODE == MG_PRE) {
            *sel_ptr(out, oa[s][k], sink) = (float)(((double)uu - c * (double)Au) * inv_sigma);
        } else {
            const bool ok = oa[s][k] >= 0;
            double rv;
            if constexpr (kQueue)
                rv = (double)rq[k][0];
            else
                rv = ((double)uu - (double)oe[s][k]) / c;
            const float zs = (float)(((double)uu + c * (rv - (double)Au)) * inv_sigma);
            rho += ok ? rv * ((double)zs * sigma) : 0.0;
            *sel_ptr(out, oa[s][k], sink) = zs;
        }
    }
};

// direction pass of the preconditioned iteration: u = z + beta p_old
// (z at scale sz, p_old at scale sp), rounded to the stored p_new (scale sz)
// before A is applied; sums p.Ap
template <typename R, int K, int KH, int S = 1>
struct PMgDir {
    static constexpr int kSlots = S;
    const float *z, *pold;
    float *pnew, *sink;
    double beta, sz, sp, inv_sz;
    bool load_p;
    double pap = 0.0;
    float fz[S][K], fp[S][K];
    int fa[S][K];
    float hz[S][KH], hp[S][KH];
    int ha[S][KH];
    __device__ __forceinline__ float round_p(float zz, float pp) const
    {
        return (float)(((double)zz * sz + beta * ((double)pp * sp)) * inv_sz);
    }
    __device__ __forceinline__ void fetch_own(int s, int k, int a)
    {
        fa[s][k] = a;
        fz[s][k] = raw_load(z, a);
        fp[s][k] = load_p ? raw_load(pold, a) : 0.f;
    }
    __device__ __forceinline__ R fin_own(int s, int k)
    {
        const bool ok = fa[s][k] >= 0;
        const float ps = ok ? round_p(fz[s][k], fp[s][k]) : 0.f;
        *sel_ptr(pnew, fa[s][k], sink) = ps;
        return (R)((double)ps * sz);
    }
    __device__ __forceinline__ void fetch_halo(int s, int j, int a)
    {
        ha[s][j] = a;
        hz[s][j] = raw_load(z, a);
        hp[s][j] = load_p ? raw_load(pold, a) : 0.f;
    }
    __device__ __forceinline__ R fin_halo(int s, int j)
    {
        return ha[s][j] >= 0 ? (R)((double)round_p(hz[s][j], hp[s][j]) * sz) : (R)0;
    }
    __device__ __forceinline__ void fetch_out(int, int, int) {}
    __device__ __forceinline__ void output(int, int, R u, R Au) { pap += (double)u * (double)Au; }
};

// update pass of the preconditioned iteration: p = sz * stored p;
// r = rsrc - alpha A p at output time (r in R), sums r.r; the iterate
// (FP64) at load time by mode XM as in the plain iteration, each increment
// times xscale (XM_PAIR adds alpha2 sq q + alpha p, q the previous direction
// at its scale sq)
template <typename R, int K, int KH, int XM, int S = 1>
struct PMgUpd {
    static constexpr int kSlots = S;
    const float *p;
    const R *rsrc;
    double *x;
    R *r, *sink;
    double *xsink;              // where invalid lanes store their x
    double alpha, sz;
    bool load_x;
    const float *q = nullptr;
    double alpha2 = 0.0, sq = 0.0;
    double xscale = 1.0;
    double rr = 0.0;
    float fp[S][K], fq[S][K];
    double fx[S][K];
    int fa[S][K];
    float hp[S][KH];
    int ha[S][KH];
    R orr[S][K];
    int oa[S][K];
    __device__ __forceinline__ void fetch_own(int s, int k, int a)
    {
        fa[s][k] = a;
        fp[s][k] = raw_load(p, a);
        if constexpr (XM != XM_SKIP) fx[s][k] = load_x ? raw_load(x, a) : 0.0;
        if constexpr (XM == XM_PAIR) fq[s][k] = raw_load(q, a);
    }
    __device__ __forceinline__ R fin_own(int s, int k)
    {
        const double pv = fa[s][k] >= 0 ? (double)fp[s][k] * sz : 0.0;
        double *xs = sel_ptr(x, fa[s][k], xsink);
        if constexpr (XM == XM_STEP) *xs = fx[s][k] + xscale * (alpha * pv);
        if constexpr (XM == XM_PAIR) *xs = fx[s][k] + xscale * (alpha2 * ((double)fq[s][k] * sq) + alpha * pv);
        return (R)pv;
    }
    __device__ __forceinline__ void fetch_halo(int s, int j, int a)
    {
        ha[s][j] = a;
        hp[s][j] = raw_load(p, a);
    }
    __device__ __forceinline__ R fin_halo(int s, int j) { return ha[s][j] >= 0 ? (R)((double)hp[s][j] * sz) : (R)0; }
    __device__ __forceinline__ void fetch_out(int s, int k, int a)
    {
        oa[s][k] = a;
        orr[s][k] = raw_load(rsrc, a);
    }
    __device__ __forceinline__ void output(int s, int k, R, R Au)
    {
        const R t = oa[s][k] >= 0 ? (R)((double)orr[s][k] - alpha * (double)Au) : (R)0;
        *sel_ptr(r, oa[s][k], sink) = t;
        rr += (double)t * (double)t;
    }
};

// Cells c = threadIdx.x + k T of a level in order, with their (x, y, z)
// stepped without divisions.
struct CellWalk {
    int c, x, y, z, sx, sy, sz, nx, ny;
    __device__ __forceinline__ CellWalk(const MgLevel &L, int T)
    {
        c = threadIdx.x;
        x = c % L.nx;
        y = (c / L.nx) % L.ny;
        z = c / (L.nx * L.ny);
        sx = T % L.nx;
        sy = (T / L.nx) % L.ny;
        sz = T / (L.nx * L.ny);
        nx = L.nx;
        ny = L.ny;
    }
    __device__ __forceinline__ void next(int T)
    {
        c += T;
        x += sx;
        if (x >= nx) { x -= nx; ++y; }
        y += sy;
        if (y >= ny) { y -= ny; ++z; }
        z += sz;
    }
};

// Branch-free loop over the cells of a level: each thread takes U cells
// (stride T) at a time, evaluates body(c, x, y, z) for all U (loads of the U
// cells in flight together), then stores the U results to out[c].  Cells
// past the end evaluate cell 0 and store nothing.
template <int T, int U, typename CT, class F>
__device__ __forceinline__ void mg_cells(const MgLevel &L, CT *out, F body)
{
    const int n = L.nx * L.ny * L.nz;
    CellWalk w(L, T);
    while (w.c < n) {
        int cc[U];
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = w.c < n;
            cc[u] = ok ? w.c : -1;
            v[u] = body(ok ? w.c : 0, ok ? w.x : 0, ok ? w.y : 0, ok ? w.z : 0);
            w.next(T);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (cc[u] >= 0) out[cc[u]] = (CT)v[u];
    }
}

// sum over the six neighbours of cell (x, y, z) of s_a v(neighbour), zero
// outside the box (branch-free: a missing neighbour reads the cell itself)
template <typename CT>
__device__ __forceinline__ double mg_nbsum(const MgLevel &L, const CT *v, int c, int x, int y, int z,
                                           const double (&s)[3])
{
    const int sxy = L.nx * L.ny;
    const bool xm = x > 0, xp = x + 1 < L.nx, ym = y > 0, yp = y + 1 < L.ny, zm = z > 0, zp = z + 1 < L.nz;
    const double a0 = (double)v[xm ? c - 1 : c], a1 = (double)v[xp ? c + 1 : c];
    const double b0 = (double)v[ym ? c - L.nx : c], b1 = (double)v[yp ? c + L.nx : c];
    const double d0 = (double)v[zm ? c - sxy : c], d1 = (double)v[zp ? c + sxy : c];
    return s[0] * ((xm ? a0 : 0.0) + (xp ? a1 : 0.0)) + s[1] * ((ym ? b0 : 0.0) + (yp ? b1 : 0.0)) +
           s[2] * ((zm ? d0 : 0.0) + (zp ? d1 : 0.0));
}

__device__ __forceinline__ void mg_spacing(const SolveArgs &a, int l, double (&s)[3])
{
    const double f = (double)(2 << l);      // level l + 1 has spacing 2^(l+1) h
#pragma unroll
    for (int d = 0; d < 3; ++d) s[d] = 1.0 / ((f * a.h[d]) * (f * a.h[d]));
}

constexpr int MG_U = 4;     // cells per thread in flight

// level-1 right-hand side: the average of each cell's fine residuals, read
// from the dense PE box (stored / sigma in FP32; children outside PE hold
// stale values and cm masks them; cells outside the domain read the box's
// first line and yield zero)
template <int T, typename CT>
__device__ void mg_restrict_dense(const MgLevel &L, const float *__restrict__ t, double sigma, CT *__restrict__ f)
{
    const int dnx = 2 * L.nx, dnxy = 4 * L.nx * L.ny;
    const double w = 0.125 * sigma;
    mg_cells<T, MG_U, CT>(L, f, [&](int c, int x, int y, int z) -> double {
        const int m = L.cm[c];
        const float *p = t + (m ? (long long)(2 * z) * dnxy + (2 * y) * dnx + 2 * x : 0);
        const float2 v0 = *reinterpret_cast<const float2 *>(p);
        const float2 v1 = *reinterpret_cast<const float2 *>(p + dnx);
        const float2 v2 = *reinterpret_cast<const float2 *>(p + dnxy);
        const float2 v3 = *reinterpret_cast<const float2 *>(p + dnxy + dnx);
        const double sum = ((m & 1) ? (double)v0.x : 0.0) + ((m & 2) ? (double)v0.y : 0.0) +
                           ((m & 4) ? (double)v1.x : 0.0) + ((m & 8) ? (double)v1.y : 0.0) +
                           ((m & 16) ? (double)v2.x : 0.0) + ((m & 32) ? (double)v2.y : 0.0) +
                           ((m & 64) ? (double)v3.x : 0.0) + ((m & 128) ? (double)v3.y : 0.0);
        return w * sum;
    });
    __syncthreads();
}

// V-cycle on the coarse levels: e_1 ~ C f_1, the right-hand side f of each
// level zero outside its domain.  Per level: f at off, e at off + n, t at
// off + 2n; the result e_1 is returned.
template <int T, typename CT>
__device__ const CT *mg_vcycle(const SolveArgs &a, const MgClass &M, CT *ms)
{
    const int nl = M.levels;
    const double wc = a.mg_omega_c;
    // down: the residual after one damped Jacobi step from zero,
    // f(c) - L(wc D^-1 f)(c) = (1 - wc) f(c) + wc d sum_a s_a (f(c - e_a) + f(c + e_a)),
    // averaged over the children in the domain of each coarser cell
    for (int l = 0; l + 1 < nl; ++l) {
        const MgLevel L = M.lv[l], Lc = M.lv[l + 1];
        const CT *f = ms + L.off;
        double s[3];
        mg_spacing(a, l, s);
        const double wd = wc / (2.0 * (s[0] + s[1] + s[2]));
        mg_cells<T, 1, CT>(Lc, ms + Lc.off, [&](int C, int X, int Y, int Z) -> double {
            const int m = Lc.cm[C];
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const bool in = (m >> k) & 1;
                const int x = in ? 2 * X + (k & 1) : 0, y = in ? 2 * Y + ((k >> 1) & 1) : 0,
                          z = in ? 2 * Z + (k >> 2) : 0;
                const int c = (z * L.ny + y) * L.nx + x;
                const double t = (1.0 - wc) * (double)f[c] + wd * mg_nbsum(L, f, c, x, y, z, s);
                sum += in ? t : 0.0;
            }
            return 0.125 * sum;
        });
        __syncthreads();
    }
    // coarsest: damped Jacobi sweeps from zero, e and t in turn
    const CT *ec;
    {
        const MgLevel L = M.lv[nl - 1];
        const int n = L.nx * L.ny * L.nz;
        const CT *f = ms + L.off;
        CT *e = ms + L.off + n, *t = e + n;
        double s[3];
        mg_spacing(a, nl - 1, s);
        const double wd = wc / (2.0 * (s[0] + s[1] + s[2]));
        for (int c = threadIdx.x; c < n; c += T) e[c] = (CT)(wd * (double)f[c]);
        __syncthreads();
        for (int sw = 1; sw < a.mg_coarse_sweeps; ++sw) {
            const CT *eo = e;
            mg_cells<T, 1, CT>(L, t, [&](int c, int x, int y, int z) -> double {
                const double v = (1.0 - wc) * (double)eo[c] + wd * ((double)f[c] + mg_nbsum(L, eo, c, x, y, z, s));
                return L.cm[c] ? v : 0.0;
            });
            __syncthreads();
            CT *u = e; e = t; t = u;
        }
        ec = e;
    }
    // up: u(c) = wc d f(c) + e_coarse(parent of c) on the domain, then one
    // damped Jacobi sweep, e(c) = (1 - wc) u(c) + wc d (f(c) + sum_a s_a u(neighbours));
    // on level 1, times the coarse-correction scale
    for (int l = nl - 2; l >= 0; --l) {
        const MgLevel L = M.lv[l], Lc = M.lv[l + 1];
        const int n = L.nx * L.ny * L.nz;
        const CT *f = ms + L.off;
        CT *e = ms + L.off + n, *u = e + n;
        double s[3];
        mg_spacing(a, l, s);
        const double wd = wc / (2.0 * (s[0] + s[1] + s[2]));
        const CT *ecl = ec;
        mg_cells<T, MG_U, CT>(L, u, [&](int c, int x, int y, int z) -> double {
            const double v = wd * (double)f[c] + (double)ecl[((z >> 1) * Lc.ny + (y >> 1)) * Lc.nx + (x >> 1)];
            return L.cm[c] ? v : 0.0;
        });
        __syncthreads();
        // the correction handed to the fine level (l = 0) is scaled by
        // mg_coarse_scale, folded into the sweep's two coefficients
        const double gsc = l == 0 ? a.mg_coarse_scale : 1.0;
        const double a1 = gsc * (1.0 - wc), a2 = gsc * wd;
        mg_cells<T, MG_U, CT>(L, e, [&](int c, int x, int y, int z) -> double {
            const double v = a1 * (double)u[c] + a2 * ((double)f[c] + mg_nbsum(L, u, c, x, y, z, s));
            return L.cm[c] ? v : 0.0;
        });
        __syncthreads();
        ec = e;
    }
    return ec;
}

// Kernel modes: FP64 CG from zero, FP64 CG from the guess in vout (one more
// pass type, so more registers), FP32 CG with FP64 reliable updates (guess
// read at run time), FP64 CG preconditioned by the multigrid V-cycle (guess
// read at run time), and the multigrid-preconditioned iteration in FP32 with
// FP64 residual replacement (guess read at run time).
enum { CG_FP64 = 0, CG_FP64_GUESS = 1, CG_MIXED = 2, CG_MG = 3, CG_MG_MIXED = 4 };

// Residual replacement of the FP32 multigrid iteration: the true FP64
// residual replaces the recursive one once the recursive norm has fallen by
// this factor since the last replacement (or claims convergence).
constexpr double kMgMixedDrop = 1e-3;

// One pair: FP64 CG, FP32 CG with FP64 iterative refinement, or the
// multigrid-preconditioned iteration in FP64 or FP32.  PF64 / PF32: planes of
// loads in flight in the FP64 / FP32 passes.
template <int T, int K, int KH, int K32, int KH32, int MODE, int PF64, int PF32>
__device__ __forceinline__ void cg_zmarch_pair(const SolveArgs &a, int pair, long long slot, double *lds, double *red,
                                               int &par)
{
    constexpr bool MIXED = MODE == CG_MIXED;
    const int tid = threadIdx.x;
    const int4 pg = a.pair_gc[pair];
    const ClassDev g = a.cls[pg.w];
    double *x = a.vout + a.out_off[pair];
    const double *b = a.rhs + a.rhs_off[pair];
    const StencilW<double> w64 = stencil_w<double>(a);
    const bool guess = (MIXED || MODE == CG_MG || MODE == CG_MG_MIXED) ? a.guess != 0 : MODE == CG_FP64_GUESS;
    int it = 0, conv = 0, outer = 0;
    double bb = 0.0;

    if constexpr (MODE == CG_MG) {
        // PCG with the multigrid V-cycle as M: per slot r (FP64), then z and
        // two direction buffers (FP32, scaled); x from zero or the guess
        double *r = a.scratch + slot * 4 * a.slot_n;
        double *rsink = r + a.slot_n - 1;
        float *zv = reinterpret_cast<float *>(r + a.slot_n);
        float *pold = zv + a.slot_n, *pnew = pold + a.slot_n;
        double *ms = a.mg_scratch + slot * a.mg_slot_n;
        const MgClass &M = a.mgc[pg.w];
        const MgLevel L1 = M.lv[0];
        float *dense = reinterpret_cast<float *>(ms + M.dense_off);
        float *dsink = dense + 8LL * L1.nx * L1.ny * L1.nz;
        const double cfine = a.mg_omega / (-w64.c);
        const double n_el = (double)g.n_pe;
        const double *rsrc = b;
        double rr = 0.0;
        if (guess) {
            PRes<K, KH, double, double, PF64> pr{x, x, b, r, rsink, false, 0.0};
            zmarch<double, T, K, KH>(g, lds, par, pr, w64, pg, a.nx, a.ny, a.nz);
            ++outer;
            rr = block_sum<T>(pr.rr, red);
            bb = block_sum<T>(pr.bb, red);
            rsrc = r;
        } else {
            double s2 = 0.0;
            for (int q = tid; q < g.n_pe; q += T) s2 += b[q] * b[q];
            bb = rr = block_sum<T>(s2, red);
        }
        // z = M rs at scale sz (stored / sz); returns rs . z
        auto precond = [&](const double *rs, double sz) -> double {
            PMg<double, K, KH, MG_PRE, PF64> pre{rs, nullptr, dense, dsink, cfine, sz, 1.0 / sz, g.pxlo, g.pylo,
                                               g.pzlo, 2 * L1.nx, 4 * L1.nx * L1.ny, L1.nx, L1.nx * L1.ny};
            zmarch<double, T, K, KH>(g, lds, par, pre, w64, pg, a.nx, a.ny, a.nz);
            __syncthreads();                        // the dense residual of every band is written
            mg_restrict_dense<T, double>(L1, dense, sz, ms + L1.off);
            const double *e1 = mg_vcycle<T, double>(a, M, ms);
            PMg<double, K, KH, MG_POST, PF64> post{rs, e1, zv, zv + a.slot_n - 1, cfine, sz, 1.0 / sz, g.pxlo,
                                                 g.pylo, g.pzlo, 2 * L1.nx, 4 * L1.nx * L1.ny, L1.nx,
                                                 L1.nx * L1.ny};
            zmarch<double, T, K, KH>(g, lds, par, post, w64, pg, a.nx, a.ny, a.nz);
            return block_sum<T>(post.rho, red);
        };
        const double stop = a.tol * a.tol * bb;
        if (bb == 0.0) {
            for (int q = tid; q < g.n_pe; q += T) x[q] = 0.0;
            __syncthreads();
            conv = 1;
        } else if (rr <= stop) {
            conv = 1;
        } else {
            double sz = pow2_scale(rr, n_el);
            double rho = precond(rsrc, sz);
            double pap;
            {
                PMgDir<double, K, KH, PF64> pd{zv, pold, pnew, pnew + a.slot_n - 1, 0.0, sz, sz, 1.0 / sz, false};
                zmarch<double, T, K, KH>(g, lds, par, pd, w64, pg, a.nx, a.ny, a.nz);
                pap = block_sum<T>(pd.pap, red);
            }
            double sp = sz;                         // scale of the stored direction
            // x is updated every other iteration; `owed` alpha p (p in pnew at
            // scale s_owed) is not yet in x
            double owed = 0.0, s_owed = 0.0;
            bool pending = false;
            for (;;) {
                const double alpha = rho / pap;
                if (!pending) {
                    PMgUpd<double, K, KH, XM_SKIP, PF64> pu{pnew, rsrc, x, r, rsink, rsink, alpha, sp, false};
                    zmarch<double, T, K, KH>(g, lds, par, pu, w64, pg, a.nx, a.ny, a.nz);
                    rr = block_sum<T>(pu.rr, red);
                    owed = alpha;
                    s_owed = sp;
                    pending = true;
                } else {
                    PMgUpd<double, K, KH, XM_PAIR, PF64> pu{pnew, rsrc, x, r, rsink, rsink, alpha, sp, guess || it > 1,
                                                          pold, owed, s_owed};
                    zmarch<double, T, K, KH>(g, lds, par, pu, w64, pg, a.nx, a.ny, a.nz);
                    rr = block_sum<T>(pu.rr, red);
                    pending = false;
                }
                ++it;
                rsrc = r;
                if (rr <= stop) { conv = 1; break; }
                if (it >= a.maxit) break;
                sz = pow2_scale(rr, n_el);
                const double rho_new = precond(r, sz);
                const double beta = rho_new / rho;
                rho = rho_new;
                float *t = pold; pold = pnew; pnew = t;
                PMgDir<double, K, KH, PF64> pd{zv, pold, pnew, pnew + a.slot_n - 1, beta, sz, sp, 1.0 / sz, true};
                zmarch<double, T, K, KH>(g, lds, par, pd, w64, pg, a.nx, a.ny, a.nz);
                pap = block_sum<T>(pd.pap, red);
                sp = sz;
            }
            if (pending) {
                // the last iteration's step (its p is still in pnew); x holds a
                // value once a paired update has run or a guess was given
                const bool xv = guess || it > 2;
                const double w = owed * s_owed;
                for (int q = tid; q < g.n_pe; q += T) x[q] = (xv ? x[q] : 0.0) + w * (double)pnew[q];
                __syncthreads();
            }
        }
    } else if constexpr (MODE == CG_MG_MIXED) {
        // The multigrid-preconditioned iteration in FP32: r, z and the
        // directions in FP32 (r as r / sig, sig a power of two reset at each
        // replacement; z and p at their own power-of-two scales), every fine
        // pass and the V-cycle in FP32, x in FP64 (increments times sig).  The
        // true residual b - A x, in FP64, replaces r whenever the recursive
        // norm has fallen by kMgMixedDrop since the last replacement or
        // claims convergence; the iteration then goes on from the replaced
        // residual with its direction kept (rescaled to the new sig).
        float *r32 = a.scratch32 + slot * 4 * a.slot_n;
        float *rsink = r32 + a.slot_n - 1;
        float *zv = r32 + a.slot_n, *pold = zv + a.slot_n, *pnew = pold + a.slot_n;
        double *msd = a.mg_scratch + slot * a.mg_slot_n;
        float *ms = reinterpret_cast<float *>(msd);   // coarse levels in FP32, in the FP64 region's first half
        const MgClass &M = a.mgc[pg.w];
        const MgLevel L1 = M.lv[0];
        float *dense = reinterpret_cast<float *>(msd + M.dense_off);
        float *dsink = dense + 8LL * L1.nx * L1.ny * L1.nz;
        double *xsink = reinterpret_cast<double *>(dsink);   // 8-byte aligned spare after the dense box
        const StencilW<float> w32 = stencil_w<float>(a);
        const double cfine = a.mg_omega / (-w64.c);
        const double n_el = (double)g.n_pe;
        {
            double s2 = 0.0;
            for (int q = tid; q < g.n_pe; q += T) s2 += b[q] * b[q];
            bb = block_sum<T>(s2, red);
        }
        const double stop = a.tol * a.tol * bb;
        if (bb == 0.0) {
            for (int q = tid; q < g.n_pe; q += T) x[q] = 0.0;
            __syncthreads();
            conv = 1;
        } else {
            double sig = pow2_scale(bb, n_el);
            double rr;                              // r.r of the current residual, unscaled
            if (guess) {
                PRes<K, KH, double, float, PF64> pr{x, x, b, r32, rsink, false, 0.0, 1.0 / sig};
                zmarch<double, T, K, KH>(g, lds, par, pr, w64, pg, a.nx, a.ny, a.nz);
                ++outer;
                rr = block_sum<T>(pr.rr, red);
            } else {
                const double inv = 1.0 / sig;
                for (int q = tid; q < g.n_pe; q += T) {
                    x[q] = 0.0;
                    r32[q] = (float)(b[q] * inv);
                }
                __syncthreads();
                rr = bb;
            }
            if (rr <= stop) {
                conv = 1;
            } else {
                // z = M rs at scale sz (stored / sz); returns rs . z
                auto precond = [&](double sz) -> double {
                    PMg<float, K32, KH32, MG_PRE, PF32> pre{r32, nullptr, dense, dsink, cfine, sz, 1.0 / sz,
                                                            g.pxlo, g.pylo, g.pzlo, 2 * L1.nx, 4 * L1.nx * L1.ny,
                                                            L1.nx, L1.nx * L1.ny};
                    zmarch<float, T, K32, KH32>(g, lds, par, pre, w32, pg, a.nx, a.ny, a.nz);
                    __syncthreads();
                    mg_restrict_dense<T, float>(L1, dense, sz, ms + L1.off);
                    const float *e1 = mg_vcycle<T, float>(a, M, ms);
                    PMg<float, K32, KH32, MG_POST, PF32> post{r32, e1, zv, zv + a.slot_n - 1, cfine, sz, 1.0 / sz,
                                                              g.pxlo, g.pylo, g.pzlo, 2 * L1.nx,
                                                              4 * L1.nx * L1.ny, L1.nx, L1.nx * L1.ny};
                    zmarch<float, T, K32, KH32>(g, lds, par, post, w32, pg, a.nx, a.ny, a.nz);
                    return block_sum<T>(post.rho, red);
                };
                double rr_s = rr / (sig * sig);     // r.r in the units of r32
                double rr_rep = rr;                 // unscaled r.r at the last replacement
                double sz = pow2_scale(rr_s, n_el);
                double rho = precond(sz);
                double pap;
                {
                    PMgDir<float, K32, KH32, PF32> pd{zv, pold, pnew, pnew + a.slot_n - 1, 0.0, sz, sz, 1.0 / sz,
                                                      false};
                    zmarch<float, T, K32, KH32>(g, lds, par, pd, w32, pg, a.nx, a.ny, a.nz);
                    pap = block_sum<T>(pd.pap, red);
                }
                double sp = sz;
                double owed = 0.0, s_owed = 0.0;
                bool pending = false;
                // the owed step alpha p (p in pnew at scale s_owed), into x
                auto flush = [&]() {
                    const double w = sig * owed * s_owed;
                    for (int q = tid; q < g.n_pe; q += T) x[q] += w * (double)pnew[q];
                    __syncthreads();
                    pending = false;
                };
                for (;;) {
                    const double alpha = rho / pap;
                    if (!pending) {
                        PMgUpd<float, K32, KH32, XM_SKIP, PF32> pu{pnew, r32, x, r32, rsink, xsink, alpha, sp, true};
                        zmarch<float, T, K32, KH32>(g, lds, par, pu, w32, pg, a.nx, a.ny, a.nz);
                        rr_s = block_sum<T>(pu.rr, red);
                        owed = alpha;
                        s_owed = sp;
                        pending = true;
                    } else {
                        PMgUpd<float, K32, KH32, XM_PAIR, PF32> pu{pnew, r32, x, r32, rsink, xsink, alpha, sp, true,
                                                                   pold, owed, s_owed, sig};
                        zmarch<float, T, K32, KH32>(g, lds, par, pu, w32, pg, a.nx, a.ny, a.nz);
                        rr_s = block_sum<T>(pu.rr, red);
                        pending = false;
                    }
                    ++it;
                    const double rr_est = rr_s * sig * sig;
                    if (rr_est <= stop || rr_est <= kMgMixedDrop * kMgMixedDrop * rr_rep || it >= a.maxit ||
                        !(rr_s == rr_s)) {
                        if (pending) flush();
                        const double sig_new = rr_est > 0.0 && rr_est == rr_est ? pow2_scale(rr_est, n_el) : sig;
                        PRes<K, KH, double, float, PF64> pr{x, x, b, r32, rsink, false, 0.0, 1.0 / sig_new};
                        zmarch<double, T, K, KH>(g, lds, par, pr, w64, pg, a.nx, a.ny, a.nz);
                        ++outer;
                        const double rr_true = block_sum<T>(pr.rr, red);
                        if (rr_true <= stop) { conv = 1; break; }
                        if (it >= a.maxit) break;
                        // carry the iteration into the new units of r32
                        const double f = sig / sig_new;
                        sp *= f;
                        rho *= f * f;
                        sig = sig_new;
                        rr_rep = rr_true;
                        rr_s = rr_true / (sig * sig);
                    }
                    sz = pow2_scale(rr_s, n_el);
                    const double rho_new = precond(sz);
                    const double beta = rho_new / rho;
                    rho = rho_new;
                    float *t = pold; pold = pnew; pnew = t;
                    PMgDir<float, K32, KH32, PF32> pd{zv, pold, pnew, pnew + a.slot_n - 1, beta, sz, sp, 1.0 / sz,
                                                      true};
                    zmarch<float, T, K32, KH32>(g, lds, par, pd, w32, pg, a.nx, a.ny, a.nz);
                    pap = block_sum<T>(pd.pap, red);
                    sp = sz;
                }
                if (pending) flush();
            }
        }
    } else if constexpr (!MIXED) {

        double *r = a.scratch + slot * 3 * a.slot_n;
        double *pold = r + a.slot_n, *pnew = pold + a.slot_n;
        const double *rsrc = b;
        double rr = 0.0, pap = 0.0;
        if constexpr (MODE == CG_FP64_GUESS) {
            PRes<K, KH, double, double, PF64> pr{x, x, b, r, r + a.slot_n - 1, false, 0.0};
            zmarch<double, T, K, KH>(g, lds, par, pr, w64, pg, a.nx, a.ny, a.nz);
            ++outer;
            rr = block_sum<T>(pr.rr, red);
            bb = block_sum<T>(pr.bb, red);
            rsrc = r;
        }
        {
            PDir<double, K, KH, PF64> pd{rsrc, pold, pnew, pnew + a.slot_n - 1, 0.0, false, !guess};
            zmarch<double, T, K, KH>(g, lds, par, pd, w64, pg, a.nx, a.ny, a.nz);
            pap = block_sum<T>(pd.pap, red);
            if (!guess) rr = bb = block_sum<T>(pd.bb, red);
        }
        const double stop = a.tol * a.tol * bb;
        if (bb == 0.0) {
            for (int q = tid; q < g.n_pe; q += T) x[q] = 0.0;
            conv = 1;
        } else if (rr <= stop) {
            conv = 1;
        } else {
            // x is updated every other iteration (PUpd XM_SKIP / XM_PAIR);
            // `owed` is the step alpha p not yet in x, with p in pnew
            double owed = 0.0;
            bool pending = false;
            for (;;) {
                const double alpha = rr / pap;
                double rn;
                if (!pending) {
                    PUpd<double, K, KH, XM_SKIP, PF64> pu{pnew, rsrc, x, r, r + a.slot_n - 1, alpha, false};
                    zmarch<double, T, K, KH>(g, lds, par, pu, w64, pg, a.nx, a.ny, a.nz);
                    rn = block_sum<T>(pu.rr, red);
                    owed = alpha;
                    pending = true;
                } else {
                    PUpd<double, K, KH, XM_PAIR, PF64> pu{pnew, rsrc, x, r, r + a.slot_n - 1, alpha, guess || it > 1, pold,
                                                   owed};
                    zmarch<double, T, K, KH>(g, lds, par, pu, w64, pg, a.nx, a.ny, a.nz);
                    rn = block_sum<T>(pu.rr, red);
                    pending = false;
                }
                ++it;
                const double beta = rn / rr;
                rr = rn;
                rsrc = r;
                if (rr <= stop) { conv = 1; break; }
                if (it >= a.maxit) break;
                double *t = pold; pold = pnew; pnew = t;
                PDir<double, K, KH, PF64> pd{r, pold, pnew, pnew + a.slot_n - 1, beta, true, false};
                zmarch<double, T, K, KH>(g, lds, par, pd, w64, pg, a.nx, a.ny, a.nz);
                pap = block_sum<T>(pd.pap, red);
            }
            if (pending) {
                // the last iteration's step (its p is still in pnew); x holds
                // a value once a paired update has run or a guess was given
                const bool xv = guess || it > 2;
                for (int q = tid; q < g.n_pe; q += T) x[q] = (xv ? x[q] : 0.0) + owed * pnew[q];
                __syncthreads();
            }
        }
    } else {
        // FP32 CG with reliable updates.  The FP32 system is scaled so its
        // residual has unit RMS (pair densities of distant orbitals are far
        // below the FP32 range); the FP32 solution increment d is folded into
        // the FP64 x, and the residual replaced by the true FP64 b - A x,
        // whenever the recursive residual has dropped by a factor 10 since the
        // last replacement or claims convergence.  The search direction is
        // kept across replacements.
        double *r64 = a.scratch + slot * 3 * a.slot_n;
        float *r32 = a.scratch32 + slot * 4 * a.slot_n;
        float *d32 = r32 + a.slot_n;
        float *pold = d32 + a.slot_n, *pnew = pold + a.slot_n;
        const StencilW<float> w32 = stencil_w<float>(a);
        const double n_el = (double)g.n_pe;
        const double stop_rel2 = a.tol * a.tol;
        if (!guess) {
            for (int q = tid; q < g.n_pe; q += T) x[q] = 0.0;
            __syncthreads();
        }
        double sigma = 1.0, rr_s = 0.0, rmax = 0.0, beta = 0.0;
        bool have_d = false, first = true;
        for (;;) {
            // true residual of x (+ sigma d), in FP64
            PRes<K, KH, float, double, PF64> pr{x, d32, b, r64, r64 + a.slot_n - 1, have_d, sigma};
            zmarch<double, T, K, KH>(g, lds, par, pr, w64, pg, a.nx, a.ny, a.nz);
            ++outer;
            const double rr_true = block_sum<T>(pr.rr, red);
            if (first) bb = block_sum<T>(pr.bb, red);
            if (have_d) {
                for (int q = tid; q < g.n_pe; q += T) x[q] += sigma * (double)d32[q];
                __syncthreads();
            }
            if (bb == 0.0 || rr_true <= stop_rel2 * bb) {
                if (bb == 0.0) {
                    for (int q = tid; q < g.n_pe; q += T) x[q] = 0.0;
                    __syncthreads();
                }
                conv = 1;
                break;
            }
            if (it >= a.maxit) break;
            const double sigma_new = sqrt(rr_true / n_el);
            const double inv = 1.0 / sigma_new;            // scale in FP64, then round
            for (int q = tid; q < g.n_pe; q += T) r32[q] = (float)(r64[q] * inv);
            __syncthreads();
            // direction update with the replaced residual: beta = |r_new|^2 / |r_old|^2
            // in unscaled units; p_old was scaled by sigma, rescale it to sigma_new
            const double beta_eff = first ? 0.0 : (rr_true / (rr_s * sigma * sigma)) * (sigma / sigma_new);
            rr_s = rr_true / (sigma_new * sigma_new);
            sigma = sigma_new;
            rmax = rr_true;
            have_d = false;
            beta = beta_eff;
            // d is updated every other iteration, as x in the FP64 loop
            float owed = 0.f;
            bool pending = false;
            for (;;) {
                double pap;
                {
                    if (!first) { float *t = pold; pold = pnew; pnew = t; }
                    PDir<float, K32, KH32, PF32> pd{r32, pold, pnew, pnew + a.slot_n - 1, (float)beta, !first, false};
                    zmarch<float, T, K32, KH32>(g, lds, par, pd, w32, pg, a.nx, a.ny, a.nz);
                    pap = block_sum<T>(pd.pap, red);
                }
                first = false;
                const float alpha = (float)(rr_s / pap);
                double rn_s;
                if (!pending) {
                    PUpd<float, K32, KH32, XM_SKIP, PF32> pu{pnew, r32, d32, r32, r32 + a.slot_n - 1, alpha, false};
                    zmarch<float, T, K32, KH32>(g, lds, par, pu, w32, pg, a.nx, a.ny, a.nz);
                    rn_s = block_sum<T>(pu.rr, red);
                    owed = alpha;
                    pending = true;
                } else {
                    PUpd<float, K32, KH32, XM_PAIR, PF32> pu{pnew, r32, d32, r32, r32 + a.slot_n - 1, alpha, have_d, pold,
                                                      owed};
                    zmarch<float, T, K32, KH32>(g, lds, par, pu, w32, pg, a.nx, a.ny, a.nz);
                    rn_s = block_sum<T>(pu.rr, red);
                    have_d = true;
                    pending = false;
                }
                ++it;
                const double rr_un = rn_s * sigma * sigma;
                if (rr_un <= stop_rel2 * bb || rr_un <= 0.01 * rmax || it >= a.maxit || !(rn_s == rn_s)) {
                    // replace the residual: rr_s keeps |r_k|^2 of the step just taken,
                    // the next beta uses the true |r_k+1|^2
                    break;
                }
                beta = rn_s / rr_s;
                rr_s = rn_s;
            }
            if (pending) {
                // the owed step of the last iteration (its p is still in pnew)
                for (int q = tid; q < g.n_pe; q += T) d32[q] = (have_d ? d32[q] : 0.f) + owed * pnew[q];
                __syncthreads();
                have_d = true;
            }
        }
    }

    PFin<K, KH, PF64> pf{x, b};
    zmarch<double, T, K, KH>(g, lds, par, pf, w64, pg, a.nx, a.ny, a.nz);
    const double res = block_sum<T>(pf.res, red);
    if (tid == 0) {
        a.iters_out[pair] = it;
        a.outer_out[pair] = outer;
        a.conv_out[pair] = conv;
        a.relres_out[pair] = bb > 0.0 ? sqrt(res / bb) : 0.0;
    }
    __syncthreads();
}

template <int T, int K, int KH, int K32, int KH32, int WPE, int MODE, int PF64, int PF32>
__global__ __launch_bounds__(T, WPE) void k_cg_zmarch(SolveArgs a)
{
    extern __shared__ double lds_dyn[];
    __shared__ double red[T / 64];
    __shared__ int s_pair;
    if (a.clock && threadIdx.x == 0) atomicMin(&a.clock[0], (unsigned long long)wall_clock64());
    int par = 0;
    int last_cls = -1;
    for (;;) {
        if (threadIdx.x == 0) s_pair = atomicAdd(a.counter, 1);
        __syncthreads();
        const int k = s_pair;
        __syncthreads();
        if (k >= a.wave_n) break;
        const int pair = a.queue ? a.queue[a.wave_begin + k] : a.wave_begin + k;
        const int cls = a.pair_gc[pair].w;
        if (cls != last_cls) {
            // the row-offset table of the class lives at the start of LDS
            const ClassDev g = a.cls[cls];
            int *tbl = reinterpret_cast<int *>(lds_dyn);
            for (int t = threadIdx.x; t < g.pnz * g.pny; t += T) tbl[t] = g.pe_off[t];
            __syncthreads();
            last_cls = cls;
        }
        cg_zmarch_pair<T, K, KH, K32, KH32, MODE, PF64, PF32>(a, pair, blockIdx.x, lds_dyn, red, par);
    }
    if (a.clock && threadIdx.x == 0) atomicMax(&a.clock[1], (unsigned long long)wall_clock64());
}

// ---------------------------------------------------------------------------
// pair energy (Step V, Eq. exx_omega): e_ij = h^3 sum_PE rho_ij x, rho_ij
// re-gathered from the orbital boxes.  One work-group per pair of the wave.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(PREP_BLOCK) void k_pair_energy(SolveArgs a)
{
    __shared__ double red[PREP_BLOCK / 64];
    const int pair = a.wave_begin + blockIdx.x;
    const int4 pg = a.pair_gc[pair];
    const int2 ij = a.pair_ij[pair];
    const ClassDev &g = a.cls[pg.w];
    const double *x = a.vout + a.out_off[pair];
    const long long oi = (long long)ij.x * a.box.vol, oj = (long long)ij.y * a.box.vol;
    const int4 org_i = a.box.org[ij.x], org_j = a.box.org[ij.y];
    double e = 0.0;
    for (int q = threadIdx.x; q < g.n_pe; q += PREP_BLOCK) {
        int ox, oy, oz;
        unpack_xyz(g.pe_xyz[q], ox, oy, oz);
        e += pair_rho(a, pg, oi, oj, org_i, org_j, ox, oy, oz) * x[q];
    }
    e = block_sum<PREP_BLOCK>(e, red);
    if (threadIdx.x == 0) a.e_out[pair] = e * (a.h[0] * a.h[1] * a.h[2]);
}

// ---------------------------------------------------------------------------
// initial guess from earlier steps, and the history it reads
// ---------------------------------------------------------------------------

// x0(o) = sum_k c_k v_{t-k}(o + shift_k) on PE, zero where the shifted point
// lies outside the earlier PE sphere.  One work-group per pair of the wave.
__global__ __launch_bounds__(256) void k_guess(GuessArgs a)
{
    const int pair = a.wave_begin + blockIdx.x;
    const int4 pg = a.pair_gc[pair];
    const ClassDev g = a.cls[pg.w];
    const PairGuess pgs = a.guess[pair];
    double *x = a.vout + a.out_off[pair];
    for (int q = threadIdx.x; q < g.n_pe; q += 256) {
        int ox, oy, oz;
        unpack_xyz(g.pe_xyz[q], ox, oy, oz);
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (pgs.off[k] < 0) continue;
            const int4 sh = pgs.shift[k];
            const int src = pe_index(g, ox + sh.x, oy + sh.y, oz + sh.z);
            if (src >= 0) v += pgs.coef[k] * (double)a.hist[k][pgs.off[k] + src];
        }
        x[q] = v;
    }
}

// hist[hist_off[p] + q] = v_p on PE (FP32), for every pair.
__global__ __launch_bounds__(256) void k_save_history(const double *vout, const long long *out_off,
                                                      const long long *hist_off, const int4 *pair_gc, int4 n_pe,
                                                      int wave_begin, float *hist)
{
    const int p = wave_begin + blockIdx.x;
    const int w = pair_gc[p].w;
    const int n = w == 0 ? n_pe.x : w == 1 ? n_pe.y : w == 2 ? n_pe.z : n_pe.w;
    const double *src = vout + out_off[p];
    float *dst = hist + hist_off[p];
    for (int q = threadIdx.x; q < n; q += 256) dst[q] = (float)src[q];
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

__global__ void k_wave_reset(int *counter, unsigned long long *clock)
{
    if (threadIdx.x == 0) {
        counter[0] = 0;
        clock[0] = ~0ULL;
        clock[1] = 0;
    }
}

// ---------------------------------------------------------------------------
// fixed device scratch of the allocation-free solve
// ---------------------------------------------------------------------------

// The CG work vectors of exx_solve_static live here instead of in the
// context's buffers.  Each GPU the library runs on holds its own copy from
// module load until the process ends.  In host code the name is a host-side
// stand-in, never a device address: the address comes from
// hipGetSymbolAddress, per device (static_scratch_address).
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

size_t static_scratch_bytes() { return kStaticScratchBytes; }

// Device address of this GPU's scratch array; call with the device current.
hipError_t static_scratch_address(void **ptr) { return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch)); }

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// (threads, FP64 columns / halo columns per thread, FP32 columns / halo
// columns per thread, min waves per SIMD, planes of loads in flight in the
// FP64 / FP32 passes, the modes it is built for as a bit mask over CG_*).
// The kernel inlines every pass of its mode, and the register allocation
// covers all of them at once: 8 FP32 columns per thread fit beside 4 FP64
// columns in the FP32 modes only without the multigrid V-cycle, so the FP32
// multigrid mode runs 4 FP32 columns.  Two planes in flight need a second
// copy of every loaded value, more than a wave has beside the rest of a mode
// (they are supported by the march, not built).
constexpr int MODES_ALL = 0x1f;
constexpr int MODES_BUT_MGMIX = MODES_ALL & ~(1 << 4);
constexpr int MODES_MGMIX = 1 << 4;
#define EXX_ZM_VARIANTS(X)                                                                                \
    X(256, 4, 2, 8, 2, 2, 1, 1, MODES_BUT_MGMIX) X(512, 4, 1, 8, 1, 2, 1, 1, MODES_BUT_MGMIX)              \
    X(512, 6, 1, 8, 1, 2, 1, 1, MODES_BUT_MGMIX) X(256, 4, 2, 4, 2, 2, 1, 1, MODES_MGMIX)                \
    X(512, 4, 1, 4, 1, 2, 1, 1, MODES_MGMIX)

static const CgVariant kVariants[] = {
    {0, 256, 0, 0, 0, 0, 0, 1, 1, MODES_ALL},
#define EXX_V(T, K, KH, K32, KH32, W, P64, P32, MS) {1, T, K, KH, K32, KH32, W, P64, P32, MS},
    EXX_ZM_VARIANTS(EXX_V)
#undef EXX_V
};

int cg_variants(CgVariant *out, int max_n)
{
    int n = 0;
    for (const CgVariant &v : kVariants)
        if (n < max_n) out[n++] = v;
    return n;
}

bool cg_variant_applies(const CgVariant &v, int mode) { return (v.modes >> mode) & 1; }

template <int T, int K, int KH, int K32, int KH32, int W, int M, int P64, int P32, int MS>
static hipError_t zm_occ(size_t lds, int *per_cu)
{
    if constexpr (!((MS >> M) & 1)) {
        return hipErrorInvalidValue;
    } else {
        auto *f = &k_cg_zmarch<T, K, KH, K32, KH32, W, M, P64, P32>;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(f),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, f, T, lds);
    }
}

template <int T, int K, int KH, int K32, int KH32, int W, int M, int P64, int P32, int MS>
static hipError_t zm_launch(const SolveArgs &a, int grid, size_t lds, hipStream_t s)
{
    if constexpr (!((MS >> M) & 1)) {
        return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((k_cg_zmarch<T, K, KH, K32, KH32, W, M, P64, P32>), dim3(grid), dim3(T), lds, s, a);
        return hipGetLastError();
    }
}

#define EXX_MATCH(v, T, K, KH, K32, KH32, W, P64, P32, MS)                                              \
    ((v).block == T && (v).cols == K && (v).halo == KH && (v).cols32 == K32 && (v).halo32 == KH32 &&  \
     (v).wpe == W && (v).pf64 == P64 && (v).pf32 == P32 && (v).modes == MS)

int cg_mode(int precision, int guess, int mg)
{
    return mg ? (precision ? CG_MG_MIXED : CG_MG) : precision ? CG_MIXED : guess ? CG_FP64_GUESS : CG_FP64;
}

hipError_t cg_occupancy(const CgVariant &v, int mode, size_t lds, int *blocks_per_cu)
{
    if (!v.zmarch) return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_solve<256>, 256, 0);
#define EXX_V(T, K, KH, K32, KH32, W, P64, P32, MS)                                                          \
    if (EXX_MATCH(v, T, K, KH, K32, KH32, W, P64, P32, MS)) {                                                     \
        switch (mode) {                                                                                       \
        case CG_MG_MIXED: return zm_occ<T, K, KH, K32, KH32, W, CG_MG_MIXED, P64, P32, MS>(lds, blocks_per_cu);   \
        case CG_MG: return zm_occ<T, K, KH, K32, KH32, W, CG_MG, P64, P32, MS>(lds, blocks_per_cu);               \
        case CG_MIXED: return zm_occ<T, K, KH, K32, KH32, W, CG_MIXED, P64, P32, MS>(lds, blocks_per_cu);         \
        case CG_FP64_GUESS: return zm_occ<T, K, KH, K32, KH32, W, CG_FP64_GUESS, P64, P32, MS>(lds, blocks_per_cu); \
        default: return zm_occ<T, K, KH, K32, KH32, W, CG_FP64, P64, P32, MS>(lds, blocks_per_cu);                \
        }                                                                                                     \
    }
    EXX_ZM_VARIANTS(EXX_V)
#undef EXX_V
    return hipErrorInvalidValue;
}

hipError_t launch_cg(const CgVariant &v, const SolveArgs &a, int grid, size_t lds, hipStream_t s)
{
    if (!v.zmarch) {
        hipLaunchKernelGGL(k_solve<256>, dim3(grid), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    const int mode = cg_mode(a.precision, a.guess, a.mg);
#define EXX_V(T, K, KH, K32, KH32, W, P64, P32, MS)                                               \
    if (EXX_MATCH(v, T, K, KH, K32, KH32, W, P64, P32, MS)) {                                          \
        switch (mode) {                                                                            \
        case CG_MG_MIXED: return zm_launch<T, K, KH, K32, KH32, W, CG_MG_MIXED, P64, P32, MS>(a, grid, lds, s); \
        case CG_MG: return zm_launch<T, K, KH, K32, KH32, W, CG_MG, P64, P32, MS>(a, grid, lds, s);    \
        case CG_MIXED: return zm_launch<T, K, KH, K32, KH32, W, CG_MIXED, P64, P32, MS>(a, grid, lds, s); \
        case CG_FP64_GUESS: return zm_launch<T, K, KH, K32, KH32, W, CG_FP64_GUESS, P64, P32, MS>(a, grid, lds, s); \
        default: return zm_launch<T, K, KH, K32, KH32, W, CG_FP64, P64, P32, MS>(a, grid, lds, s);     \
        }                                                                                          \
    }
    EXX_ZM_VARIANTS(EXX_V)
#undef EXX_V
    return hipErrorInvalidValue;
}

hipError_t launch_pair_energy(const SolveArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_pair_energy, dim3(a.wave_n), dim3(PREP_BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_prep(const SolveArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_prep, dim3(a.wave_n), dim3(PREP_BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_energy(const double *e, const int2 *ij, int n_pairs, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(1024), 0, s, e, ij, n_pairs, out);
    return hipGetLastError();
}

hipError_t launch_guess(const GuessArgs &a, int n_pairs, hipStream_t s)
{
    hipLaunchKernelGGL(k_guess, dim3(n_pairs), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_save_history(const double *vout, const long long *out_off, const long long *hist_off,
                               const int4 *pair_gc, int4 n_pe, int wave_begin, int wave_n, float *hist,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_save_history, dim3(wave_n), dim3(256), 0, s, vout, out_off, hist_off, pair_gc, n_pe,
                       wave_begin, hist);
    return hipGetLastError();
}

hipError_t launch_wave_reset(int *counter, unsigned long long *clock, hipStream_t s)
{
    hipLaunchKernelGGL(k_wave_reset, dim3(1), dim3(64), 0, s, counter, clock);
    return hipGetLastError();
}

hipError_t launch_zero_int(int *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_int, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace exx
