// exx_dxx.hip -- accumulation of the exchange potentials (Sec. III.C Step V,
// Eq. Dxx_mlwf_omega): D^k = sum over the pairs (k, j) of v_kj phi_j, over the
// whole ME sphere of each pair, owner computes, in pair order, no atomics.
//
// One work-group per compact tile of orbital k's box (DXX_TX x DXX_TY x
// DXX_TZ points; each thread a run of DXX_PER_THREAD consecutive x points of
// one row, so one lookup of the pair's ME row table serves the run).  The
// work-group walks k's pairs of the current wave in pair order and skips, as
// a whole, every pair whose ME bounding box misses the tile's bounding box; a
// compact tile meets few of the pairs, and of a pair it meets most points lie
// in the ME box.  Each point adds the contributions of
// the pairs whose ME sphere holds it in pair order, so the sum is the same
// FP64 sum whatever the tiling.  With the pairs in waves the sums are carried
// across waves in FP64 partial sums and rounded once at the end.
#include "exx_internal.h"

#include <algorithm>

namespace exx {

// 32 x 8 x 8 points, runs of 8: the fastest of the shapes timed on the
// 512-water step (runs of 4, 8 or 16 in x; 32 x 4 x 16 and 32 x 16 x 4;
// columns of 4 points along z in 16 x 8 x 8 and 32 x 8 x 4 tiles)
constexpr int DXX_TX = 32, DXX_TY = 8, DXX_TZ = 8, DXX_PER_THREAD = 8;
constexpr int DXX_BLOCK = DXX_TX / DXX_PER_THREAD * DXX_TY * DXX_TZ;

// Do the cyclic index ranges [a0, a0 + alen) and [b0, b0 + blen) of Z_n meet
// (a0, b0 in [0, n); lengths at most n)?
__device__ __forceinline__ bool cyclic_meet(int a0, int alen, int b0, int blen, int n)
{
    int d1 = a0 - b0, d2 = b0 - a0;
    d1 += d1 < 0 ? n : 0;
    d2 += d2 < 0 ? n : 0;
    return d1 < blen || d2 < alen;
}

// grid (tiles of one box, n_orb).  A tile no pair of the wave reaches writes
// zeros (the first wave, or D directly) or nothing (a later wave's partial
// sums are unchanged).
template <typename TO, bool ACC>
__global__ __launch_bounds__(DXX_BLOCK) void k_dxx(DxxArgs a)
{
    const int k = blockIdx.y;
    const OrbBox &B = a.box;
    const int ntx = (B.bx + DXX_TX - 1) / DXX_TX, nty = (B.by + DXX_TY - 1) / DXX_TY;
    const int tile = blockIdx.x;
    const int bx0 = (tile % ntx) * DXX_TX, by0 = ((tile / ntx) % nty) * DXX_TY, bz0 = (tile / (ntx * nty)) * DXX_TZ;
    const int4 ok_org = B.org[k];
    // this orbital's pairs inside [pair_lo, pair_hi): its list is ascending
    int lo = a.orb_ptr[k], hi = a.orb_ptr[k + 1];
    {
        int l = lo, r = hi;
        while (l < r) { const int m = (l + r) >> 1; if (a.orb_pairs[m] < a.pair_lo) l = m + 1; else r = m; }
        int l2 = l, r2 = hi;
        while (l2 < r2) { const int m = (l2 + r2) >> 1; if (a.orb_pairs[m] < a.pair_hi) l2 = m + 1; else r2 = m; }
        lo = l;
        hi = l2;
    }
    // the tile's bounding box in global grid coordinates (start, length per axis)
    const int xlen = min(DXX_TX, B.bx - bx0), ylen = min(DXX_TY, B.by - by0), zlen = min(DXX_TZ, B.bz - bz0);
    const int xs = wrap_n(ok_org.x + bx0, a.nx), ys = wrap_n(ok_org.y + by0, a.ny), zs = wrap_n(ok_org.z + bz0, a.nz);
    auto meets = [&](int pair) -> bool {
        const int4 pg = a.pair_gc[pair];
        const ClassDev &g = a.cls[pg.w];
        return cyclic_meet(zs, zlen, wrap_n(pg.z + g.mzlo, a.nz), g.mnz, a.nz) &&
               cyclic_meet(ys, ylen, wrap_n(pg.y + g.mylo, a.ny), g.mny, a.ny) &&
               cyclic_meet(xs, xlen, wrap_n(pg.x + g.mxlo, a.nx), g.mnx, a.nx);
    };
    // this thread's run of DXX_PER_THREAD consecutive x points at (y, z)
    constexpr int QX = DXX_TX / DXX_PER_THREAD;
    const int lx0 = bx0 + DXX_PER_THREAD * (threadIdx.x % QX);
    const int ly = by0 + (threadIdx.x / QX) % DXX_TY, lz = bz0 + threadIdx.x / (QX * DXX_TY);
    const bool row_ok = ly < B.by && lz < B.bz;
    bool any = false;
    for (int pp = lo; pp < hi && !any; ++pp) any = meets(a.orb_pairs[pp]);
    if (!any) {
        if (ACC && !a.acc_first) return;
#pragma unroll
        for (int e = 0; e < DXX_PER_THREAD; ++e) {
            const int lx = lx0 + e;
            if (!row_ok || lx >= B.bx) continue;
            const long long li = ((long long)lz * B.by + ly) * B.bx + lx;
            if (ACC)
                a.acc[(long long)k * B.vol + li] = 0.0;
            else
                static_cast<TO *>(a.dxx)[(long long)k * B.vol + li] = (TO)0.0;
        }
        return;
    }
    const int gy = wrap_n(ok_org.y + (row_ok ? ly : 0), a.ny), gz = wrap_n(ok_org.z + (row_ok ? lz : 0), a.nz);
    double acc[DXX_PER_THREAD];
    int gx[DXX_PER_THREAD];
    bool ok[DXX_PER_THREAD];
    long long li[DXX_PER_THREAD];
#pragma unroll
    for (int e = 0; e < DXX_PER_THREAD; ++e) {
        const int lx = lx0 + e;
        ok[e] = row_ok && lx < B.bx;
        li[e] = ok[e] ? ((long long)lz * B.by + ly) * B.bx + lx : 0;
        gx[e] = wrap_n(ok_org.x + (ok[e] ? lx : 0), a.nx);
        acc[e] = ACC && !a.acc_first && ok[e] ? a.acc[(long long)k * B.vol + li[e]] : 0.0;
    }
    for (int pp = lo; pp < hi; ++pp) {
        const int pair = a.orb_pairs[pp];
        if (!meets(pair)) continue;
        const int4 pg = a.pair_gc[pair];
        const int2 ij = a.pair_ij[pair];
        const int other = ij.x == k ? ij.y : ij.x;
        const ClassDev &g = a.cls[pg.w];
        const double *v = a.vout + a.out_off[pair];
        const long long oo = (long long)other * B.vol;
        const int4 oo_org = B.org[other];
        // the run's row of the pair's ME box (shared by its points)
        const int ty = wrap_n(gy - pg.y - g.mylo, a.ny), tz = wrap_n(gz - pg.z - g.mzlo, a.nz);
        if (ty >= g.mny || tz >= g.mnz) continue;
        const int row = tz * g.mny + ty;
        const int4 r0 = g.me_rows[2 * row];
        const int4 r1 = g.me_rows[2 * row + 1];
#pragma unroll
        for (int e = 0; e < DXX_PER_THREAD; ++e) {
            if (!ok[e]) continue;
            const int tx = wrap_n(gx[e] - pg.x - g.mxlo, a.nx);
            if (tx >= g.mnx) continue;
            const int ox = tx + g.mxlo;
            if (ox < r1.x || ox > r1.y) continue;
            double vv;
            if (ox >= r0.y && ox <= r0.z)
                vv = v[r0.x + ox - r0.y];
            else
                vv = v[g.n_pe + r0.w + (ox < r0.y ? ox - r1.x : (r0.y - r1.x) + (ox - r0.z - 1))];
            acc[e] += vv * load_orb(a.phi, a.f32, B, oo, oo_org, gx[e], gy, gz, a.nx, a.ny, a.nz);
        }
    }
#pragma unroll
    for (int e = 0; e < DXX_PER_THREAD; ++e) {
        if (!ok[e]) continue;
        if (ACC)
            a.acc[(long long)k * B.vol + li[e]] = acc[e];
        else
            static_cast<TO *>(a.dxx)[(long long)k * B.vol + li[e]] = (TO)acc[e];
    }
}

// dxx = the FP64 partial sums, rounded to the orbital dtype.
template <typename TO>
__global__ void k_dxx_final(const double *acc, TO *dxx, long long n)
{
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
        dxx[t] = (TO)acc[t];
}

hipError_t launch_dxx(const DxxArgs &a, int n_orb, int accumulate, hipStream_t s)
{
    const long long tiles = (long long)((a.box.bx + DXX_TX - 1) / DXX_TX) * ((a.box.by + DXX_TY - 1) / DXX_TY) *
                            ((a.box.bz + DXX_TZ - 1) / DXX_TZ);
    const dim3 grid((unsigned)tiles, (unsigned)n_orb);
    if (accumulate)
        hipLaunchKernelGGL((k_dxx<double, true>), grid, dim3(DXX_BLOCK), 0, s, a);
    else if (a.f32)
        hipLaunchKernelGGL((k_dxx<float, false>), grid, dim3(DXX_BLOCK), 0, s, a);
    else
        hipLaunchKernelGGL((k_dxx<double, false>), grid, dim3(DXX_BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_dxx_final(const DxxArgs &a, int n_orb, hipStream_t s)
{
    const long long n = (long long)n_orb * a.box.vol;
    const dim3 grid((unsigned)std::min<long long>((n + 255) / 256, 1LL << 20));
    if (a.f32)
        hipLaunchKernelGGL(k_dxx_final<float>, grid, dim3(256), 0, s, a.acc, static_cast<float *>(a.dxx), n);
    else
        hipLaunchKernelGGL(k_dxx_final<double>, grid, dim3(256), 0, s, a.acc, static_cast<double *>(a.dxx), n);
    return hipGetLastError();
}

}  // namespace exx
