// exx_pairs.hip -- the pair list on the GPU (Step II of Sec. III C): every
// orbital pair whose centres lie closer than R_pair under the minimum image,
// with the pair origin of Step III.
//
// The centres are binned on the host into a periodic cell list whose cells
// are at least R_pair wide, so every pair within R_pair lies in the same or
// an adjacent cell.  One thread per orbital i scans the (up to 27) distinct
// neighbouring cells for partners j > i, counts them, and after the host's
// prefix sum writes its segment: the self pair first, then the partners in
// ascending j (an insertion sort of the segment), each with its origin and
// subdomain class.  The list therefore comes out in the order of the plain
// double loop over i <= j.
//
// Bit-exact with the plain O(N^2) test: the distance and the origin use the
// same FP64 operations in the same order, with contraction into FMA off (a
// fused multiply-add rounds once where the definition rounds twice, which
// could move a pair across the cutoff or an origin across a half-way point).
#pragma clang fp contract(off)

#include "exx_internal.h"

namespace exx {

namespace {

__device__ __forceinline__ long nint_away_d(double v)
{
    return (long)(v >= 0.0 ? floor(v + 0.5) : -floor(-v + 0.5));
}

__device__ __forceinline__ int mod_pos_d(long a, int n)
{
    const long r = a % n;
    return (int)(r < 0 ? r + n : r);
}

// minimum-image displacement C_j - C_i and its squared length
__device__ __forceinline__ double min_image(const PairArgs &a, int i, int j, double (&d)[3])
{
    double dd = 0.0;
    for (int k = 0; k < 3; ++k) {
        double v = a.C[3 * j + k] - a.C[3 * i + k];
        v -= a.L[k] * (double)nint_away_d(v / a.L[k]);
        d[k] = v;
        dd += v * v;
    }
    return dd;
}

// calls f(j) for every partner j > i within R_pair
template <class F>
__device__ __forceinline__ void for_partners(const PairArgs &a, int i, F f)
{
    const int ci = a.cell_of[i];
    const int cx = ci % a.nc[0], cy = (ci / a.nc[0]) % a.nc[1], cz = ci / (a.nc[0] * a.nc[1]);
    // distinct neighbour offsets per axis: {0} for 1 cell, {0, 1} for 2, {-1, 0, 1} for 3 or more
    int lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = a.nc[k] >= 3 ? -1 : 0;
        hi[k] = a.nc[k] >= 2 ? 1 : 0;
    }
    for (int oz = lo[2]; oz <= hi[2]; ++oz)
        for (int oy = lo[1]; oy <= hi[1]; ++oy)
            for (int ox = lo[0]; ox <= hi[0]; ++ox) {
                const int nx = mod_pos_d(cx + ox, a.nc[0]), ny = mod_pos_d(cy + oy, a.nc[1]),
                          nz = mod_pos_d(cz + oz, a.nc[2]);
                const int cell = (nz * a.nc[1] + ny) * a.nc[0] + nx;
                for (int t = a.cell_start[cell]; t < a.cell_start[cell + 1]; ++t) {
                    const int j = a.cell_items[t];
                    if (j <= i) continue;
                    double d[3];
                    if (min_image(a, i, j, d) < a.r2) f(j);
                }
            }
}

__global__ void k_pair_count(PairArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_orb) return;
    int n = 1;                                   // the self pair
    for_partners(a, i, [&](int) { ++n; });
    a.count[i] = n;
}

__global__ void k_pair_fill(PairArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_orb) return;
    const long long s = a.start[i];
    int n = 0;
    a.ij[s] = int2{i, i};
    ++n;
    for_partners(a, i, [&](int j) {
        // insertion into the sorted tail of the segment
        long long p = s + n;
        while (p > s + 1 && a.ij[p - 1].y > j) {
            a.ij[p] = a.ij[p - 1];
            --p;
        }
        a.ij[p] = int2{i, j};
        ++n;
    });
    // origins (Step III): the minimum-image midpoint, wrapped into the cell,
    // snapped to the nearest grid point; class 0 for the self pair
    for (int t = 0; t < n; ++t) {
        const int j = a.ij[s + t].y;
        double d[3];
        (void)min_image(a, i, j, d);
        int g[3];
        for (int k = 0; k < 3; ++k) {
            double m = a.C[3 * i + k] + 0.5 * d[k];
            m -= a.L[k] * floor(m / a.L[k]);
            g[k] = mod_pos_d(nint_away_d(m / a.h[k]), a.N[k]);
        }
        a.gc[s + t] = int4{g[0], g[1], g[2], i == j ? 0 : 1};
    }
}

}  // namespace

hipError_t launch_pair_count(const PairArgs &a, hipStream_t s)
{
    const int T = 256;
    hipLaunchKernelGGL(k_pair_count, dim3((a.n_orb + T - 1) / T), dim3(T), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pair_fill(const PairArgs &a, hipStream_t s)
{
    const int T = 256;
    hipLaunchKernelGGL(k_pair_fill, dim3((a.n_orb + T - 1) / T), dim3(T), 0, s, a);
    return hipGetLastError();
}

}  // namespace exx
