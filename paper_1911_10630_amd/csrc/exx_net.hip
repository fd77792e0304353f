// exx_net.hip -- learned initial guess for the pair Poisson solves.
//
// The paper (Sec. III.C, Step IV) starts each pair's CG from a guess (the
// previous MD step's potential, extrapolated) and points to better guesses
// as the way to fewer iterations (Sec. IV.B).  Here a small convolutional
// U-Net maps a pair's right-hand side b, averaged onto a coarse cube around
// the pair, to the coarse solution; its output is trilinearly interpolated
// back onto the PE sphere and used as the CG starting point.  CG then runs to
// the same residual target, so the guess changes the iteration count, never
// the converged result.
//
// Net (coarse edge D, multiple of 8; channels-last bf16 activations; bf16
// weights with FP32 master copies; FP32 accumulation; ReLU; no biases):
//   e1 = c1(c0(in))        D     3 (padded to 16) -> 16 -> 16
//   e2 = c3(c2(pool e1))   D/2   16 -> 32 -> 32
//   e3 = c5(c4(pool e2))   D/4   32 -> 64 -> 64
//   e4 = c7(c6(pool e3))   D/8   64 -> 64 -> 64
//   d3 = c8 (cat(up e4, e3))  D/4  128 -> 64
//   d2 = c9 (cat(up d3, e2))  D/2   96 -> 32
//   d1 = c10(cat(up d2, e1))  D     48 -> 16
//   out = c11(d1)             D     16 -> 16 (channel 0 is the potential; no ReLU)
// Convolutions are 3x3x3 with zero padding, computed as implicit GEMMs on the
// 16x16x32 bf16 MFMA: M = voxels, N = output channels, K = taps x input
// channels, the input tile staged in LDS once per 16-channel chunk and read
// by all 27 taps.  The input gradient is the same kernel with tap-flipped,
// transposed weights; the weight gradient is a second MFMA kernel whose K is
// the voxels.  pool = 2x2x2 mean, up = nearest-neighbour 2x.
#include "exx_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

namespace exx {

typedef unsigned short bf16_t;
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef short s8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16_t f2bf(float f)
{
    const unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (bf16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));   // inf / nan
    return (bf16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);                                           // nearest even
}
__device__ __forceinline__ float bf2f(bf16_t b) { return __uint_as_float(((unsigned)b) << 16); }

// ---------------------------------------------------------------------------
// convolutions
// ---------------------------------------------------------------------------

// Y[v][co] = sum_tap sum_ci X[v + off(tap)][ci] W[tap][co][ci], off(tap) =
// (tap % 3, tap / 3 % 3, tap / 9) - 1 in (x, y, z).  N samples of D^3 voxels.
//
// Implicit GEMM on the 16x16x32 bf16 MFMA: M = voxels, N = output channels,
// K = 28 taps (the last one zero) x 16-channel chunks, two taps per MFMA.
// A work-group (four waves) computes an 8 x 8 x TZ tile of one sample and
// every output channel; per 16-channel chunk it stages the tile's input halo
// (10 x 10 x (TZ + 2) voxels, zero outside the cube) in LDS, and all 27 taps
// read their A fragments from there.  An M tile is a 4 x 4 (x, y) patch of
// one plane; each wave holds MV of them times NCO = Cout / 16 channel tiles,
// so a weight fragment feeds MV MFMAs and an input fragment NCO.
//
// Weights are packed per chunk and tap pair, Wk[chunk][s][co][32]: slots
// 0..15 hold tap 2s, slots 16..31 tap 2s + 1, 16 input channels each (tap
// 27 is zero).  Lane group g = lane / 16 supplies k slots 8g .. 8g + 7 of
// both operands, i.e. tap 2s + g / 2 and channels 8 (g % 2) .. + 7 of the
// chunk; the product is independent of which physical k the hardware
// assigns to a slot, since A and B use the same slot map.
constexpr int CT_XY = 8;                 // tile edge in x and y
constexpr int CH_XY = CT_XY + 2;         // halo edge
constexpr int CH_RP = 12;                // LDS row pitch (voxels): rows 8 banks apart
constexpr int CH_PP = CH_XY * CH_RP;     // LDS plane pitch (voxels)

template <int MV, int NCO, bool RELU, bool OUT_F32>
__global__ __launch_bounds__(256) void k_conv3(const bf16_t *__restrict__ X, const bf16_t *__restrict__ W, void *Yv,
                                               int N, int D, int Cin)
{
    constexpr int TZ = MV, HZ = TZ + 2, Cout = 16 * NCO;
    __shared__ uint4 tile[HZ * CH_PP * 2];   // 16 channels = two uint4 per voxel
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int nxy = (D + CT_XY - 1) / CT_XY, nzt = (D + TZ - 1) / TZ;
    int b = blockIdx.x;
    const int bx = b % nxy;
    b /= nxy;
    const int by = b % nxy;
    b /= nxy;
    const int bz = b % nzt;
    const int n = b / nzt;
    const int x0 = bx * CT_XY, y0 = by * CT_XY, z0 = bz * TZ;
    // this lane's voxel (row m of A) in each of the wave's M tiles, in uint4 units
    int abase[MV];
#pragma unroll
    for (int u = 0; u < MV; ++u) {
        const int ut = wv * MV + u, lz = ut >> 2, p = ut & 3;
        const int lx = (p & 1) * 4 + (m & 3), ly = (p >> 1) * 4 + (m >> 2);
        abase[u] = ((lz + 1) * CH_PP + (ly + 1) * CH_RP + (lx + 1)) * 2 + (g & 1);
    }
    f4_t acc[MV][NCO];
#pragma unroll
    for (int u = 0; u < MV; ++u)
#pragma unroll
        for (int t = 0; t < NCO; ++t) acc[u][t] = (f4_t){0.f, 0.f, 0.f, 0.f};
    const int nch = Cin / 16;
    for (int ch = 0; ch < nch; ++ch) {
        if (ch) __syncthreads();   // the previous chunk's reads are done
        for (int i = tid; i < HZ * CH_XY * CH_XY * 2; i += 256) {
            const int h = i >> 1, half = i & 1;
            const int hx = h % CH_XY, hy = (h / CH_XY) % CH_XY, hz = h / (CH_XY * CH_XY);
            const int x = x0 - 1 + hx, y = y0 - 1 + hy, z = z0 - 1 + hz;
            uint4 v = {0u, 0u, 0u, 0u};
            if ((unsigned)x < (unsigned)D && (unsigned)y < (unsigned)D && (unsigned)z < (unsigned)D)
                v = *reinterpret_cast<const uint4 *>(X + ((((long long)n * D + z) * D + y) * D + x) * Cin + ch * 16 +
                                                     half * 8);
            tile[(hz * CH_PP + hy * CH_RP + hx) * 2 + half] = v;
        }
        __syncthreads();
        const bf16_t *wp = W + ((long long)ch * 14 * Cout + m) * 32 + g * 8;
#pragma unroll
        for (int s = 0; s < 14; ++s) {
            const int tap = 2 * s + (g >> 1);
            const int toff = tap < 27 ? ((tap / 9 - 1) * CH_PP + ((tap / 3) % 3 - 1) * CH_RP + (tap % 3 - 1)) * 2 : 0;
            bf8_t bw[NCO];
#pragma unroll
            for (int t = 0; t < NCO; ++t)
                bw[t] = __builtin_bit_cast(bf8_t, *reinterpret_cast<const uint4 *>(wp + ((long long)s * Cout + t * 16) * 32));
#pragma unroll
            for (int u = 0; u < MV; ++u) {
                const bf8_t a = __builtin_bit_cast(bf8_t, tile[abase[u] + toff]);
#pragma unroll
                for (int t = 0; t < NCO; ++t)
                    acc[u][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[t], acc[u][t], 0, 0, 0);
            }
        }
    }
    // row 4g + i of an M tile is voxel (x + i, y + g) of its patch
#pragma unroll
    for (int u = 0; u < MV; ++u) {
        const int ut = wv * MV + u, p = ut & 3;
        const int z = z0 + (ut >> 2), y = y0 + (p >> 1) * 4 + g;
        if (z >= D || y >= D) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int x = x0 + (p & 1) * 4 + i;
            if (x >= D) continue;
            const long long v = (((long long)n * D + z) * D + y) * D + x;
#pragma unroll
            for (int t = 0; t < NCO; ++t) {
                float val = acc[u][t][i];
                if (RELU) val = fmaxf(val, 0.f);
                const long long o = v * Cout + t * 16 + m;
                if (OUT_F32)
                    static_cast<float *>(Yv)[o] = val;
                else
                    static_cast<bf16_t *>(Yv)[o] = f2bf(val);
            }
        }
    }
}

// The same convolution for cubes smaller than a tile (D < CT_XY, the coarse
// levels, where a tile would be mostly padding and a launch has few tiles).
// grid (ceil(N D^3 / 16), Cout / 16), 256 threads: a work-group computes one
// M tile of 16 consecutive voxels (sample-major, x fastest) times one
// 16-channel output tile, its four waves splitting the K steps (chunk, tap
// pair) four ways, their partial tiles summed in LDS in wave order.  The A
// fragments come straight from global memory (these activations are small
// and stay in L2); same packed weights and slot map as k_conv3.
template <bool RELU, bool OUT_F32>
__global__ __launch_bounds__(256) void k_conv3_small(const bf16_t *__restrict__ X, const bf16_t *__restrict__ W,
                                                     void *Yv, int N, int D, int Cin, int Cout)
{
    __shared__ f4_t part[3][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int D3 = D * D * D, nvox = N * D3;
    const int va = blockIdx.x * 16 + m;
    const bool av = va < nvox;
    const int vs = av ? va : 0;
    const int n = vs / D3, r = vs - n * D3;
    const int z = r / (D * D), y = (r / D) % D, x = r % D;
    const int co = blockIdx.y * 16 + m;
    f4_t acc = {0.f, 0.f, 0.f, 0.f};
    const int nk = (Cin / 16) * 14;
    for (int kk = wv; kk < nk; kk += 4) {
        const int ch = kk / 14, s = kk - ch * 14;
        const int tap = 2 * s + (g >> 1);
        const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
        const bf8_t bw = __builtin_bit_cast(
            bf8_t, *reinterpret_cast<const uint4 *>(W + (((long long)ch * 14 + s) * Cout + co) * 32 + g * 8));
        const int zz = z + dz, yy = y + dy, xx = x + dx;
        const bool ok = av && tap < 27 && (unsigned)zz < (unsigned)D && (unsigned)yy < (unsigned)D &&
                        (unsigned)xx < (unsigned)D;
        const long long vn = ok ? ((long long)n * D + zz) * D * D + (long long)yy * D + xx : 0;
        uint4 raw = *reinterpret_cast<const uint4 *>(X + vn * Cin + ch * 16 + (g & 1) * 8);
        if (!ok) raw = (uint4){0u, 0u, 0u, 0u};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8_t, raw), bw, acc, 0, 0, 0);
    }
    if (wv) part[wv - 1][lane] = acc;
    __syncthreads();
    if (wv) return;
#pragma unroll
    for (int w = 0; w < 3; ++w) acc += part[w][lane];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int v = blockIdx.x * 16 + 4 * g + i;
        if (v >= nvox) continue;
        float val = acc[i];
        if (RELU) val = fmaxf(val, 0.f);
        const long long o = (long long)v * Cout + co;
        if (OUT_F32)
            static_cast<float *>(Yv)[o] = val;
        else
            static_cast<bf16_t *>(Yv)[o] = f2bf(val);
    }
}

// work-groups of k_conv3 for N samples of edge D
__host__ __device__ constexpr long long conv_tiles(int N, int D, int TZ)
{
    return (long long)N * ((D + TZ - 1) / TZ) * ((D + CT_XY - 1) / CT_XY) * ((D + CT_XY - 1) / CT_XY);
}

// dW[tap][co][ci] += sum_v dY[v][co] X[v + off(tap)][ci].
// grid (ceil(N D^3 / chunk), 27, (Cout / 16) (Cin / 16)), 256 threads; each
// wave walks 32-voxel slices of the chunk with stride 128 on the 16x16x32
// MFMA (K = voxels).  A wave's four lane groups take eight consecutive
// voxels each; their coordinates are carried incrementally.
__global__ __launch_bounds__(256) void k_conv3_wgrad(const bf16_t *__restrict__ X, const bf16_t *__restrict__ dY,
                                                     float *dW, int N, int D, int Cin, int Cout, int chunk)
{
    __shared__ float red[4][256];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int tap = blockIdx.y;
    const int nci = Cin / 16;
    const int co_base = (blockIdx.z / nci) * 16, ci_base = (blockIdx.z % nci) * 16;
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const int D3 = D * D * D, nvox = N * D3;
    const int c0 = blockIdx.x * chunk;
    const int c1 = min(c0 + chunk, nvox);
    f4_t acc = {0.f, 0.f, 0.f, 0.f};
    for (int vb = c0 + wv * 32; vb < c1; vb += 128) {
        const int v = vb + 8 * kq;
        int n = v / D3, r = v - n * D3;
        int z = r / (D * D), y = (r / D) % D, x = r % D;
        s8_t a, b;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const bool ok = v + i < c1;
            const int zz = z + dz, yy = y + dy, xx = x + dx;
            const bool okn = ok && (unsigned)zz < (unsigned)D && (unsigned)yy < (unsigned)D && (unsigned)xx < (unsigned)D;
            const long long vn = okn ? (long long)n * D3 + (zz * D + yy) * D + xx : 0;
            const long long vo = ok ? (long long)(v + i) : 0;
            const bf16_t av = dY[vo * Cout + co_base + m];
            const bf16_t bv = X[vn * Cin + ci_base + m];
            a[i] = ok ? (short)av : (short)0;
            b[i] = okn ? (short)bv : (short)0;
            if (++x == D) { x = 0; if (++y == D) { y = 0; if (++z == D) { z = 0; ++n; } } }
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8_t, a), __builtin_bit_cast(bf8_t, b), acc, 0,
                                                      0, 0);
    }
    // sum the four waves' tiles in LDS, then one atomic per element
#pragma unroll
    for (int i = 0; i < 4; ++i) red[wv][(4 * kq + i) * 16 + m] = acc[i];
    __syncthreads();
    const int t = threadIdx.x;
    const float s = red[0][t] + red[1][t] + red[2][t] + red[3][t];
    atomicAdd(&dW[((long long)tap * Cout + co_base + t / 16) * Cin + ci_base + t % 16], s);
}

// ---------------------------------------------------------------------------
// resampling and elementwise kernels (channels-last)
// ---------------------------------------------------------------------------

#define GRID_STRIDE(t, total) \
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < (total); t += (long long)gridDim.x * blockDim.x)

// coarse voxel u of edge D/2 -> first child (edge D)
__device__ __forceinline__ long long child0(long long u, int Dh)
{
    const int x = (int)(u % Dh), y = (int)((u / Dh) % Dh), z = (int)((u / Dh / Dh) % Dh);
    const long long n = u / ((long long)Dh * Dh * Dh);
    const int D = 2 * Dh;
    return ((n * D + 2 * z) * D + 2 * y) * D + 2 * x;
}
// fine voxel v of edge D -> parent (edge D/2)
__device__ __forceinline__ long long parent(long long v, int D)
{
    const int x = (int)(v % D), y = (int)((v / D) % D), z = (int)((v / D / D) % D);
    const long long n = v / ((long long)D * D * D);
    const int Dh = D / 2;
    return ((n * Dh + z / 2) * Dh + y / 2) * Dh + x / 2;
}

// Y[u][c] = mean of X over the 8 children of u (edge D -> D/2)
__global__ void k_pool2(const bf16_t *X, bf16_t *Y, int N, int D, int C)
{
    const int Dh = D / 2;
    GRID_STRIDE(t, (long long)N * Dh * Dh * Dh * C)
    {
        const int c = (int)(t % C);
        const long long v0 = child0(t / C, Dh);
        float s = 0.f;
        for (int k = 0; k < 8; ++k) s += bf2f(X[(v0 + ((k >> 2) * D + ((k >> 1) & 1)) * D + (k & 1)) * C + c]);
        Y[t] = f2bf(0.125f * s);
    }
}

// dX[v][c] = dY[parent(v)][c] / 8
__global__ void k_pool2_bwd(const bf16_t *dY, bf16_t *dX, int N, int D, int C)
{
    GRID_STRIDE(t, (long long)N * D * D * D * C)
    {
        const int c = (int)(t % C);
        dX[t] = f2bf(0.125f * bf2f(dY[parent(t / C, D) * C + c]));
    }
}

// Y[v][0:C1] = L[parent(v)][:], Y[v][C1:C1+C2] = S[v][:]   (Y, S edge D; L edge D/2)
__global__ void k_upcat(const bf16_t *L, const bf16_t *S, bf16_t *Y, int N, int D, int C1, int C2)
{
    const int C = C1 + C2;
    GRID_STRIDE(t, (long long)N * D * D * D * C)
    {
        const int c = (int)(t % C);
        const long long v = t / C;
        Y[t] = c >= C1 ? S[v * C2 + (c - C1)] : L[parent(v, D) * C1 + c];
    }
}

// dL[u][c] = sum over the children v of u of dY[v][c]; dS[v][c] = dY[v][C1 + c]
__global__ void k_upcat_bwd(const bf16_t *dY, bf16_t *dL, bf16_t *dS, int N, int D, int C1, int C2)
{
    const int Dh = D / 2, C = C1 + C2;
    const long long totS = (long long)N * D * D * D * C2;
    const long long totL = (long long)N * Dh * Dh * Dh * C1;
    GRID_STRIDE(t, totS + totL)
    {
        if (t < totS) {
            const int c = (int)(t % C2);
            dS[t] = dY[(t / C2) * C + C1 + c];
        } else {
            const long long tl = t - totS;
            const int c = (int)(tl % C1);
            const long long v0 = child0(tl / C1, Dh);
            float s = 0.f;
            for (int k = 0; k < 8; ++k) s += bf2f(dY[(v0 + ((k >> 2) * D + ((k >> 1) & 1)) * D + (k & 1)) * C + c]);
            dL[tl] = f2bf(s);
        }
    }
}

// dX = (Y > 0) ? dX + dA : 0   (Y = relu output; dA optional)
__global__ void k_relu_bwd(bf16_t *dX, const bf16_t *Y, const bf16_t *dA, long long n)
{
    GRID_STRIDE(t, n)
    {
        float g = bf2f(dX[t]);
        if (dA) g += bf2f(dA[t]);
        dX[t] = bf2f(Y[t]) > 0.f ? f2bf(g) : (bf16_t)0;
    }
}

// Masked squared error on channel 0: tgt[v] = {value, weight}.  dOut
// (16 channels, bf16) = 2 w (out - value) / n_vox; acc[0] += sum w (out -
// value)^2, acc[1] += sum w.
__global__ void k_loss(const float *out, const float2 *tgt, bf16_t *dout, float *acc, long long nvox)
{
    float part = 0.f, wsum = 0.f;
    const float inv = 1.f / (float)nvox;
    GRID_STRIDE(v, nvox)
    {
        const float2 tw = tgt[v];
        const float d = tw.y * (out[v * 16] - tw.x);
        part += d * d;
        wsum += tw.y;
        dout[v * 16] = f2bf(2.f * d * inv);
#pragma unroll
        for (int c = 1; c < 16; ++c) dout[v * 16 + c] = 0;
    }
    for (int off = 32; off > 0; off >>= 1) {
        part += __shfl_xor(part, off);
        wsum += __shfl_xor(wsum, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(acc, part);
        atomicAdd(acc + 1, wsum);
    }
}

// Adam on the FP32 master weights W[tap][co][ci] (gradient cleared after
// use), then the bf16 copies packed for k_conv3: the forward one, and the
// input-gradient one of the transposed layer (Cout inputs, Cin outputs, tap
// 26 - tap).  lr = 0 only refreshes the bf16 copies.
__global__ void k_adam(float *w, float *m, float *v, float *g, bf16_t *w16, bf16_t *wt16, int Cin, int Cout, float lr,
                       float b1, float b2, float c1, float c2, float eps)
{
    GRID_STRIDE(t, 27LL * Cin * Cout)
    {
        float wn = w[t];
        if (lr != 0.f) {
            const float gg = g[t];
            const float mm = b1 * m[t] + (1.f - b1) * gg;
            const float vv = b2 * v[t] + (1.f - b2) * gg * gg;
            m[t] = mm;
            v[t] = vv;
            wn -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
            w[t] = wn;
        }
        g[t] = 0.f;
        const int ci = (int)(t % Cin), co = (int)((t / Cin) % Cout), tap = (int)(t / ((long long)Cin * Cout));
        const int tt = 26 - tap;
        w16[((long long)(ci / 16 * 14 + tap / 2) * Cout + co) * 32 + (tap & 1) * 16 + ci % 16] = f2bf(wn);
        wt16[((long long)(co / 16 * 14 + tt / 2) * Cin + ci) * 32 + (tt & 1) * 16 + co % 16] = f2bf(wn);
    }
}

// ---------------------------------------------------------------------------
// pair <-> coarse cube
// ---------------------------------------------------------------------------
//
// Coarse cell c (per axis, 0 <= c < D) covers the f fine offsets
// -fD/2 + f c + {0 .. f-1}; its centre sits at -fD/2 + f c + (f - 1) / 2.

__device__ __forceinline__ int pair_of(const int *pairs, int base, int k) { return pairs ? pairs[k] : base + k; }

// flag[q] = 1 if the stencil of PE point q reaches outside PE (b carries the
// Dirichlet term there).  PE is convex, so the six far ends decide.
__global__ void k_pe_boundary(ClassDev g, unsigned char *flag)
{
    GRID_STRIDE(q, g.n_pe)
    {
        int ox, oy, oz;
        unpack_xyz(g.pe_xyz[q], ox, oy, oz);
        const bool inner = pe_index(g, ox - FD_N, oy, oz) >= 0 && pe_index(g, ox + FD_N, oy, oz) >= 0 &&
                           pe_index(g, ox, oy - FD_N, oz) >= 0 && pe_index(g, ox, oy + FD_N, oz) >= 0 &&
                           pe_index(g, ox, oy, oz - FD_N) >= 0 && pe_index(g, ox, oy, oz + FD_N) >= 0;
        flag[q] = inner ? 0 : 1;
    }
}

// Sum of b^2 over PE, in fixed-order partial sums: grid (kScaleChunks,
// samples); chunk j of sample k covers q = j * 256 + t (mod stride).
constexpr int kScaleChunks = 64;
__global__ __launch_bounds__(256) void k_net_sumsq(NetPairArgs a, const int *pairs, int base, double *part)
{
    __shared__ double red[4];
    const int k = blockIdx.y;
    const int pair = pair_of(pairs, base, k);
    const ClassDev &g = a.cls[a.pair_gc[pair].w];
    const double *b = a.rhs + a.rhs_off[pair];
    double ss = 0.0;
    for (int q = blockIdx.x * 256 + threadIdx.x; q < g.n_pe; q += kScaleChunks * 256) ss += b[q] * b[q];
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
    __syncthreads();
    if (threadIdx.x == 0) part[k * kScaleChunks + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// scale[k] = RMS of b over PE for sample k (FP64), from the partial sums.
__global__ void k_net_scale(NetPairArgs a, const int *pairs, int base, int nb, const double *part, double *scale)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nb) return;
    const int pair = pair_of(pairs, base, k);
    const ClassDev &g = a.cls[a.pair_gc[pair].w];
    double tot = 0.0;
    for (int j = 0; j < kScaleChunks; ++j) tot += part[k * kScaleChunks + j];
    scale[k] = tot > 0.0 ? sqrt(tot / (double)g.n_pe) : 0.0;
}

// One thread per coarse cell: grid (ceil(D^3 / 256), samples).  Input
// channels, each a mean over the cell's f^3 fine offsets: 0 = b / s at PE
// points whose stencil stays in PE, 1 = b / s at PE points next to the
// boundary, 2 = fraction of the cell in PE; 3..15 zero.  Training target
// (tgt != NULL): mean of v / (s h^2) over the cell's points in ME (PE values
// from x, shell values from x + n_pe), weight 1 where the cell meets ME.
// The cell's points are walked row by row: f^2 (y, z) rows of f points.
__global__ __launch_bounds__(256) void k_net_cells(NetPairArgs a, const int *pairs, int base, int D, int f, bf16_t *in,
                                                   float2 *tgt, const double *scale)
{
    const int D3 = D * D * D;
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= D3) return;
    const int k = blockIdx.y;
    const int pair = pair_of(pairs, base, k);
    const int cls = a.pair_gc[pair].w;
    const ClassDev &g = a.cls[cls];
    const unsigned char *bnd = a.bnd[cls];
    const double *b = a.rhs + a.rhs_off[pair];
    const double *x = a.vout + a.out_off[pair];
    const double s = scale[k];
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    const double invx = s > 0.0 ? 1.0 / (s * a.h2) : 0.0;
    const int half = f * D / 2;
    const int cx = c % D, cy = (c / D) % D, cz = c / (D * D);
    const int x0 = -half + f * cx, y0 = -half + f * cy, z0 = -half + f * cz;
    double s_in = 0.0, s_bd = 0.0, s_x = 0.0;
    int n_pe = 0, n_me = 0;
    for (int r = 0; r < f * f; ++r) {
        const int oy = y0 + r % f, oz = z0 + r / f;
        const int pz = oz - g.pzlo, py = oy - g.pylo;
        if ((unsigned)pz < (unsigned)g.pnz && (unsigned)py < (unsigned)g.pny) {
            const int4 row = g.pe_rows[pz * g.pny + py];     // {base, xlo, xhi}
            const int lo = max(x0, row.y), hi = min(x0 + f - 1, row.z);
            for (int ox = lo; ox <= hi; ++ox) {
                const int q = row.x + ox - row.y;
                (bnd[q] ? s_bd : s_in) += b[q];
                ++n_pe;
            }
        }
        if (tgt) {
            const int mz = oz - g.mzlo, my = oy - g.mylo;
            if ((unsigned)mz < (unsigned)g.mnz && (unsigned)my < (unsigned)g.mny) {
                const int4 ra = g.me_rows[2 * (mz * g.mny + my)];       // {pe_base, plo, phi, sh_base}
                const int4 rb = g.me_rows[2 * (mz * g.mny + my) + 1];   // {mlo, mhi}
                const int lo = max(x0, rb.x), hi = min(x0 + f - 1, rb.y);
                for (int ox = lo; ox <= hi; ++ox) {
                    const long long idx = (ox >= ra.y && ox <= ra.z)
                                              ? (long long)ra.x + ox - ra.y
                                              : (long long)g.n_pe + ra.w + (ox < ra.y ? ox - rb.x : (ra.y - rb.x) + (ox - ra.z - 1));
                    s_x += x[idx];
                    ++n_me;
                }
            }
        }
    }
    const double invf3 = 1.0 / (double)(f * f * f);
    bf16_t *cell = in + ((long long)k * D3 + c) * 16;
    cell[0] = f2bf((float)(s_in * inv * invf3));
    cell[1] = f2bf((float)(s_bd * inv * invf3));
    cell[2] = f2bf((float)(n_pe * invf3));
#pragma unroll
    for (int ch = 3; ch < 16; ++ch) cell[ch] = 0;
    if (tgt) tgt[(long long)k * D3 + c] = n_me ? make_float2((float)(s_x * invx / n_me), 1.f) : make_float2(0.f, 0.f);
}

// One thread per PE point: grid (ceil(max n_pe / 256), samples).
// v(o) = s h^2 trilinear(out[.][0]) at PE point o (cell centres as nodes,
// clamped at the cube faces).  A non-finite value (a diverged or corrupt
// model) becomes 0, so CG always starts from a finite guess.
__global__ __launch_bounds__(256) void k_net_output(NetPairArgs a, int base, int D, int f, const float *out,
                                                    const double *scale)
{
    const int k = blockIdx.y;
    const int pair = base + k;
    const ClassDev &g = a.cls[a.pair_gc[pair].w];
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= g.n_pe) return;
    double *x = a.vout + a.out_off[pair];
    const double sc = scale[k] * a.h2;
    const float *op = out + (long long)k * D * D * D * 16;
    const float half = 0.5f * f * D, c0 = 0.5f * (f - 1), invf = 1.f / f;
    int ox, oy, oz;
    unpack_xyz(g.pe_xyz[q], ox, oy, oz);
    const float u[3] = {(ox + half - c0) * invf, (oy + half - c0) * invf, (oz + half - c0) * invf};
    int i0[3], i1[3];
    float t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float fl = floorf(u[d]);
        t[d] = u[d] - fl;
        const int lo = (int)fl;
        i0[d] = min(max(lo, 0), D - 1);
        i1[d] = min(max(lo + 1, 0), D - 1);
    }
    float v = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int xx = (j & 1) ? i1[0] : i0[0], yy = (j & 2) ? i1[1] : i0[1], zz = (j & 4) ? i1[2] : i0[2];
        const float wgt = ((j & 1) ? t[0] : 1.f - t[0]) * ((j & 2) ? t[1] : 1.f - t[1]) * ((j & 4) ? t[2] : 1.f - t[2]);
        v += wgt * op[((long long)(zz * D + yy) * D + xx) * 16];
    }
    const double val = sc * (double)v;
    x[q] = isfinite(val) ? val : 0.0;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

namespace {

constexpr int kLayers = 12;
const int kCin[kLayers] = {16, 16, 16, 32, 32, 64, 64, 64, 128, 96, 48, 16};
const int kCout[kLayers] = {16, 16, 32, 32, 64, 64, 64, 64, 64, 32, 16, 16};
constexpr int kInChannels = 3;   // real channels of the input layer

// Activation roles: channels and level (edge D >> level).
enum Role { IN, E1A, E1, P1, E2A, E2, P2, E3A, E3, P3, E4A, E4, U3, D3R, U2, D2R, U1, D1R, OUT, SK1, SK2, SK3, NROLE };
const int kRoleC[NROLE] = {16, 16, 16, 16, 32, 32, 32, 64, 64, 64, 64, 64, 128, 64, 96, 32, 48, 16, 16, 16, 32, 64};
const int kRoleL[NROLE] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 3, 3, 3, 2, 2, 1, 1, 0, 0, 0, 0, 1, 2};

inline unsigned grid_for(long long n) { return (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 1LL << 20)); }

constexpr char kMagic[8] = {'E', 'X', 'X', 'N', 'E', 'T', '0', '1'};

}  // namespace

struct ExxNet {
    int f = 2;
    struct Layer {
        int cin = 0, cout = 0;
        float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
        bf16_t *w16 = nullptr, *wt16 = nullptr;
    } L[kLayers];
    int step = 0;
    // buffers for `cap` samples of edge `capD` (grad only when training)
    int cap = 0, capD = 0;
    bool cap_grad = false;
    bf16_t *act[NROLE] = {}, *grad[NROLE] = {};
    float *out = nullptr, *acc = nullptr;
    float2 *tgt = nullptr;
    double *scale = nullptr, *part = nullptr;
    int *pairs = nullptr;
    int pairs_cap = 0;
    unsigned long long generation = 0;   // bumped whenever the buffers move
    hipEvent_t ev[2] = {};
};

unsigned long long net_generation(const ExxNet *net) { return net->generation; }

int net_coarsen(const ExxNet *net) { return net->f; }

int net_layer_dims(int l, int *cin, int *cout)
{
    if (l < 0 || l >= kLayers) return -1;
    *cin = kCin[l];
    *cout = kCout[l];
    return 0;
}

int net_edge(int f, int r_max)
{
    const int need = (2 * (r_max + 1) + f - 1) / f;
    return (need + 7) / 8 * 8;
}

size_t net_buffer_bytes(int batch, int D, bool training)
{
    const size_t v1 = (size_t)batch * D * D * D;
    size_t b = 0;
    for (int r = 0; r < NROLE; ++r) b += (v1 >> (3 * kRoleL[r])) * kRoleC[r] * sizeof(bf16_t) + 256;
    if (training) b *= 2;
    b += v1 * 16 * sizeof(float) + v1 * sizeof(float2) + batch * (sizeof(double) + sizeof(int)) + 1024;
    return b;
}

static void free_buffers(ExxNet *net)
{
    for (auto *arr : {net->act, net->grad})
        for (int r = 0; r < NROLE; ++r)
            if (arr[r]) { (void)hipFree(arr[r]); arr[r] = nullptr; }
    for (void *p : {(void *)net->out, (void *)net->tgt, (void *)net->scale, (void *)net->part, (void *)net->acc})
        if (p) (void)hipFree(p);
    net->part = nullptr;
    net->out = nullptr;
    net->tgt = nullptr;
    net->scale = nullptr;
    net->acc = nullptr;
    net->cap = net->capD = 0;
    net->cap_grad = false;
}

static hipError_t net_alloc(ExxNet *net, int batch, int D, bool training)
{
    if (batch <= net->cap && D == net->capD && (net->cap_grad || !training)) return hipSuccess;
    free_buffers(net);
    ++net->generation;
    const long long v1 = (long long)batch * D * D * D;
    hipError_t e;
    for (int r = 0; r < NROLE; ++r) {
        const size_t n = (size_t)(v1 >> (3 * kRoleL[r])) * kRoleC[r] * sizeof(bf16_t) + 256;
        if ((e = hipMalloc(&net->act[r], n)) != hipSuccess) return e;
        if (training && (e = hipMalloc(&net->grad[r], n)) != hipSuccess) return e;
    }
    if ((e = hipMalloc(&net->out, (size_t)v1 * 16 * sizeof(float))) != hipSuccess) return e;
    if ((e = hipMalloc(&net->tgt, (size_t)v1 * sizeof(float2))) != hipSuccess) return e;
    if ((e = hipMalloc(&net->scale, (size_t)batch * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc(&net->part, (size_t)batch * kScaleChunks * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc(&net->acc, 2 * sizeof(float))) != hipSuccess) return e;
    net->cap = batch;
    net->capD = D;
    net->cap_grad = training;
    return hipSuccess;
}

static void refresh_bf16(ExxNet *net, hipStream_t s)
{
    for (auto &ly : net->L) {
        const long long n = 27LL * ly.cin * ly.cout;
        hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, s, ly.w, ly.m, ly.v, ly.g, ly.w16, ly.wt16, ly.cin,
                           ly.cout, 0.f, 0.9f, 0.999f, 1.f, 1.f, 1.f);
    }
}

ExxNet *net_create(int f, unsigned long long seed, hipError_t *err)
{
    ExxNet *net = new ExxNet();
    net->f = f;
    std::mt19937_64 rng(seed);
    *err = hipSuccess;
    for (int l = 0; l < kLayers; ++l) {
        auto &ly = net->L[l];
        ly.cin = kCin[l];
        ly.cout = kCout[l];
        const size_t n = 27ULL * ly.cin * ly.cout;
        std::vector<float> w(n), zero(n, 0.f);
        // He initialization over the real fan-in; the input layer's padding
        // channels carry zero weights
        const int real_in = l == 0 ? kInChannels : ly.cin;
        std::normal_distribution<float> nd(0.f, std::sqrt(2.f / (27.f * real_in)));
        for (size_t t = 0; t < n; ++t) w[t] = (l == 0 && (int)(t % ly.cin) >= kInChannels) ? 0.f : nd(rng);
        for (float **p : {&ly.w, &ly.m, &ly.v, &ly.g})
            if ((*err = hipMalloc(p, n * sizeof(float))) != hipSuccess) return net;
        // packed copies: 14 tap pairs per 16-channel chunk, the 28th tap zero
        const size_t n16 = 28ULL * ly.cin * ly.cout * sizeof(bf16_t);
        for (bf16_t **p : {&ly.w16, &ly.wt16}) {
            if ((*err = hipMalloc(p, n16)) != hipSuccess) return net;
            if ((*err = hipMemset(*p, 0, n16)) != hipSuccess) return net;
        }
        if ((*err = hipMemcpy(ly.w, w.data(), n * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) return net;
        for (float *p : {ly.m, ly.v, ly.g})
            if ((*err = hipMemcpy(p, zero.data(), n * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) return net;
    }
    for (auto &e : net->ev)
        if ((*err = hipEventCreate(&e)) != hipSuccess) return net;
    refresh_bf16(net, 0);
    *err = hipDeviceSynchronize();
    return net;
}

void net_destroy(ExxNet *net)
{
    if (!net) return;
    for (auto &ly : net->L)
        for (void *p : {(void *)ly.w, (void *)ly.m, (void *)ly.v, (void *)ly.g, (void *)ly.w16, (void *)ly.wt16})
            if (p) (void)hipFree(p);
    free_buffers(net);
    if (net->pairs) (void)hipFree(net->pairs);
    for (auto &e : net->ev)
        if (e) (void)hipEventDestroy(e);
    delete net;
}

static void conv(ExxNet *net, int l, const bf16_t *X, void *Y, int N, int D, bool relu, bool f32, bool transposed,
                 hipStream_t s)
{
    const auto &ly = net->L[l];
    const int cin = transposed ? ly.cout : ly.cin, cout = transposed ? ly.cin : ly.cout;
    const bf16_t *W = transposed ? ly.wt16 : ly.w16;
    // M tiles per wave (= tile depth): eight MFMA accumulators per wave; cubes
    // smaller than a tile take the flat kernel
    switch (cout / 16 * 4 + (f32 ? 2 : 0) + (relu ? 1 : 0)) {
#define EXX_CONV_CASE(NCO, RELU, F32)                                                                       \
    case NCO * 4 + (F32 ? 2 : 0) + (RELU ? 1 : 0): {                                                        \
        constexpr int MV = NCO == 1 ? 8 : NCO == 2 ? 4 : NCO <= 4 ? 2 : 1;                                  \
        if (D >= CT_XY) {                                                                                   \
            const dim3 grid((unsigned)conv_tiles(N, D, MV));                                                \
            hipLaunchKernelGGL((k_conv3<MV, NCO, RELU, F32>), grid, dim3(256), 0, s, X, W, Y, N, D, cin);    \
        } else {                                                                                            \
            const long long nvox = (long long)N * D * D * D;                                                \
            const dim3 grid((unsigned)((nvox + 15) / 16), (unsigned)NCO);                                   \
            hipLaunchKernelGGL((k_conv3_small<RELU, F32>), grid, dim3(256), 0, s, X, W, Y, N, D, cin, cout); \
        }                                                                                                   \
        break;                                                                                              \
    }
#define EXX_CONV_CASES(NCO) EXX_CONV_CASE(NCO, false, false) EXX_CONV_CASE(NCO, true, false) EXX_CONV_CASE(NCO, false, true)
        // every channel count of the layers and of their transposes (16 .. 128)
        EXX_CONV_CASES(1) EXX_CONV_CASES(2) EXX_CONV_CASES(3) EXX_CONV_CASES(4) EXX_CONV_CASES(6) EXX_CONV_CASES(8)
#undef EXX_CONV_CASES
#undef EXX_CONV_CASE
        default: break;
    }
}

static void wgrad(const ExxNet::Layer &ly, const bf16_t *X, const bf16_t *dY, float *dW, int N, int D, hipStream_t s)
{
    const long long nvox = (long long)N * D * D * D;
    const int chunk = 2048;   // 16 passes of the 4 waves over 128 voxels
    const dim3 grid((unsigned)((nvox + chunk - 1) / chunk), 27u, (unsigned)((ly.cout / 16) * (ly.cin / 16)));
    hipLaunchKernelGGL(k_conv3_wgrad, grid, dim3(256), 0, s, X, dY, dW, N, D, ly.cin, ly.cout, chunk);
}

static void pool(const bf16_t *X, bf16_t *Y, int N, int D, int C, hipStream_t s)
{
    const long long n = (long long)N * (D / 2) * (D / 2) * (D / 2) * C;
    hipLaunchKernelGGL(k_pool2, dim3(grid_for(n)), dim3(256), 0, s, X, Y, N, D, C);
}
static void pool_bwd(const bf16_t *dY, bf16_t *dX, int N, int D, int C, hipStream_t s)
{
    const long long n = (long long)N * D * D * D * C;
    hipLaunchKernelGGL(k_pool2_bwd, dim3(grid_for(n)), dim3(256), 0, s, dY, dX, N, D, C);
}
static void upcat(const bf16_t *L, const bf16_t *S, bf16_t *Y, int N, int D, int C1, int C2, hipStream_t s)
{
    const long long n = (long long)N * D * D * D * (C1 + C2);
    hipLaunchKernelGGL(k_upcat, dim3(grid_for(n)), dim3(256), 0, s, L, S, Y, N, D, C1, C2);
}
static void upcat_bwd(const bf16_t *dY, bf16_t *dL, bf16_t *dS, int N, int D, int C1, int C2, hipStream_t s)
{
    const long long n = (long long)N * D * D * D * C2 + (long long)N * (D / 2) * (D / 2) * (D / 2) * C1;
    hipLaunchKernelGGL(k_upcat_bwd, dim3(grid_for(n)), dim3(256), 0, s, dY, dL, dS, N, D, C1, C2);
}
static void relu_bwd(bf16_t *dX, const bf16_t *Y, const bf16_t *dA, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_relu_bwd, dim3(grid_for(n)), dim3(256), 0, s, dX, Y, dA, n);
}

static void forward(ExxNet *net, int N, int D, hipStream_t s)
{
    bf16_t **a = net->act;
    const int D2 = D / 2, D4 = D / 4, D8 = D / 8;
    conv(net, 0, a[IN], a[E1A], N, D, true, false, false, s);
    conv(net, 1, a[E1A], a[E1], N, D, true, false, false, s);
    pool(a[E1], a[P1], N, D, 16, s);
    conv(net, 2, a[P1], a[E2A], N, D2, true, false, false, s);
    conv(net, 3, a[E2A], a[E2], N, D2, true, false, false, s);
    pool(a[E2], a[P2], N, D2, 32, s);
    conv(net, 4, a[P2], a[E3A], N, D4, true, false, false, s);
    conv(net, 5, a[E3A], a[E3], N, D4, true, false, false, s);
    pool(a[E3], a[P3], N, D4, 64, s);
    conv(net, 6, a[P3], a[E4A], N, D8, true, false, false, s);
    conv(net, 7, a[E4A], a[E4], N, D8, true, false, false, s);
    upcat(a[E4], a[E3], a[U3], N, D4, 64, 64, s);
    conv(net, 8, a[U3], a[D3R], N, D4, true, false, false, s);
    upcat(a[D3R], a[E2], a[U2], N, D2, 64, 32, s);
    conv(net, 9, a[U2], a[D2R], N, D2, true, false, false, s);
    upcat(a[D2R], a[E1], a[U1], N, D, 32, 16, s);
    conv(net, 10, a[U1], a[D1R], N, D, true, false, false, s);
    conv(net, 11, a[D1R], net->out, N, D, false, true, false, s);
}

// Gradients of every layer's weights given dOut in grad[OUT].
static void backward(ExxNet *net, int N, int D, hipStream_t s)
{
    bf16_t **a = net->act, **g = net->grad;
    const int D2 = D / 2, D4 = D / 4, D8 = D / 8;
    const long long v1 = (long long)N * D * D * D, v2 = v1 / 8, v4 = v2 / 8, v8 = v4 / 8;
    auto W = [&](int l, const bf16_t *x, const bf16_t *dy, int d) { wgrad(net->L[l], x, dy, net->L[l].g, N, d, s); };
    auto T = [&](int l, const bf16_t *dy, bf16_t *dx, int d) { conv(net, l, dy, dx, N, d, false, false, true, s); };
    W(11, a[D1R], g[OUT], D);
    T(11, g[OUT], g[D1R], D);
    relu_bwd(g[D1R], a[D1R], nullptr, v1 * 16, s);
    W(10, a[U1], g[D1R], D);
    T(10, g[D1R], g[U1], D);
    upcat_bwd(g[U1], g[D2R], g[SK1], N, D, 32, 16, s);
    relu_bwd(g[D2R], a[D2R], nullptr, v2 * 32, s);
    W(9, a[U2], g[D2R], D2);
    T(9, g[D2R], g[U2], D2);
    upcat_bwd(g[U2], g[D3R], g[SK2], N, D2, 64, 32, s);
    relu_bwd(g[D3R], a[D3R], nullptr, v4 * 64, s);
    W(8, a[U3], g[D3R], D4);
    T(8, g[D3R], g[U3], D4);
    upcat_bwd(g[U3], g[E4], g[SK3], N, D4, 64, 64, s);
    relu_bwd(g[E4], a[E4], nullptr, v8 * 64, s);
    W(7, a[E4A], g[E4], D8);
    T(7, g[E4], g[E4A], D8);
    relu_bwd(g[E4A], a[E4A], nullptr, v8 * 64, s);
    W(6, a[P3], g[E4A], D8);
    T(6, g[E4A], g[P3], D8);
    pool_bwd(g[P3], g[E3], N, D4, 64, s);
    relu_bwd(g[E3], a[E3], g[SK3], v4 * 64, s);        // e3 feeds the pool and the skip
    W(5, a[E3A], g[E3], D4);
    T(5, g[E3], g[E3A], D4);
    relu_bwd(g[E3A], a[E3A], nullptr, v4 * 64, s);
    W(4, a[P2], g[E3A], D4);
    T(4, g[E3A], g[P2], D4);
    pool_bwd(g[P2], g[E2], N, D2, 32, s);
    relu_bwd(g[E2], a[E2], g[SK2], v2 * 32, s);
    W(3, a[E2A], g[E2], D2);
    T(3, g[E2], g[E2A], D2);
    relu_bwd(g[E2A], a[E2A], nullptr, v2 * 32, s);
    W(2, a[P1], g[E2A], D2);
    T(2, g[E2A], g[P1], D2);
    pool_bwd(g[P1], g[E1], N, D, 16, s);
    relu_bwd(g[E1], a[E1], g[SK1], v1 * 16, s);
    W(1, a[E1A], g[E1], D);
    T(1, g[E1], g[E1A], D);
    relu_bwd(g[E1A], a[E1A], nullptr, v1 * 16, s);
    W(0, a[IN], g[E1A], D);
}

static void net_input(ExxNet *net, const NetPairArgs &a, const int *pairs, int base, int nb, int D, bool target,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_net_sumsq, dim3((unsigned)kScaleChunks, (unsigned)nb), dim3(256), 0, s, a, pairs, base, net->part);
    hipLaunchKernelGGL(k_net_scale, dim3((unsigned)((nb + 63) / 64)), dim3(64), 0, s, a, pairs, base, nb,
                       (const double *)net->part, net->scale);
    const dim3 grid((unsigned)((D * D * D + 255) / 256), (unsigned)nb);
    hipLaunchKernelGGL(k_net_cells, grid, dim3(256), 0, s, a, pairs, base, D, net->f, net->act[IN],
                       target ? net->tgt : (float2 *)nullptr, (const double *)net->scale);
}

hipError_t net_boundary_flags(const ClassDev &g, unsigned char *flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_pe_boundary, dim3(grid_for(g.n_pe)), dim3(256), 0, s, g, flag);
    return hipGetLastError();
}

static int infer_batch(int D)
{
    // about 1 GiB of activations
    const size_t per = net_buffer_bytes(1, D, false);
    return (int)std::max<size_t>(1, std::min<size_t>(64, ((size_t)1 << 30) / per));
}

hipError_t net_reserve(ExxNet *net, int n, int D)
{
    const int B = std::min(infer_batch(D), std::max(n, 1));
    return net_alloc(net, std::max(B, net->cap), D, net->cap_grad);
}

hipError_t net_infer(ExxNet *net, const NetPairArgs &a, int n, int D, double *ms, hipStream_t s)
{
    const int B = std::min(infer_batch(D), std::max(n, 1));
    hipError_t e = net_alloc(net, std::max(B, net->cap), D, net->cap_grad);
    if (e != hipSuccess) return e;
    if (ms && (e = hipEventRecord(net->ev[0], s)) != hipSuccess) return e;
    for (int b0 = 0; b0 < n; b0 += B) {
        const int nb = std::min(B, n - b0);
        const int base = a.wave_begin + b0;
        net_input(net, a, nullptr, base, nb, D, false, s);
        forward(net, nb, D, s);
        int npe = 0;
        for (int k = 0; k < KMAX; ++k) npe = std::max(npe, a.cls[k].n_pe);
        hipLaunchKernelGGL(k_net_output, dim3((unsigned)((npe + 255) / 256), (unsigned)nb), dim3(256), 0, s, a, base, D,
                           net->f, net->out, net->scale);
    }
    if (ms) {
        if ((e = hipEventRecord(net->ev[1], s)) != hipSuccess) return e;
        if ((e = hipEventSynchronize(net->ev[1])) != hipSuccess) return e;
        float t = 0.f;
        if ((e = hipEventElapsedTime(&t, net->ev[0], net->ev[1])) != hipSuccess) return e;
        *ms = t;
    }
    return hipGetLastError();
}

hipError_t net_train(ExxNet *net, const NetPairArgs &a, const int *pairs, int n_pairs, int D, int epochs, int batch,
                     float lr, unsigned long long seed, double *loss, hipStream_t s)
{
    hipError_t e = net_alloc(net, batch, D, true);
    if (e != hipSuccess) return e;
    if (net->pairs_cap < n_pairs) {
        if (net->pairs) (void)hipFree(net->pairs);
        net->pairs = nullptr;
        if ((e = hipMalloc(&net->pairs, (size_t)n_pairs * sizeof(int))) != hipSuccess) return e;
        net->pairs_cap = n_pairs;
    }
    std::vector<int> order(pairs, pairs + n_pairs);
    std::mt19937_64 rng(seed);
    const float b1 = 0.9f, b2 = 0.999f;
    double last = 0.0;
    std::vector<float> accs;
    if (epochs == 0) {
        // evaluation only: the masked squared error over every pair, no update
        if ((e = hipMemcpyAsync(net->pairs, order.data(), (size_t)n_pairs * sizeof(int), hipMemcpyHostToDevice, s)) !=
            hipSuccess)
            return e;
        const int nbat = (n_pairs + batch - 1) / batch;
        accs.assign((size_t)2 * nbat, 0.f);
        for (int bi = 0; bi < nbat; ++bi) {
            const int nb = std::min(batch, n_pairs - bi * batch);
            net_input(net, a, net->pairs + bi * batch, 0, nb, D, true, s);
            forward(net, nb, D, s);
            const long long nvox = (long long)nb * D * D * D;
            if ((e = hipMemsetAsync(net->acc, 0, 2 * sizeof(float), s)) != hipSuccess) return e;
            hipLaunchKernelGGL(k_loss, dim3(grid_for(nvox)), dim3(256), 0, s, net->out, net->tgt, net->grad[OUT], net->acc,
                               nvox);
            if ((e = hipMemcpyAsync(&accs[2 * bi], net->acc, 2 * sizeof(float), hipMemcpyDeviceToHost, s)) != hipSuccess)
                return e;
        }
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        double num = 0.0, den = 0.0;
        for (int bi = 0; bi < nbat; ++bi) {
            num += accs[2 * bi];
            den += accs[2 * bi + 1];
        }
        *loss = den > 0.0 ? num / den : 0.0;
        return hipGetLastError();
    }
    for (int ep = 0; ep < epochs; ++ep) {
        std::shuffle(order.begin(), order.end(), rng);
        if ((e = hipMemcpyAsync(net->pairs, order.data(), (size_t)n_pairs * sizeof(int), hipMemcpyHostToDevice, s)) !=
            hipSuccess)
            return e;
        const int nbat = n_pairs / batch;
        accs.assign((size_t)2 * nbat, 0.f);
        for (int bi = 0; bi < nbat; ++bi) {
            net_input(net, a, net->pairs + bi * batch, 0, batch, D, true, s);
            forward(net, batch, D, s);
            const long long nvox = (long long)batch * D * D * D;
            if ((e = hipMemsetAsync(net->acc, 0, 2 * sizeof(float), s)) != hipSuccess) return e;
            hipLaunchKernelGGL(k_loss, dim3(grid_for(nvox)), dim3(256), 0, s, net->out, net->tgt, net->grad[OUT], net->acc,
                               nvox);
            backward(net, batch, D, s);
            ++net->step;
            const float c1 = 1.f - std::pow(b1, (float)net->step), c2 = 1.f - std::pow(b2, (float)net->step);
            for (auto &ly : net->L) {
                const long long n = 27LL * ly.cin * ly.cout;
                hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, s, ly.w, ly.m, ly.v, ly.g, ly.w16, ly.wt16,
                                   ly.cin, ly.cout, lr, b1, b2, c1, c2, 1e-8f);
            }
            if ((e = hipMemcpyAsync(&accs[2 * bi], net->acc, 2 * sizeof(float), hipMemcpyDeviceToHost, s)) != hipSuccess)
                return e;
        }
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        double sum = 0.0;
        for (int bi = 0; bi < nbat; ++bi) sum += accs[2 * bi + 1] > 0.f ? accs[2 * bi] / accs[2 * bi + 1] : 0.0;
        last = nbat ? sum / nbat : 0.0;
    }
    *loss = last;
    return hipGetLastError();
}

// Blob: 8-byte magic, int32 coarsening factor, int32 layer count, then each
// layer's FP32 weights [27][Cout][Cin] in layer order.
size_t net_model_bytes()
{
    size_t n = 16;
    for (int l = 0; l < kLayers; ++l) n += 27ULL * kCin[l] * kCout[l] * sizeof(float);
    return n;
}

hipError_t net_save(ExxNet *net, void *host)
{
    char *p = static_cast<char *>(host);
    std::memcpy(p, kMagic, 8);
    const int32_t hdr[2] = {net->f, kLayers};
    std::memcpy(p + 8, hdr, 8);
    p += 16;
    for (auto &ly : net->L) {
        const size_t n = 27ULL * ly.cin * ly.cout * sizeof(float);
        hipError_t e = hipMemcpy(p, ly.w, n, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return e;
        p += n;
    }
    return hipSuccess;
}

int net_blob_coarsen(const void *host, size_t bytes)
{
    if (!host || bytes != net_model_bytes() || std::memcmp(host, kMagic, 8) != 0) return -1;
    int32_t hdr[2];
    std::memcpy(hdr, static_cast<const char *>(host) + 8, 8);
    if ((hdr[0] != 2 && hdr[0] != 4 && hdr[0] != 8) || hdr[1] != kLayers) return -1;
    return hdr[0];
}

int net_load(ExxNet *net, const void *host, size_t bytes, hipError_t *err)
{
    *err = hipSuccess;
    const int f = net_blob_coarsen(host, bytes);
    if (f < 0) return -1;
    net->f = f;
    const char *p = static_cast<const char *>(host) + 16;
    for (auto &ly : net->L) {
        const size_t n = 27ULL * ly.cin * ly.cout;
        if ((*err = hipMemcpy(ly.w, p, n * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) return -2;
        p += n * sizeof(float);
    }
    refresh_bf16(net, 0);
    *err = hipDeviceSynchronize();
    return *err == hipSuccess ? 0 : -2;
}

hipError_t net_conv_test(ExxNet *net, int l, int transposed, const void *x, float *y, int N, int D, hipStream_t s)
{
    conv(net, l, static_cast<const bf16_t *>(x), y, N, D, false, true, transposed != 0, s);
    return hipGetLastError();
}

hipError_t net_wgrad_test(ExxNet *net, int l, const void *x, const void *dy, float *dw, int N, int D, hipStream_t s)
{
    const auto &ly = net->L[l];
    hipError_t e = hipMemsetAsync(dw, 0, 27ULL * ly.cin * ly.cout * sizeof(float), s);
    if (e != hipSuccess) return e;
    wgrad(ly, static_cast<const bf16_t *>(x), static_cast<const bf16_t *>(dy), dw, N, D, s);
    return hipGetLastError();
}

}  // namespace exx
