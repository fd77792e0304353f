// exx_stream.hip -- measured HBM streaming rates of plain kernels, the
// practical ceiling that the pair CG's bandwidth is compared against beside
// the nominal 8 TB/s.
//
// Each kind moves whole arrays once per launch in 16-byte (dwordx4)
// accesses from a grid-stride loop with several accesses of each array in
// flight per thread:
//   0 read   s += a[i] + b[i]                    (2 arrays read)
//   1 copy   c[i] = a[i]                         (1 read, 1 write)
//   2 triad  c[i] = a[i] + s b[i]                (2 read, 1 write: the CG's
//                                                 read:write mix of about 2:1)
//   3 cg     c[i] = a[i] + s b[i], d[i] = b[i] - s a[i] + e[i]
//                                                (3 read, 2 write per pair of
//                                                 outputs, the direction and
//                                                 update passes together)
// The rate of a kind is the best over work-group counts, in-flight depths
// and plain or non-temporal accesses.
#include "exx.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>

namespace {

constexpr int SB = 256;   // threads per work-group

template <bool NT>
__device__ __forceinline__ double2 ld(const double2 *p)
{
    if constexpr (NT) {
        double2 v;
        v.x = __builtin_nontemporal_load(&p->x);
        v.y = __builtin_nontemporal_load(&p->y);
        return v;
    } else {
        return *p;
    }
}

template <bool NT>
__device__ __forceinline__ void st(double2 *p, double2 v)
{
    if constexpr (NT) {
        __builtin_nontemporal_store(v.x, &p->x);
        __builtin_nontemporal_store(v.y, &p->y);
    } else {
        *p = v;
    }
}

// n is a multiple of SB * U (the host rounds the arrays down to it).
template <int KIND, int U, bool NT>
__global__ __launch_bounds__(SB) void k_stream(const double2 *__restrict__ a, const double2 *__restrict__ b,
                                              const double2 *__restrict__ e, double2 *__restrict__ c,
                                              double2 *__restrict__ d, double s, long long n, double *sink)
{
    const long long stride = (long long)gridDim.x * SB * U;
    double acc = 0.0;
    for (long long base = (long long)blockIdx.x * SB * U + threadIdx.x; base < n; base += stride) {
        double2 va[U], vb[U], ve[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = base + (long long)u * SB;
            va[u] = ld<NT>(a + i);
            if constexpr (KIND != 1) vb[u] = ld<NT>(b + i);
            if constexpr (KIND == 3) ve[u] = ld<NT>(e + i);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = base + (long long)u * SB;
            if constexpr (KIND == 0) {
                acc += va[u].x + va[u].y + vb[u].x + vb[u].y;
            } else if constexpr (KIND == 1) {
                st<NT>(c + i, va[u]);
            } else {
                st<NT>(c + i, make_double2(va[u].x + s * vb[u].x, va[u].y + s * vb[u].y));
                if constexpr (KIND == 3)
                    st<NT>(d + i, make_double2(vb[u].x - s * va[u].x + ve[u].x, vb[u].y - s * va[u].y + ve[u].y));
            }
        }
    }
    // the read kind's sum goes to memory only if it is the impossible value
    // -1 (keeps the loads live without adding write traffic)
    if (KIND == 0 && acc == -1.0) sink[0] = acc;
}

template <int KIND, int U, bool NT>
hipError_t launch(int grid, const double2 *a, const double2 *b, const double2 *e, double2 *c, double2 *d, long long n,
                  double *sink, hipStream_t s)
{
    hipLaunchKernelGGL((k_stream<KIND, U, NT>), dim3(grid), dim3(SB), 0, s, a, b, e, c, d, 1e-3, n, sink);
    return hipGetLastError();
}

// Bytes one launch of a kind moves per element (a double2 of every array).
int bytes_per_elem(int kind) { return kind == 0 ? 32 : kind == 1 ? 32 : kind == 2 ? 48 : 80; }

}  // namespace

extern "C" exx_status exx_stream_rates(int device, int64_t bytes_per_array, int32_t reps, double *gbs,
                                       char *detail, int32_t detail_len)
{
    if (!gbs || bytes_per_array < (1 << 20) || reps < 1) return EXX_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return EXX_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return EXX_EDEVICE;
    const int n_cu = prop.multiProcessorCount;
    constexpr int kUMax = 4;
    const long long n = bytes_per_array / 16 / (SB * kUMax) * (SB * kUMax);
    double2 *buf[5] = {};
    double *sink = nullptr;
    hipEvent_t ev[2] = {};
    exx_status st = EXX_OK;
    for (auto &p : buf)
        if (hipMalloc(&p, (size_t)n * 16) != hipSuccess) st = EXX_ENOMEM;
    if (st == EXX_OK && hipMalloc(&sink, 8) != hipSuccess) st = EXX_ENOMEM;
    if (st == EXX_OK && (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess))
        st = EXX_EDEVICE;
    for (int k = 0; st == EXX_OK && k < 5; ++k)
        if (hipMemset(buf[k], 0, (size_t)n * 16) != hipSuccess) st = EXX_EDEVICE;
    int best_cfg[4] = {0, 0, 0, 0};
    for (int kind = 0; kind < 4 && st == EXX_OK; ++kind) {
        double best = 0.0;
        for (int wg_per_cu : {4, 8, 16}) {
            const int grid = wg_per_cu * n_cu;
            for (int cfg = 0; cfg < 6 && st == EXX_OK; ++cfg) {
                const int u = cfg % 3 == 0 ? 1 : cfg % 3 == 1 ? 2 : 4;
                const bool nt = cfg >= 3;
                auto go = [&]() -> hipError_t {
#define EXX_S(K)                                                                                              \
    if (kind == K) {                                                                                          \
        if (nt) return u == 1 ? launch<K, 1, true>(grid, buf[0], buf[1], buf[2], buf[3], buf[4], n, sink, 0)  \
                       : u == 2 ? launch<K, 2, true>(grid, buf[0], buf[1], buf[2], buf[3], buf[4], n, sink, 0) \
                                : launch<K, 4, true>(grid, buf[0], buf[1], buf[2], buf[3], buf[4], n, sink, 0); \
        return u == 1 ? launch<K, 1, false>(grid, buf[0], buf[1], buf[2], buf[3], buf[4], n, sink, 0)          \
               : u == 2 ? launch<K, 2, false>(grid, buf[0], buf[1], buf[2], buf[3], buf[4], n, sink, 0)        \
                        : launch<K, 4, false>(grid, buf[0], buf[1], buf[2], buf[3], buf[4], n, sink, 0);       \
    }
                    EXX_S(0) EXX_S(1) EXX_S(2) EXX_S(3)
#undef EXX_S
                    return hipErrorInvalidValue;
                };
                if (go() != hipSuccess || hipDeviceSynchronize() != hipSuccess) { st = EXX_EDEVICE; break; }
                for (int r = 0; r < reps; ++r) {
                    float ms = 0.f;
                    if (hipEventRecord(ev[0], 0) != hipSuccess || go() != hipSuccess ||
                        hipEventRecord(ev[1], 0) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
                        hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) {
                        st = EXX_EDEVICE;
                        break;
                    }
                    const double rate = (double)n * bytes_per_elem(kind) / (ms * 1e-3) / 1e9;
                    if (rate > best) {
                        best = rate;
                        best_cfg[kind] = wg_per_cu * 100 + u * 10 + (nt ? 1 : 0);
                    }
                }
            }
        }
        gbs[kind] = best;
    }
    if (detail && detail_len > 0)
        snprintf(detail, (size_t)detail_len,
                 "%lld B per array; best (work-groups per CU, accesses in flight, non-temporal): "
                 "read %d/%d/%d copy %d/%d/%d triad %d/%d/%d cg %d/%d/%d",
                 n * 16, best_cfg[0] / 100, best_cfg[0] / 10 % 10, best_cfg[0] % 10, best_cfg[1] / 100,
                 best_cfg[1] / 10 % 10, best_cfg[1] % 10, best_cfg[2] / 100, best_cfg[2] / 10 % 10, best_cfg[2] % 10,
                 best_cfg[3] / 100, best_cfg[3] / 10 % 10, best_cfg[3] % 10);
    for (auto &p : buf)
        if (p) (void)hipFree(p);
    if (sink) (void)hipFree(sink);
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    (void)hipGetLastError();
    return st;
}
