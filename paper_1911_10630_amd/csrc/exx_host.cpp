// exx_host.cpp -- host side of the MI355X pair-Poisson exact-exchange library:
// parameter validation, proto-subdomain tables (Alg. 2), pair list and pair
// origins (Sec. III.C Steps II-III), device memory, and the C ABI of exx.h.
#include "exx.h"
#include "exx_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

using namespace exx;

namespace {

// Central-difference weights of the second derivative for n = 3 (Eq. d2_1).
constexpr double kFD[4] = {-49.0 / 18.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0};

// messages live in fixed buffers so that reporting a failure never allocates
char g_setup_error[512] = "no error";

// Device address of the fixed CG scratch array on each device, taken once per
// device (with that device current) by the first exx_setup on it.
constexpr int kMaxDevices = 64;
void *g_static_scratch[kMaxDevices] = {};
std::mutex g_static_mutex;

hipError_t static_scratch_for(int device, void **ptr)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_static_mutex);
    if (!g_static_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = static_scratch_address(&p);
        if (e != hipSuccess) return e;
        g_static_scratch[device] = p;
    }
    *ptr = g_static_scratch[device];
    return hipSuccess;
}

// Fortran NINT: nearest integer, halves away from zero.
long nint_away(double v) { return (long)(v >= 0.0 ? std::floor(v + 0.5) : -std::floor(-v + 0.5)); }
int mod_pos(long a, int n) { long r = a % n; return (int)(r < 0 ? r + n : r); }

struct HostClass {
    double r_pe = 0, r_me = 0;
    int n_pe = 0, n_sh = 0;
    int pxlo = 0, pxhi = -1, pylo = 0, pyhi = -1, pzlo = 0, pzhi = -1;
    int mxlo = 0, mxhi = -1, mylo = 0, myhi = -1, mzlo = 0, mzhi = -1;
    std::vector<int4> pe_rows, me_rows;
    std::vector<int> pe_xyz, sh_xyz, cols;
    std::vector<int> colz, pe_off;
    std::vector<int> bands, bands32;   // [n][12] for the selected CG variant
    std::vector<int> bnd_q, bnd_ptr, bnd_ent;   // PE-to-shell stencil coupling (CSR)
    int plane_rows = 0, plane_rows32 = 0;
    int4 *d_pe_rows = nullptr, *d_me_rows = nullptr;
    int *d_pe_xyz = nullptr, *d_sh_xyz = nullptr, *d_cols = nullptr, *d_bands = nullptr;
    int *d_colz = nullptr, *d_pe_off = nullptr, *d_bands32 = nullptr;
    int *d_bnd_q = nullptr, *d_bnd_ptr = nullptr, *d_bnd_ent = nullptr;
    // multigrid coarse levels: dims and masks (host), device masks, offsets
    int mg_levels = 0;
    int mg_n[MG_MAX][3] = {};
    std::vector<unsigned char> mg_mask[MG_MAX];
    unsigned char *d_mg_mask[MG_MAX] = {};
    long long mg_off[MG_MAX] = {};
    long long mg_doubles = 0;   // f, e, t of every level, the dense box and its sink
    long long mg_dense_off = 0;
    int64_t mg_cells_bytes = 0; // algorithmic bytes of one V-cycle (FP64 coarse values)
    int64_t mg_cells_bytes32 = 0; // the same with FP32 coarse values
};

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
};

}  // namespace

struct exx_ctx {
    exx_params prm{};
    int device = 0;
    int n_cu = 0;
    double h[3] = {0, 0, 0};
    int c0[3] = {0, 0, 0};
    HostClass cls[KMAX];
    int n_cls = 2;            // classes in use (self / non-self unless params.n_classes >= 2)
    int64_t class_capped = 0; // pairs of the list whose domain the largest class does not cover
    char err[512] = "no error";
    int state = 0;  // 1 set up, 2 pairs built, 3 solved

    // pairs
    int n_orb = 0;
    int64_t n_pairs = 0, n_self = 0;
    std::vector<int2> ij;
    std::vector<int4> gc;
    std::vector<long long> out_off;
    std::vector<long long> rhs_off;   // per pair: offset of its b in rhs (relative to its wave)
    std::vector<int> orb_ptr, orb_pairs;
    long long vout_n = 0;

    DevBuf<int2> d_ij;
    DevBuf<int4> d_gc;
    DevBuf<long long> d_off, d_rhs_off;
    std::vector<int> queue;     // CG queue order per wave (empty: pair order)
    DevBuf<int> d_queue;
    DevBuf<int> d_orb_ptr, d_orb_pairs;
    // pair-list construction
    DevBuf<double> d_pC;
    DevBuf<int> d_cell_of, d_cell_start, d_cell_items, d_pcount;
    DevBuf<long long> d_pstart;
    DevBuf<int2> d_pij;
    DevBuf<int4> d_pgc;
    std::vector<double> centers;  // [n_orb][3] of the current pair list
    std::vector<int> owner;     // Alg. 1 owner per pair (filled on request)
    int owner_sweeps = 0;
    DevBuf<double> d_vout, d_q, d_e, d_relres, d_scratch, d_E, d_rhs, d_rho_keep;
    DevBuf<int> d_iters, d_outer, d_conv, d_counter;
    DevBuf<unsigned long long> d_clock;   // per wave: first start, last end of its CG launch
    int clock_khz = 0;                    // device wall-clock rate
    DevBuf<float> d_scratch32;
    DevBuf<double> d_mg_scratch;

    // orbital boxes
    int box[3] = {0, 0, 0};
    long long box_vol = 0;
    std::vector<int4> box_org;
    DevBuf<int4> d_box_org;
    DevBuf<double> d_dacc;   // FP64 partial sums of D across waves

    // PE potentials of earlier steps (most recent first), keyed by (i, j)
    struct Hist {
        bool valid = false;
        std::unordered_map<long long, int> index;
        std::vector<int4> gc;
        std::vector<long long> off;
        DevBuf<float> v;
    } hist[3], hist_next;
    DevBuf<PairGuess> d_guess;
    DevBuf<long long> d_hist_off;
    int guess_pairs = 0;     // pairs of the last solve that had a history
    // learned guess
    ExxNet *net = nullptr;
    int net_D = 0;           // coarse cube edge for this context's classes
    DevBuf<unsigned char> d_bnd[KMAX];   // per class: PE points whose stencil leaves PE
    double guess_ms = 0.0;   // last solve: guess kernels or net inference of wave 0

    int block = 256, grid = 0, slots = 0, wave_n = 0, n_waves = 0;
    int tuned = 0;           // variants timed by the autotuner (0: heuristic choice)
    // graph mode: the captured solve and what it was captured for
    hipStream_t gstream = nullptr;
    hipGraphExec_t gexec = nullptr;
    unsigned long long pairs_gen = 0, g_pairs_gen = 0, g_net_gen = 0;
    const void *g_phi = nullptr;
    bool g_learned = false, last_graph = false;
    int graph_builds = 0, graph_launches = 0;
    double tune_ms = 0.0;    // time of the timed tuning launches
    bool tune_on_pairs = false;   // variant to be timed on the first per-pair class mix
    CgVariant var{0, 256, 0, 0, 0, 0, 0, 1, 1, 0x1f};
    size_t lds_bytes = 0;
    long long slot_n = 0;
    const void *phi = nullptr;
    hipEvent_t ev[7] = {};
    std::vector<hipEvent_t> ev_cg;   // per wave: around the CG launch
    bool have_events = false;
    bool solved_once = false;
    int last_grid = 0;           // CG work-groups of the last solve
    bool last_cg_timed = false;  // the last solve recorded per-wave CG events
};

namespace {

exx_status fail(exx_ctx *c, exx_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c ? c->err : g_setup_error, sizeof g_setup_error, fmt, ap);
    va_end(ap);
    return st;
}

#define EXX_GUARDED(ctx, call)                                                   \
    try {                                                                        \
        return call;                                                             \
    } catch (const std::bad_alloc &) {                                           \
        return fail(ctx, EXX_ENOMEM, "host allocation failed");                  \
    } catch (...) {                                                              \
        return fail(ctx, EXX_EDEVICE, "unexpected C++ exception");               \
    }

#define HIPCHK(ctx, call)                                                                            \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return fail(ctx, e_ == hipErrorOutOfMemory ? EXX_ENOMEM : EXX_EDEVICE, "%s: %s (%s:%d)", \
                        #call, hipGetErrorString(e_), __FILE__, __LINE__);                           \
    } while (0)

template <typename T>
void dev_free(DevBuf<T> &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.n = 0;
}

// Grows a buffer to at least n elements.  Large buffers get 3 % slack so
// that the pair count drifting between MD steps does not reallocate them.
template <typename T>
exx_status dev_reserve(exx_ctx *c, DevBuf<T> &b, size_t n)
{
    if (n <= b.n && b.p) return EXX_OK;
    dev_free(b);
    if (n * sizeof(T) > ((size_t)1 << 28)) n += n / 33;
    size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        return fail(c, EXX_ENOMEM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    b.n = std::max<size_t>(n, 1);
    return EXX_OK;
}

template <typename T>
exx_status upload(exx_ctx *c, DevBuf<T> &b, const std::vector<T> &v)
{
    exx_status st = dev_reserve(c, b, v.size());
    if (st != EXX_OK) return st;
    if (!v.empty()) HIPCHK(c, hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return EXX_OK;
}

// Stream-ordered upload.  With sync the host vector may die on return;
// without, it must outlive the copy.
template <typename T>
exx_status upload_async(exx_ctx *c, DevBuf<T> &b, const std::vector<T> &v, hipStream_t s, bool sync)
{
    exx_status st = dev_reserve(c, b, v.size());
    if (st != EXX_OK) return st;
    if (!v.empty()) HIPCHK(c, hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    if (sync) HIPCHK(c, hipStreamSynchronize(s));
    return EXX_OK;
}

bool inside(const double h[3], int x, int y, int z, double R)
{
    const double dx = x * h[0], dy = y * h[1], dz = z * h[2];
    return dx * dx + dy * dy + dz * dz <= R * R * (1.0 + 1e-12);
}

// Builds the tables of one class.  Offsets o_a range over the cell points,
// [-c0_a, N_a - 1 - c0_a] (Alg. 2 loops over the grid, so a sphere wider than
// the cell is clipped and no grid point appears twice).
exx_status build_class(exx_ctx *c, HostClass &k, double r_pe, double r_me)
{
    const int *N = c->prm.n_grid;
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        const int ext = (int)std::ceil(r_me / c->h[a]) + 1;
        lo[a] = std::max(-c->c0[a], -ext);
        hi[a] = std::min(N[a] - 1 - c->c0[a], ext);
    }
    k.r_pe = r_pe;
    k.r_me = r_me;
    // ME and PE runs per (z, y)
    struct Run { int mlo, mhi, plo, phi; };
    const int ny = hi[1] - lo[1] + 1, nz = hi[2] - lo[2] + 1;
    std::vector<Run> runs((size_t)ny * nz, Run{1, 0, 1, 0});
    int mb[6] = {1 << 30, -(1 << 30), 1 << 30, -(1 << 30), 1 << 30, -(1 << 30)};
    int pb[6] = {1 << 30, -(1 << 30), 1 << 30, -(1 << 30), 1 << 30, -(1 << 30)};
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y) {
            Run &r = runs[(size_t)(z - lo[2]) * ny + (y - lo[1])];
            for (int x = lo[0]; x <= hi[0]; ++x) {
                if (inside(c->h, x, y, z, r_me)) {
                    if (r.mlo > r.mhi) r.mlo = x;
                    r.mhi = x;
                }
                if (inside(c->h, x, y, z, r_pe)) {
                    if (r.plo > r.phi) r.plo = x;
                    r.phi = x;
                }
            }
            if (r.mlo <= r.mhi) {
                mb[0] = std::min(mb[0], r.mlo); mb[1] = std::max(mb[1], r.mhi);
                mb[2] = std::min(mb[2], y); mb[3] = std::max(mb[3], y);
                mb[4] = std::min(mb[4], z); mb[5] = std::max(mb[5], z);
            }
            if (r.plo <= r.phi) {
                pb[0] = std::min(pb[0], r.plo); pb[1] = std::max(pb[1], r.phi);
                pb[2] = std::min(pb[2], y); pb[3] = std::max(pb[3], y);
                pb[4] = std::min(pb[4], z); pb[5] = std::max(pb[5], z);
            }
        }
    if (pb[0] > pb[1]) return fail(c, EXX_EINVAL, "PE sphere of radius %g holds no grid point", r_pe);
    auto run_at = [&](int y, int z) -> const Run * {
        if (y < lo[1] || y > hi[1] || z < lo[2] || z > hi[2]) return nullptr;
        return &runs[(size_t)(z - lo[2]) * ny + (y - lo[1])];
    };
    // Every stencil neighbour of every PE point must lie in PE u shell.
    for (int z = pb[4]; z <= pb[5]; ++z)
        for (int y = pb[2]; y <= pb[3]; ++y) {
            const Run *r = run_at(y, z);
            if (!r || r->plo > r->phi) continue;
            if (r->plo - FD_N < r->mlo || r->phi + FD_N > r->mhi)
                return fail(c, EXX_EINVAL, "R_ME - R_PE (%g - %g) leaves the stencil outside the ME sphere", r_me, r_pe);
            for (int s = -FD_N; s <= FD_N; ++s) {
                if (!s) continue;
                const Run *ry = run_at(y + s, z), *rz = run_at(y, z + s);
                for (const Run *q : {ry, rz})
                    if (!q || q->mlo > r->plo || q->mhi < r->phi)
                        return fail(c, EXX_EINVAL,
                                    "R_ME - R_PE (%g - %g) leaves the stencil outside the ME sphere (or the cell clips it)",
                                    r_me, r_pe);
            }
        }
    k.pxlo = pb[0]; k.pxhi = pb[1]; k.pylo = pb[2]; k.pyhi = pb[3]; k.pzlo = pb[4]; k.pzhi = pb[5];
    k.mxlo = mb[0]; k.mxhi = mb[1]; k.mylo = mb[2]; k.myhi = mb[3]; k.mzlo = mb[4]; k.mzhi = mb[5];
    const int pny = k.pyhi - k.pylo + 1, pnz = k.pzhi - k.pzlo + 1;
    const int mny = k.myhi - k.mylo + 1, mnz = k.mzhi - k.mzlo + 1;
    k.pe_rows.assign((size_t)pny * pnz, int4{0, 1, 0, 0});
    k.me_rows.assign((size_t)2 * mny * mnz, int4{0, 1, 0, 0});
    for (size_t row = 0; row < (size_t)mny * mnz; ++row) k.me_rows[2 * row + 1] = int4{1, 0, 0, 0};  // empty run
    k.pe_xyz.clear();
    k.sh_xyz.clear();
    // PE packing, z-major / y / x (the order of Alg. 2)
    int base = 0;
    for (int z = k.pzlo; z <= k.pzhi; ++z)
        for (int y = k.pylo; y <= k.pyhi; ++y) {
            const Run *r = run_at(y, z);
            if (!r || r->plo > r->phi) continue;
            k.pe_rows[(size_t)(z - k.pzlo) * pny + (y - k.pylo)] = int4{base, r->plo, r->phi, 0};
            for (int x = r->plo; x <= r->phi; ++x) k.pe_xyz.push_back(pack_xyz(x, y, z));
            base += r->phi - r->plo + 1;
        }
    k.n_pe = base;
    // Shell packing: same order, left run then right run of each row
    int sbase = 0;
    for (int z = k.mzlo; z <= k.mzhi; ++z)
        for (int y = k.mylo; y <= k.myhi; ++y) {
            const Run *r = run_at(y, z);
            if (!r || r->mlo > r->mhi) continue;
            int plo = r->plo, phi = r->phi, pe_base = 0;
            if (plo > phi) { plo = r->mhi + 1; phi = r->mhi; }
            else pe_base = k.pe_rows[(size_t)(z - k.pzlo) * pny + (y - k.pylo)].x;
            const size_t row = (size_t)(z - k.mzlo) * mny + (y - k.mylo);
            k.me_rows[2 * row] = int4{pe_base, plo, phi, sbase};
            k.me_rows[2 * row + 1] = int4{r->mlo, r->mhi, 0, 0};
            for (int x = r->mlo; x <= r->mhi; ++x)
                if (x < plo || x > phi) {
                    k.sh_xyz.push_back(pack_xyz(x, y, z));
                    ++sbase;
                }
        }
    k.n_sh = sbase;
    // Projection columns of PE onto the xy plane, sorted (y, x)
    k.cols.clear();
    k.colz.clear();
    for (int y = k.pylo; y <= k.pyhi; ++y) {
        int xl = 1 << 30, xh = -(1 << 30);
        for (int z = k.pzlo; z <= k.pzhi; ++z) {
            const Run *r = run_at(y, z);
            if (!r || r->plo > r->phi) continue;
            xl = std::min(xl, r->plo);
            xh = std::max(xh, r->phi);
        }
        for (int x = xl; x <= xh; ++x) {
            k.cols.push_back(pack_xyz(x, y, 0));
            int zl = 1 << 30, zh = -(1 << 30);
            for (int z = k.pzlo; z <= k.pzhi; ++z) {
                const Run *r = run_at(y, z);
                if (r && r->plo <= x && x <= r->phi) { zl = std::min(zl, z); zh = std::max(zh, z); }
            }
            // the z extent of a column of a convex set is one interval
            for (int z = zl; z <= zh; ++z) {
                const Run *r = run_at(y, z);
                if (!r || r->plo > x || x > r->phi)
                    return fail(c, EXX_EINVAL, "PE column (%d, %d) is not one z interval", x, y);
            }
            k.colz.push_back((zl + 512) | ((zh + 512) << 16));
        }
    }
    k.pe_off.assign((size_t)pny * pnz, 0);
    for (size_t t = 0; t < k.pe_rows.size(); ++t)
        if (k.pe_rows[t].y <= k.pe_rows[t].z) k.pe_off[t] = k.pe_rows[t].x - k.pe_rows[t].y;
    // Stencil coupling of PE points to the shell, the boundary-charge term of
    // Eq. pe_mat_red: for each PE point with a stencil neighbour outside PE,
    // its neighbours on the shell as (shell index << 4) | (axis * 3 + s - 1),
    // in the order the right-hand side adds them (s = 1..3, then -s before
    // +s, then x, y, z).  Interior points have none: only the layer within
    // three points of the surface is listed (a sixth of PE at R_PE = 41 h).
    {
        auto pe_at = [&](int x, int y, int z) -> int {
            const int zz = z - k.pzlo, yy = y - k.pylo;
            if (zz < 0 || zz >= pnz || yy < 0 || yy >= pny) return -1;
            const int4 r = k.pe_rows[(size_t)zz * pny + yy];
            return (x < r.y || x > r.z) ? -1 : r.x + x - r.y;
        };
        auto sh_at = [&](int x, int y, int z) -> int {
            const size_t row = (size_t)(z - k.mzlo) * mny + (y - k.mylo);
            const int4 a = k.me_rows[2 * row], b = k.me_rows[2 * row + 1];
            return a.w + (x < a.y ? x - b.x : (a.y - b.x) + (x - a.z - 1));
        };
        k.bnd_q.clear();
        k.bnd_ent.clear();
        k.bnd_ptr.assign(1, 0);
        for (int q = 0; q < k.n_pe; ++q) {
            int x, y, z;
            unpack_xyz(k.pe_xyz[q], x, y, z);
            const size_t before = k.bnd_ent.size();
            for (int s = 1; s <= FD_N; ++s)
                for (int sg = -1; sg <= 1; sg += 2) {
                    const int d = sg * s;
                    const int nb[3][3] = {{x + d, y, z}, {x, y + d, z}, {x, y, z + d}};
                    for (int ax = 0; ax < 3; ++ax)
                        if (pe_at(nb[ax][0], nb[ax][1], nb[ax][2]) < 0) {
                            const int sh = sh_at(nb[ax][0], nb[ax][1], nb[ax][2]);
                            if (sh < 0 || sh >= k.n_sh || sh >= (1 << 27))
                                return fail(c, EXX_EINVAL, "shell index %d of PE point %d out of range", sh, q);
                            k.bnd_ent.push_back((sh << 4) | (ax * 3 + s - 1));
                        }
                }
            if (k.bnd_ent.size() != before) {
                k.bnd_q.push_back(q);
                k.bnd_ptr.push_back((int)k.bnd_ent.size());
            }
        }
    }
    return EXX_OK;
}

// Copies the tables of one class to the current device.
exx_status upload_class(exx_ctx *c, HostClass &k)
{
    auto up = [&](auto **dst, const auto &v) -> exx_status {
        using T = std::remove_reference_t<decltype(v[0])>;
        size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(T);
        HIPCHK(c, hipMalloc((void **)dst, bytes));
        if (!v.empty()) HIPCHK(c, hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
        return EXX_OK;
    };
    exx_status st;
    if ((st = up(&k.d_pe_rows, k.pe_rows)) != EXX_OK) return st;
    if ((st = up(&k.d_me_rows, k.me_rows)) != EXX_OK) return st;
    if ((st = up(&k.d_pe_xyz, k.pe_xyz)) != EXX_OK) return st;
    if ((st = up(&k.d_sh_xyz, k.sh_xyz)) != EXX_OK) return st;
    if ((st = up(&k.d_cols, k.cols)) != EXX_OK) return st;
    if ((st = up(&k.d_colz, k.colz)) != EXX_OK) return st;
    if ((st = up(&k.d_pe_off, k.pe_off)) != EXX_OK) return st;
    if ((st = up(&k.d_bnd_q, k.bnd_q)) != EXX_OK) return st;
    if ((st = up(&k.d_bnd_ptr, k.bnd_ptr)) != EXX_OK) return st;
    if ((st = up(&k.d_bnd_ent, k.bnd_ent)) != EXX_OK) return st;
    return EXX_OK;
}

// Coarse levels of the multigrid preconditioner: level 1 cells are 2x2x2
// blocks of the PE bounding box, each level halves the previous; a cell is
// in the domain if any child is, and stores which children are.  Levels stop
// at an edge of at most 6 cells.  Per slot the scratch holds f, e, t of every
// level, then the fine residual (FP32) on the even-padded PE box and a sink.
exx_status build_mg_levels(exx_ctx *c, HostClass &k)
{
    const int pny = k.pyhi - k.pylo + 1;
    std::vector<unsigned char> prev;   // level l - 1 child bits
    int pn[3] = {k.pxhi - k.pxlo + 1, pny, k.pzhi - k.pzlo + 1};
    k.mg_levels = 0;
    k.mg_doubles = 0;
    k.mg_cells_bytes = 0;
    k.mg_cells_bytes32 = 0;
    while (k.mg_levels < MG_MAX) {
        const int l = k.mg_levels;
        int m[3];
        for (int d = 0; d < 3; ++d) m[d] = (pn[d] + 1) / 2;
        std::vector<unsigned char> cm((size_t)m[0] * m[1] * m[2], 0);
        int64_t in = 0;
        for (int z = 0; z < m[2]; ++z)
            for (int y = 0; y < m[1]; ++y)
                for (int x = 0; x < m[0]; ++x) {
                    unsigned bits = 0;
                    for (int t = 0; t < 8; ++t) {
                        const int cx = 2 * x + (t & 1), cy = 2 * y + ((t >> 1) & 1), cz = 2 * z + (t >> 2);
                        if (cx >= pn[0] || cy >= pn[1] || cz >= pn[2]) continue;
                        bool any;
                        if (l == 0) {
                            const int4 r = k.pe_rows[(size_t)cz * pny + cy];
                            any = r.y <= r.z && k.pxlo + cx >= r.y && k.pxlo + cx <= r.z;
                        } else {
                            any = prev[((size_t)cz * pn[1] + cy) * pn[0] + cx] != 0;
                        }
                        if (any) bits |= 1u << t;
                    }
                    cm[((size_t)z * m[1] + y) * m[0] + x] = (unsigned char)bits;
                    in += bits ? 1 : 0;
                }
        for (int d = 0; d < 3; ++d) k.mg_n[l][d] = m[d];
        k.mg_off[l] = k.mg_doubles;
        const long long n = (long long)m[0] * m[1] * m[2];
        k.mg_doubles += (3 * n + 1) / 2 * 2;   // even: the dense box after the levels is 16-byte aligned
        // algorithmic bytes per V-cycle: level 1 restriction (8 FP32 values
        // of the dense box, child bits, f) and the correction its POST pass
        // gathers; per level the down pass (f, bits) and the up pass (f, the
        // coarser e, bits, e)
        if (l == 0) {
            k.mg_cells_bytes += in * (32 + 1 + 8 + 8);
            k.mg_cells_bytes32 += in * (32 + 1 + 4 + 4);
        }
        k.mg_cells_bytes += in * (8 + 1 + 8 + 8 + 1 + 8);
        k.mg_cells_bytes32 += in * (4 + 1 + 4 + 4 + 1 + 4);
        if (k.d_mg_mask[l]) { (void)hipFree(k.d_mg_mask[l]); k.d_mg_mask[l] = nullptr; }
        HIPCHK(c, hipMalloc((void **)&k.d_mg_mask[l], cm.size()));
        HIPCHK(c, hipMemcpy(k.d_mg_mask[l], cm.data(), cm.size(), hipMemcpyHostToDevice));
        k.mg_mask[l] = std::move(cm);
        prev = k.mg_mask[l];
        for (int d = 0; d < 3; ++d) pn[d] = m[d];
        ++k.mg_levels;
        if (std::max({m[0], m[1], m[2]}) <= 6) break;
    }
    k.mg_dense_off = k.mg_doubles;
    k.mg_doubles += 4LL * k.mg_n[0][0] * k.mg_n[0][1] * k.mg_n[0][2] + 2;   // FP32 box and sink
    return EXX_OK;
}

long long mg_slot_doubles(const exx_ctx *c)
{
    long long m = 0;
    for (int k = 0; k < c->n_cls; ++k) m = std::max(m, c->cls[k].mg_doubles);
    return m;
}

// the class with the most PE points, and the largest PE / PE + shell sizes
int big_class(const exx_ctx *c)
{
    int b = 0;
    for (int k = 1; k < c->n_cls; ++k)
        if (c->cls[k].n_pe > c->cls[b].n_pe) b = k;
    return b;
}

ClassDev class_dev(const HostClass &k)
{
    ClassDev d{};
    d.pe_rows = k.d_pe_rows;
    d.me_rows = k.d_me_rows;
    d.pe_xyz = k.d_pe_xyz;
    d.sh_xyz = k.d_sh_xyz;
    d.cols = k.d_cols;
    d.n_cols = (int)k.cols.size();
    d.pxlo = k.pxlo; d.pylo = k.pylo; d.pzlo = k.pzlo;
    d.pnx = k.pxhi - k.pxlo + 1; d.pny = k.pyhi - k.pylo + 1; d.pnz = k.pzhi - k.pzlo + 1;
    d.mxlo = k.mxlo; d.mylo = k.mylo; d.mzlo = k.mzlo;
    d.mnx = k.mxhi - k.mxlo + 1; d.mny = k.myhi - k.mylo + 1; d.mnz = k.mzhi - k.mzlo + 1;
    d.n_pe = k.n_pe;
    d.n_sh = k.n_sh;
    d.colz = k.d_colz;
    d.pe_off = k.d_pe_off;
    d.bnd_q = k.d_bnd_q;
    d.bnd_ptr = k.d_bnd_ptr;
    d.bnd_ent = k.d_bnd_ent;
    d.n_bnd = (int)k.bnd_q.size();
    d.bands = k.d_bands;
    d.n_bands = (int)k.bands.size() / 12;
    d.tbl_ints = (d.pny * d.pnz + 3) / 4 * 4;
    d.lds_w = d.pnx + 6;
    d.plane_rows = k.plane_rows;
    d.lds_plane = k.plane_rows * (d.pnx + 6);
    d.bands32 = k.d_bands32;
    d.n_bands32 = (int)k.bands32.size() / 12;
    d.lds_plane32 = k.plane_rows32 * (d.pnx + 6);
    return d;
}

OrbBox orb_box(const exx_ctx *c)
{
    OrbBox b{};
    b.org = c->d_box_org.p;
    b.bx = c->box[0];
    b.by = c->box[1];
    b.bz = c->box[2];
    b.vol = c->box_vol;
    return b;
}

DxxArgs dxx_args(const exx_ctx *c, const void *phi, void *dxx)
{
    DxxArgs d{};
    for (int k = 0; k < c->n_cls; ++k) d.cls[k] = class_dev(c->cls[k]);
    d.pair_gc = c->d_gc.p;
    d.pair_ij = c->d_ij.p;
    d.out_off = c->d_off.p;
    d.orb_ptr = c->d_orb_ptr.p;
    d.orb_pairs = c->d_orb_pairs.p;
    d.phi = phi;
    d.box = orb_box(c);
    d.dxx = dxx;
    d.acc = c->d_dacc.p;
    d.f32 = c->prm.orbital_dtype == EXX_F32;
    d.nx = c->prm.n_grid[0];
    d.ny = c->prm.n_grid[1];
    d.nz = c->prm.n_grid[2];
    d.ngrid = (long long)d.nx * d.ny * d.nz;
    d.vout = c->d_vout.p;
    d.pair_lo = 0;
    d.pair_hi = (int)c->n_pairs;
    return d;
}

// Largest |offset| of a PE point over both classes (grid points).
int pe_rmax(const exx_ctx *c)
{
    int r = 0;
    for (const HostClass &k : c->cls)
        r = std::max({r, -k.pxlo, k.pxhi, -k.pylo, k.pyhi, -k.pzlo, k.pzhi});
    return r;
}

NetPairArgs net_args(const exx_ctx *c)
{
    NetPairArgs n{};
    for (int k = 0; k < c->n_cls; ++k) n.cls[k] = class_dev(c->cls[k]);
    n.pair_gc = c->d_gc.p;
    n.out_off = c->d_off.p;
    n.rhs = c->d_rhs.p;
    n.rhs_off = c->d_rhs_off.p;
    n.wave_begin = 0;
    n.vout = c->d_vout.p;
    n.h2 = std::cbrt(c->h[0] * c->h[1] * c->h[2]);
    n.h2 *= n.h2;
    for (int k = 0; k < c->n_cls; ++k) n.bnd[k] = c->d_bnd[k].p;
    return n;
}

// Splits the PE projection columns of one class into y bands of whole rows,
// each with at most v.cols * v.block columns and at most v.halo * v.block
// columns in its 3-row halos.  Returns false if the variant cannot hold it.
bool make_bands(const HostClass &k, int cols_per_thread, int halo_per_thread, int block, std::vector<int> &out,
                int *plane_rows)
{
    out.clear();
    *plane_rows = 0;
    const int ny = k.pyhi - k.pylo + 1;
    std::vector<int> start(ny + 1, 0);
    for (int c : k.cols) {
        int x, y, z;
        unpack_xyz(c, x, y, z);
        start[y - k.pylo + 1]++;
    }
    for (int y = 0; y < ny; ++y) start[y + 1] += start[y];
    const int ncols = start[ny];
    const long cap = (long)cols_per_thread * block;
    const int nb = (int)((ncols + cap - 1) / cap);
    const int target = (ncols + nb - 1) / nb;
    int y0 = 0;
    while (y0 < ny) {
        int y1 = y0;
        while (y1 < ny && (start[y1 + 1] - start[y0]) <= cap && (y1 == y0 || start[y1] - start[y0] < target)) ++y1;
        if (y1 == y0) return false;                  // a single row exceeds the capacity
        const int lo0 = std::max(0, y0 - 3), hi1 = std::min(ny, y1 + 3);
        const int nh = (start[y0] - start[lo0]) + (start[hi1] - start[y1]);
        if (nh > (long)halo_per_thread * block) return false;
        int zlo = 1 << 30, zhi = -(1 << 30);
        for (int z = k.pzlo; z <= k.pzhi; ++z)
            for (int y = y0; y < y1; ++y) {
                const int4 r = k.pe_rows[(size_t)(z - k.pzlo) * ny + y];
                if (r.y <= r.z) { zlo = std::min(zlo, z); zhi = std::max(zhi, z); }
            }
        out.insert(out.end(), {start[y0], start[y1], start[lo0], start[y0], start[y1], start[hi1], zlo, zhi,
                               k.pylo + y0, k.pylo + y1 - 1, 0, 0});
        *plane_rows = std::max(*plane_rows, y1 - y0 + 6);
        y0 = y1;
    }
    return true;
}

void free_class(HostClass &k)
{
    for (void *p : {(void *)k.d_pe_rows, (void *)k.d_me_rows, (void *)k.d_pe_xyz, (void *)k.d_sh_xyz,
                    (void *)k.d_cols, (void *)k.d_bands, (void *)k.d_colz, (void *)k.d_pe_off, (void *)k.d_bands32,
                    (void *)k.d_bnd_q, (void *)k.d_bnd_ptr, (void *)k.d_bnd_ent})
        if (p) (void)hipFree(p);
    k.d_pe_rows = k.d_me_rows = nullptr;
    k.d_pe_xyz = k.d_sh_xyz = k.d_cols = k.d_bands = k.d_colz = k.d_pe_off = k.d_bands32 = nullptr;
    k.d_bnd_q = k.d_bnd_ptr = k.d_bnd_ent = nullptr;
    for (auto &m : k.d_mg_mask)
        if (m) { (void)hipFree(m); m = nullptr; }
}

double fact(int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }

void ylm_norms(double *out)
{
    for (int l = 0; l <= LMAX; ++l)
        for (int m = -l; m <= l; ++m) {
            const int am = m < 0 ? -m : m;
            double v = (2 * l + 1) / (4.0 * M_PI) * fact(l - am) / fact(l + am);
            if (am) v *= 2.0;
            out[l * l + l + m] = std::sqrt(v);
        }
}

constexpr size_t kMaxLds = 160 * 1024 - 1024;   // gfx950 LDS per work-group, less static use

// LDS of the z-march kernel for one class: row-offset table + two planes.
size_t zmarch_lds(const HostClass &k, int plane_rows, int plane_rows32)
{
    const size_t pny = k.pyhi - k.pylo + 1, pnz = k.pzhi - k.pzlo + 1, pnx = k.pxhi - k.pxlo + 1;
    const size_t p64 = (2 * (size_t)plane_rows * (pnx + 6) + 2) * sizeof(double);
    const size_t p32 = (2 * (size_t)plane_rows32 * (pnx + 6) + 2) * sizeof(float);
    return (pny * pnz + 3) / 4 * 4 * sizeof(int) + std::max(p64, p32);
}

// Installs variant v: band tables of both classes on the device.
exx_status install_variant(exx_ctx *c, const CgVariant &v, size_t lds)
{
    c->var = v;
    c->lds_bytes = v.zmarch ? lds : 0;
    for (int kk = 0; kk < c->n_cls; ++kk) {
        HostClass &k = c->cls[kk];
        if (k.d_bands) { (void)hipFree(k.d_bands); k.d_bands = nullptr; }
        if (k.d_bands32) { (void)hipFree(k.d_bands32); k.d_bands32 = nullptr; }
        k.bands.clear();
        k.bands32.clear();
        k.plane_rows = k.plane_rows32 = 0;
        if (v.zmarch) {
            make_bands(k, v.cols, v.halo, v.block, k.bands, &k.plane_rows);
            HIPCHK(c, hipMalloc((void **)&k.d_bands, k.bands.size() * sizeof(int)));
            HIPCHK(c, hipMemcpy(k.d_bands, k.bands.data(), k.bands.size() * sizeof(int), hipMemcpyHostToDevice));
            if (c->prm.precision == EXX_FP32_REFINE) {
                make_bands(k, v.cols32, v.halo32, v.block, k.bands32, &k.plane_rows32);
                HIPCHK(c, hipMalloc((void **)&k.d_bands32, k.bands32.size() * sizeof(int)));
                HIPCHK(c, hipMemcpy(k.d_bands32, k.bands32.data(), k.bands32.size() * sizeof(int),
                                    hipMemcpyHostToDevice));
            }
        }
    }
    c->block = v.block;
    return EXX_OK;
}

struct Candidate {
    CgVariant v;
    size_t lds;
    int per_cu;
    long score;
    int bands;               // y bands over all classes (each re-reads 3-row halos)
};

// Multigrid arguments of the CG kernel: the levels of every class and the
// per-slot coarse scratch.
void mg_args(const exx_ctx *c, SolveArgs &a, double *scratch)
{
    a.mg = c->prm.precond == EXX_PRECOND_MG;
    if (!a.mg) return;
    for (int k = 0; k < c->n_cls; ++k) {
        const HostClass &hc = c->cls[k];
        a.mgc[k].levels = hc.mg_levels;
        a.mgc[k].dense_off = hc.mg_dense_off;
        for (int l = 0; l < hc.mg_levels; ++l)
            a.mgc[k].lv[l] = MgLevel{hc.mg_n[l][0], hc.mg_n[l][1], hc.mg_n[l][2], hc.d_mg_mask[l], hc.mg_off[l]};
    }
    a.mg_scratch = scratch;
    a.mg_slot_n = mg_slot_doubles(c);
    // damping: the fine Jacobi step keeps M positive definite for
    // omega < 2 diag(A) / lambda_max(A) ~ 0.90 (the sixth-order stencil's
    // largest eigenvalue is ~2.22 diag).  A coarse level contributes
    // 2S - S L S (S = omega_c / diag L) plus a positive semidefinite term, so
    // it stays positive definite while omega_c lambda_max(D^-1 L) < 2; the
    // masked 7-point Laplacian with Dirichlet zero outside has
    // lambda_max(D^-1 L) < 2, so omega_c = 1 qualifies.  One damped Jacobi step
    // on the coarsest level: more sweeps there (a more exact coarse solve)
    // took more PCG iterations on the water workloads (8 sweeps at
    // omega_c = 0.9: 33.2 iterations on the 512-water step and 40.2 on the
    // 64-water one; 1 step at omega_c = 1: 29.6 and 36.1).
    // The correction the V-cycle hands to the fine level is scaled by 0.5:
    // with the piecewise-constant prolongation and the 7-point coarse
    // operator the full correction overshoots (measured: 29.6 / 36.1
    // iterations at scale 1, 27.2 / 33.1 at 0.4-0.6, 28.3 / 34.2 at 0.8,
    // 31.7 / 37.5 at 1.2).  M stays positive definite for any positive scale
    // (it multiplies a positive semidefinite term).
    a.mg_omega = 0.8;
    a.mg_omega_c = 1.0;
    a.mg_coarse_sweeps = 1;
    a.mg_coarse_scale = 0.5;
}

// Measured choice among the candidates: each runs kTuneIters CG iterations
// (60; 15 with the multigrid preconditioner) on every pair of a synthetic
// batch (constant right-hand side, residual target 0 so no pair stops early;
// two pairs per resident work-group of the widest grid), after one untimed
// launch; the fastest wins, a tie within 1 % going to the fewest bands.  The
// batch is the largest class, or, given mix (pairs per class of the real
// list), the classes in those proportions, larger classes first as in the
// CG queue.  Returns the index of the winner, or -1 (heuristic) when the
// device cannot hold the batch.
int autotune(exx_ctx *c, const std::vector<Candidate> &cands, double *tune_ms, const int64_t *mix)
{
    // a preconditioned iteration costs about four plain ones
    const int kTuneIters = c->prm.precond == EXX_PRECOND_MG ? 15 : 60;
    const int kb = big_class(c);               // the synthetic batch runs the largest class
    const HostClass &k = c->cls[kb];
    int max_grid = 0;
    for (const Candidate &q : cands) max_grid = std::max(max_grid, q.per_cu * c->n_cu);
    const int n = 2 * max_grid;
    const long long slot_n = ((long long)k.n_pe + 1 + 63) / 64 * 64;
    const long long per_pair = (long long)k.n_pe + k.n_sh;
    const size_t ngrid = (size_t)c->prm.n_grid[0] * c->prm.n_grid[1] * c->prm.n_grid[2];
    const bool mixed = c->prm.precision == EXX_FP32_REFINE;
    const bool mg = c->prm.precond == EXX_PRECOND_MG;
    const int nvec = mg ? 4 : 3;
    const size_t need = (size_t)n * (slot_n + per_pair) * 8 + (size_t)max_grid * slot_n * (nvec * 8 + (mixed ? 16 : 0)) +
                        (mg ? (size_t)max_grid * mg_slot_doubles(c) * 8 : 0) + ngrid * 8 + (size_t)n * (NLM * 8 + 64);
    size_t freeb = 0, totalb = 0;
    if (hipMemGetInfo(&freeb, &totalb) != hipSuccess || need + ((size_t)2 << 30) > freeb) return -1;
    std::vector<void *> allocs;
    auto dev = [&](size_t bytes) -> void * {
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(bytes, 8)) != hipSuccess) return nullptr;
        allocs.push_back(p);
        return p;
    };
    auto release = [&]() { for (void *p : allocs) (void)hipFree(p); allocs.clear(); };
    double *phi = (double *)dev(ngrid * 8), *rhs = (double *)dev((size_t)n * slot_n * 8);
    double *vout = (double *)dev((size_t)n * per_pair * 8), *scr = (double *)dev((size_t)max_grid * nvec * slot_n * 8);
    float *scr32 = mixed ? (float *)dev((size_t)max_grid * 4 * slot_n * 4) : nullptr;
    double *mgs = mg ? (double *)dev((size_t)max_grid * mg_slot_doubles(c) * 8) : nullptr;
    double *q = (double *)dev((size_t)n * NLM * 8), *e = (double *)dev((size_t)n * 8), *rr = (double *)dev((size_t)n * 8);
    int *it = (int *)dev((size_t)n * 4), *ou = (int *)dev((size_t)n * 4), *cv = (int *)dev((size_t)n * 4);
    int *counter = (int *)dev(4);
    int4 *gc = (int4 *)dev((size_t)n * sizeof(int4));
    int4 *org = (int4 *)dev(sizeof(int4));
    int2 *ij = (int2 *)dev((size_t)n * sizeof(int2));
    long long *off = (long long *)dev((size_t)n * 8), *boff = (long long *)dev((size_t)n * 8);
    hipEvent_t ev[2] = {};
    int best = -1;
    float best_ms = 0.f;
    std::vector<float> times(cands.size(), 1e30f);
    if (allocs.size() != (size_t)(16 + (mixed ? 1 : 0) + (mg ? 1 : 0)) || hipEventCreate(&ev[0]) != hipSuccess ||
        hipEventCreate(&ev[1]) != hipSuccess) {
        release();
        for (auto &x : ev) if (x) (void)hipEventDestroy(x);
        return -1;
    }
    std::vector<int4> hgc((size_t)n, int4{0, 0, 0, kb});
    if (mix) {
        // pairs per class in proportion to the real list (each class in use
        // at least once), the larger classes first
        int64_t tot = 0;
        for (int k = 0; k < c->n_cls; ++k) tot += mix[k];
        std::vector<int> cnt(c->n_cls, 0);
        int used = 0;
        for (int k = 0; k < c->n_cls && tot > 0; ++k) {
            cnt[k] = mix[k] > 0 ? std::max(1, (int)((double)n * mix[k] / tot + 0.5)) : 0;
            used += cnt[k];
        }
        if (tot > 0) {
            int most = 0;
            for (int k = 1; k < c->n_cls; ++k) if (cnt[k] > cnt[most]) most = k;
            cnt[most] = std::max(1, cnt[most] + (n - used));
            std::vector<int> order(c->n_cls);
            for (int k = 0; k < c->n_cls; ++k) order[k] = k;
            std::stable_sort(order.begin(), order.end(), [&](int u, int v) { return c->cls[u].n_pe > c->cls[v].n_pe; });
            size_t p = 0;
            for (int k : order)
                for (int t = 0; t < cnt[k] && p < hgc.size(); ++t) hgc[p++].w = k;
            for (; p < hgc.size(); ++p) hgc[p].w = order.back();
        }
    }
    std::vector<int2> hij((size_t)n, int2{0, 0});
    std::vector<long long> hoff((size_t)n), hboff((size_t)n);
    for (int p = 0; p < n; ++p) hoff[p] = (long long)p * per_pair;
    for (int p = 0; p < n; ++p) hboff[p] = (long long)p * slot_n;
    bool ok = hipMemset(phi, 0, ngrid * 8) == hipSuccess &&
              hipMemset(rhs, 0x3f, (size_t)n * slot_n * 8) == hipSuccess &&    // b = 4.8e-4 everywhere
              hipMemset(vout, 0, (size_t)n * per_pair * 8) == hipSuccess &&
              hipMemcpy(gc, hgc.data(), hgc.size() * sizeof(int4), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(ij, hij.data(), hij.size() * sizeof(int2), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemset(org, 0, sizeof(int4)) == hipSuccess &&
              hipMemcpy(off, hoff.data(), hoff.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(boff, hboff.data(), hboff.size() * 8, hipMemcpyHostToDevice) == hipSuccess;
    SolveArgs a{};
    a.pair_gc = gc;
    a.pair_ij = ij;
    a.out_off = off;
    a.phi = phi;
    a.box = OrbBox{org, c->prm.n_grid[0], c->prm.n_grid[1], c->prm.n_grid[2], (long long)ngrid};
    a.phi_f32 = 0;
    a.nx = c->prm.n_grid[0];
    a.ny = c->prm.n_grid[1];
    a.nz = c->prm.n_grid[2];
    a.ngrid = (long long)ngrid;
    a.vout = vout;
    a.rhs = rhs;
    a.rhs_off = boff;
    a.scratch = scr;
    a.scratch32 = scr32;
    a.slot_n = slot_n;
    a.q_out = q;
    a.e_out = e;
    a.iters_out = it;
    a.outer_out = ou;
    a.conv_out = cv;
    a.relres_out = rr;
    a.counter = counter;
    a.wave_begin = 0;
    a.wave_n = n;
    a.guess = c->prm.guess != EXX_GUESS_ZERO ? 1 : 0;
    a.precision = c->prm.precision;
    for (int d = 0; d < 3; ++d) a.h[d] = c->h[d];
    for (int d = 0; d < 4; ++d) a.wfd[d] = kFD[d];
    a.tol = 0.0;
    a.inner_tol = c->prm.inner_rtol;
    a.maxit = kTuneIters;
    ylm_norms(a.ylm_norm);
    mg_args(c, a, mgs);
    for (size_t i = 0; ok && i < cands.size(); ++i) {
        if (install_variant(c, cands[i].v, cands[i].lds) != EXX_OK) { ok = false; break; }
        for (int kk = 0; kk < c->n_cls; ++kk) a.cls[kk] = class_dev(c->cls[kk]);
        const int grid = std::min(n, cands[i].per_cu * c->n_cu);
        float ms = 0.f;
        for (int rep = 0; rep < 2 && ok; ++rep) {
            ok = launch_zero_int(counter, 1, 0) == hipSuccess && hipEventRecord(ev[0], 0) == hipSuccess &&
                 launch_cg(cands[i].v, a, grid, cands[i].lds, 0) == hipSuccess && hipEventRecord(ev[1], 0) == hipSuccess &&
                 hipEventSynchronize(ev[1]) == hipSuccess && hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess;
        }
        if (ok) times[i] = ms;
        if (ok && (best < 0 || ms < best_ms)) { best = (int)i; best_ms = ms; }
        *tune_ms += ms;
    }
    (void)hipDeviceSynchronize();
    release();
    for (auto &x : ev) (void)hipEventDestroy(x);
    (void)hipGetLastError();
    if (!ok) return -1;
    // Timings within 1 % are a tie (the synthetic batch does not separate
    // them reliably): take the one with the fewest bands, the fewest halo bytes.
    int pick = best;
    for (size_t i = 0; i < cands.size(); ++i)
        if (times[i] <= best_ms * 1.01f && cands[i].bands < cands[pick].bands) pick = (int)i;
    return pick;
}

// Chooses the CG kernel among the z-march variants that fit (and match a
// requested block / cols): by measurement when params.autotune is set and
// more than one fits, else the one with the most resident waves per CU, then
// the most work-groups per CU, then the fewest bands.  The flat kernel when
// none fits.
exx_status select_variant(exx_ctx *c, const int64_t *mix = nullptr)
{
    CgVariant vs[32];
    const int nv = cg_variants(vs, 32);
    std::vector<Candidate> cands;
    const int mode = cg_mode(c->prm.precision, c->prm.guess != EXX_GUESS_ZERO, c->prm.precond == EXX_PRECOND_MG);
    bool flat = false;
    for (int i = 0; i < nv; ++i) {
        const CgVariant &v = vs[i];
        if (c->prm.cg_cols < 0) { if (!v.zmarch) { flat = true; break; } continue; }
        if (!v.zmarch || !cg_variant_applies(v, mode)) continue;
        if (c->prm.block_threads && v.block != c->prm.block_threads) continue;
        if (c->prm.cg_cols && v.cols != c->prm.cg_cols) continue;
        bool fits = true;
        size_t lds = 0;
        int nb = 0;
        for (int k = 0; k < c->n_cls && fits; ++k) {
            int r = 0, r32 = 0;
            std::vector<int> bk, fk;
            fits = make_bands(c->cls[k], v.cols, v.halo, v.block, bk, &r) &&
                   (c->prm.precision != EXX_FP32_REFINE || make_bands(c->cls[k], v.cols32, v.halo32, v.block, fk, &r32));
            if (fits) lds = std::max(lds, zmarch_lds(c->cls[k], r, r32));
            nb += (int)bk.size() / 12;
        }
        if (!fits || lds > kMaxLds) continue;
        int per_cu = 0;
        if (cg_occupancy(v, mode, lds, &per_cu) != hipSuccess || per_cu < 1) continue;
        cands.push_back({v, lds, per_cu, (long)per_cu * v.block / 64 * 1000 + per_cu * 100 - nb, nb});
    }
    c->tuned = 0;
    c->tune_ms = 0.0;
    if (cands.empty()) {
        if (!flat && (c->prm.block_threads || c->prm.cg_cols))
            return fail(c, EXX_EINVAL, "no CG kernel variant with block %d and %d columns fits this subdomain",
                        c->prm.block_threads, c->prm.cg_cols);
        for (int i = 0; i < nv; ++i)
            if (!vs[i].zmarch) return install_variant(c, vs[i], 0);
        return fail(c, EXX_EINVAL, "no CG kernel available");
    }
    int best = -1;
    c->tune_on_pairs = false;
    if (c->prm.autotune && cands.size() > 1) {
        if (c->prm.n_classes >= 2 && !mix) {
            // per-pair classes: the mix of classes is known at the first
            // exx_pairs_spread, which times the variants on it
            c->tune_on_pairs = true;
        } else {
            best = autotune(c, cands, &c->tune_ms, mix);
            if (best >= 0) c->tuned = (int)cands.size();
        }
    }
    if (best < 0) {
        best = 0;
        for (size_t i = 1; i < cands.size(); ++i)
            if (cands[i].score > cands[best].score) best = (int)i;
    }
    return install_variant(c, cands[best].v, cands[best].lds);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

void exx_default_params(exx_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->fd_half_width = 3;
    p->l_max = 6;
    p->cg_rtol = 1e-10;
    p->cg_max_iter = 20000;
    p->precision = EXX_FP64;
    p->orbital_dtype = EXX_F64;
    p->guess = EXX_GUESS_ZERO;
    p->inner_rtol = 1e-5;
    p->autotune = 1;
}

exx_status exx_setup(const exx_params *p, int device, exx_ctx **out)
{
    if (!out) return fail(nullptr, EXX_EINVAL, "exx_setup: out is NULL");
    *out = nullptr;
    if (!p) return fail(nullptr, EXX_EINVAL, "exx_setup: params is NULL");
    for (int a = 0; a < 3; ++a) {
        if (p->n_grid[a] < 8 || p->n_grid[a] > 1000)
            return fail(nullptr, EXX_EINVAL, "n_grid[%d] = %d outside [8, 1000]", a, p->n_grid[a]);
        if (!(p->cell[a] > 0.0)) return fail(nullptr, EXX_EINVAL, "cell[%d] must be positive", a);
    }
    if (p->fd_half_width != 3) return fail(nullptr, EXX_EINVAL, "only fd_half_width = 3 is implemented");
    if (p->l_max != 6) return fail(nullptr, EXX_EINVAL, "only l_max = 6 is implemented");
    if (!(p->r_pair > 0.0)) return fail(nullptr, EXX_EINVAL, "r_pair must be positive");
    if (!(p->cg_rtol > 0.0) || p->cg_max_iter < 1) return fail(nullptr, EXX_EINVAL, "cg_rtol > 0 and cg_max_iter >= 1 required");
    if (p->precision != EXX_FP64 && p->precision != EXX_FP32_REFINE)
        return fail(nullptr, EXX_EINVAL, "unknown precision %d", p->precision);
    if (p->orbital_dtype != EXX_F64 && p->orbital_dtype != EXX_F32)
        return fail(nullptr, EXX_EINVAL, "unknown orbital_dtype %d", p->orbital_dtype);
    if (p->guess < EXX_GUESS_ZERO || p->guess > EXX_GUESS_LEARNED)
        return fail(nullptr, EXX_EINVAL, "unknown guess %d", p->guess);
    if (p->precond != EXX_PRECOND_NONE && p->precond != EXX_PRECOND_MG)
        return fail(nullptr, EXX_EINVAL, "unknown precond %d", p->precond);
    for (int a = 0; a < 3; ++a)
        if (p->box_dims[a] < 0 || p->box_dims[a] > p->n_grid[a])
            return fail(nullptr, EXX_EINVAL, "box_dims[%d] = %d outside [0, n_grid]", a, p->box_dims[a]);
    if (p->precision == EXX_FP32_REFINE && !(p->inner_rtol > 0.0 && p->inner_rtol < 1.0))
        return fail(nullptr, EXX_EINVAL, "inner_rtol must lie in (0, 1)");
    double hmax = 0.0;
    for (int a = 0; a < 3; ++a) hmax = std::max(hmax, p->cell[a] / p->n_grid[a]);
    if (p->n_classes != 0 && (p->n_classes < 2 || p->n_classes > EXX_MAX_CLASSES))
        return fail(nullptr, EXX_EINVAL, "n_classes = %d: 0 or 2..%d", p->n_classes, EXX_MAX_CLASSES);
    const bool classed = p->n_classes >= 2;
    if (classed && !(p->omega_scale > 0.0 && std::isfinite(p->omega_scale)))
        return fail(nullptr, EXX_EINVAL, "omega_scale must be positive");
    const int ncls = classed ? p->n_classes : 2;
    double rpe[KMAX], rme[KMAX];
    for (int c = 0; c < ncls; ++c) {
        rpe[c] = classed ? p->class_r_pe[c] : p->r_pe[c];
        rme[c] = classed ? p->class_r_me[c] : p->r_me[c];
        const char *pn = classed ? "class_" : "";
        if (!(rpe[c] > 0.0)) return fail(nullptr, EXX_EINVAL, "%sr_pe[%d] must be positive", pn, c);
        if (rme[c] - rpe[c] < 3 * hmax * (1.0 - 1e-12))
            return fail(nullptr, EXX_EINVAL, "%sr_me[%d] - %sr_pe[%d] = %g < n max(h) = %g", pn, c, pn, c,
                        rme[c] - rpe[c], 3 * hmax);
        if (classed && c > 0 && !(rpe[c] > rpe[c - 1]))
            return fail(nullptr, EXX_EINVAL, "class_r_pe must be strictly ascending");
    }
    if (device < 0) return fail(nullptr, EXX_EINVAL, "device %d is negative", device);
    exx_ctx *c = new (std::nothrow) exx_ctx();
    if (!c) return fail(nullptr, EXX_ENOMEM, "host allocation failed");
    c->prm = *p;
    c->device = device;
    auto bail = [&](exx_status st) {
        std::snprintf(g_setup_error, sizeof g_setup_error, "%s", c->err);
        exx_destroy(c);
        return st;
    };
    try {
        // the proto-subdomain tables first: they need no device
        for (int a = 0; a < 3; ++a) {
            c->h[a] = p->cell[a] / p->n_grid[a];
            c->c0[a] = (int)nint_away(0.5 * p->n_grid[a]);
            c->box[a] = p->box_dims[a] > 0 ? p->box_dims[a] : p->n_grid[a];
        }
        c->box_vol = (long long)c->box[0] * c->box[1] * c->box[2];
        c->n_cls = ncls;
        for (int k = 0; k < ncls; ++k) {
            exx_status st = build_class(c, c->cls[k], rpe[k], rme[k]);
            if (st != EXX_OK) return bail(st);
        }
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
            return bail(fail(c, EXX_EDEVICE, "no HIP device available"));
        if (device >= ndev) return bail(fail(c, EXX_EINVAL, "device %d out of range [0, %d)", device, ndev));
        if (hipSetDevice(device) != hipSuccess) return bail(fail(c, EXX_EDEVICE, "hipSetDevice(%d) failed", device));
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) != hipSuccess)
            return bail(fail(c, EXX_EDEVICE, "hipGetDeviceProperties failed"));
        c->n_cu = prop.multiProcessorCount;
        if (hipDeviceGetAttribute(&c->clock_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess)
            c->clock_khz = 0;
        {
            void *sp = nullptr;
            if (static_scratch_for(device, &sp) != hipSuccess)
                return bail(fail(c, EXX_EDEVICE, "hipGetSymbolAddress of the static CG scratch failed"));
        }
        for (int k = 0; k < ncls; ++k) {
            exx_status st = upload_class(c, c->cls[k]);
            if (st != EXX_OK) return bail(st);
            if (p->precond == EXX_PRECOND_MG && (st = build_mg_levels(c, c->cls[k])) != EXX_OK) return bail(st);
        }
        {
            exx_status st = select_variant(c);
            if (st != EXX_OK) return bail(st);
        }
        for (auto &e : c->ev)
            if (hipEventCreate(&e) != hipSuccess) return bail(fail(c, EXX_EDEVICE, "hipEventCreate failed"));
        c->have_events = true;
    } catch (const std::bad_alloc &) {
        return bail(fail(c, EXX_ENOMEM, "exx_setup: host allocation failed"));
    } catch (...) {
        return bail(fail(c, EXX_EDEVICE, "exx_setup: unexpected C++ exception"));
    }
    c->state = 1;
    *out = c;
    return EXX_OK;
}

// The pair list and origins (Step II, Step III) on the GPU: the host bins the
// centres into a periodic cell list (cells at least R_pair wide, with a
// relative margin of 1e-9 so rounding in the binning cannot separate a pair
// by two cells), the kernels count, fill and sort each orbital's partners.
exx_status build_pair_list(exx_ctx *c, int n_orb, const double *C)
{
    const double *L = c->prm.cell;
    PairArgs a{};
    a.n_orb = n_orb;
    for (int k = 0; k < 3; ++k) {
        a.L[k] = L[k];
        a.h[k] = c->h[k];
        a.N[k] = c->prm.n_grid[k];
        a.nc[k] = std::max(1, (int)std::floor(L[k] / (c->prm.r_pair * (1.0 + 1e-9))));
        a.nc[k] = std::min(a.nc[k], 1024);
    }
    // at most about 8 cells per orbital (wider cells only add candidates)
    while ((long long)a.nc[0] * a.nc[1] * a.nc[2] > 8LL * n_orb + 64) {
        int k = 0;
        for (int d = 1; d < 3; ++d)
            if (a.nc[d] > a.nc[k]) k = d;
        a.nc[k] = std::max(1, a.nc[k] / 2);
    }
    a.r2 = c->prm.r_pair * c->prm.r_pair;
    const int ncell = a.nc[0] * a.nc[1] * a.nc[2];
    std::vector<int> cell_of((size_t)n_orb), start((size_t)ncell + 1, 0), items((size_t)n_orb);
    for (int i = 0; i < n_orb; ++i) {
        int ci[3];
        for (int k = 0; k < 3; ++k) {
            const double u = C[3 * i + k] - L[k] * std::floor(C[3 * i + k] / L[k]);
            ci[k] = std::min(std::max((int)(u / (L[k] / a.nc[k])), 0), a.nc[k] - 1);
        }
        cell_of[i] = (ci[2] * a.nc[1] + ci[1]) * a.nc[0] + ci[0];
        start[cell_of[i] + 1]++;
    }
    for (int k = 0; k < ncell; ++k) start[k + 1] += start[k];
    {
        std::vector<int> fill(start.begin(), start.end() - 1);
        for (int i = 0; i < n_orb; ++i) items[fill[cell_of[i]]++] = i;
    }
    exx_status st;
    if ((st = dev_reserve(c, c->d_pC, (size_t)3 * n_orb)) != EXX_OK) return st;
    if ((st = dev_reserve(c, c->d_cell_of, (size_t)n_orb)) != EXX_OK) return st;
    if ((st = dev_reserve(c, c->d_cell_start, (size_t)ncell + 1)) != EXX_OK) return st;
    if ((st = dev_reserve(c, c->d_cell_items, (size_t)n_orb)) != EXX_OK) return st;
    if ((st = dev_reserve(c, c->d_pcount, (size_t)n_orb)) != EXX_OK) return st;
    if ((st = dev_reserve(c, c->d_pstart, (size_t)n_orb)) != EXX_OK) return st;
    HIPCHK(c, hipMemcpy(c->d_pC.p, C, sizeof(double) * 3 * n_orb, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_cell_of.p, cell_of.data(), sizeof(int) * n_orb, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_cell_start.p, start.data(), sizeof(int) * (ncell + 1), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_cell_items.p, items.data(), sizeof(int) * n_orb, hipMemcpyHostToDevice));
    a.C = c->d_pC.p;
    a.cell_of = c->d_cell_of.p;
    a.cell_start = c->d_cell_start.p;
    a.cell_items = c->d_cell_items.p;
    a.count = c->d_pcount.p;
    HIPCHK(c, launch_pair_count(a, 0));
    std::vector<int> cnt((size_t)n_orb);
    HIPCHK(c, hipMemcpy(cnt.data(), c->d_pcount.p, sizeof(int) * n_orb, hipMemcpyDeviceToHost));
    std::vector<long long> pst((size_t)n_orb);
    long long np = 0;
    for (int i = 0; i < n_orb; ++i) {
        pst[i] = np;
        np += cnt[i];
    }
    if (np > (long long)INT32_MAX) return fail(c, EXX_EINVAL, "%lld pairs exceed the supported 2^31 - 1", np);
    if ((st = dev_reserve(c, c->d_pij, (size_t)np)) != EXX_OK) return st;
    if ((st = dev_reserve(c, c->d_pgc, (size_t)np)) != EXX_OK) return st;
    HIPCHK(c, hipMemcpy(c->d_pstart.p, pst.data(), sizeof(long long) * n_orb, hipMemcpyHostToDevice));
    a.start = c->d_pstart.p;
    a.ij = c->d_pij.p;
    a.gc = c->d_pgc.p;
    HIPCHK(c, launch_pair_fill(a, 0));
    c->ij.resize((size_t)np);
    c->gc.resize((size_t)np);
    HIPCHK(c, hipMemcpy(c->ij.data(), c->d_pij.p, sizeof(int2) * np, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(c->gc.data(), c->d_pgc.p, sizeof(int4) * np, hipMemcpyDeviceToHost));
    return EXX_OK;
}

// Alg. 1: the unique pair list Lu refined from the non-unique list L0, as
// the owner of every pair.  A pair (i, j), i != j, is redundant while both
// row i and row j of L0 list it; a sweep takes the orbitals in index order
// and each orbital claims the nearest pair of its own that is still
// redundant (the partner's row drops it); sweeps repeat until one claims
// nothing.  Here each pair has an owner slot, -1 while it is redundant;
// each orbital's pairs are kept in ascending squared minimum-image distance
// of the partner, ties by partner index (the row order of L0).
void unique_pair_owners(exx_ctx *c)
{
    const int n = c->n_orb;
    const size_t np = c->ij.size();
    const double *L = c->prm.cell;
    // each orbital's non-self pairs, as (d^2, partner, pair)
    std::vector<int> rs((size_t)n + 1, 0);
    for (const int2 &q : c->ij)
        if (q.y != q.x) {
            rs[q.x + 1]++;
            rs[q.y + 1]++;
        }
    for (int i = 0; i < n; ++i) rs[i + 1] += rs[i];
    struct Ent { double d2; int j; int p; };
    std::vector<Ent> mine((size_t)rs[n]);
    c->owner.assign(np, -1);
    {
        std::vector<int> fill(rs.begin(), rs.end() - 1);
        for (size_t p = 0; p < np; ++p) {
            const int i = c->ij[p].x, j = c->ij[p].y;
            if (i == j) {
                c->owner[p] = i;          // a self pair is never redundant
                continue;
            }
            double dd = 0.0;
            for (int a = 0; a < 3; ++a) {
                double v = c->centers[3 * j + a] - c->centers[3 * i + a];
                v -= L[a] * (double)nint_away(v / L[a]);
                dd += v * v;
            }
            mine[fill[i]++] = Ent{dd, j, (int)p};
            mine[fill[j]++] = Ent{dd, i, (int)p};
        }
    }
    for (int i = 0; i < n; ++i)
        std::sort(mine.begin() + rs[i], mine.begin() + rs[i + 1], [](const Ent &u, const Ent &v) {
            return u.d2 < v.d2 || (u.d2 == v.d2 && u.j < v.j);
        });
    int sweeps = 0;
    for (bool claimed = true; claimed;) {
        claimed = false;
        ++sweeps;
        for (int i = 0; i < n; ++i)
            for (int t = rs[i]; t < rs[i + 1]; ++t)
                if (c->owner[mine[t].p] < 0) {
                    c->owner[mine[t].p] = i;
                    claimed = true;
                    break;
                }
    }
    c->owner_sweeps = sweeps;
}

// Radius the PE sphere about the pair origin g needs to hold the pair domain
// Omega_ij = Omega_i cap Omega_j (balls of radius omega_scale * spread about
// the centres): |g - c| + rho for the smallest ball (c, rho) enclosing the
// lens, in the cases the header lists; 0 for an empty domain.
double pair_domain_radius(const exx_ctx *c, int i, int j, const int4 &g, const double *C, const double *spr)
{
    const double *L = c->prm.cell;
    const double Ri = c->prm.omega_scale * spr[i], Rj = c->prm.omega_scale * spr[j];
    const int gg[3] = {g.x, g.y, g.z};
    double d[3], o[3], dd = 0.0;
    for (int a = 0; a < 3; ++a) {
        double v = C[3 * j + a] - C[3 * i + a];
        v -= L[a] * (double)nint_away(v / L[a]);
        d[a] = v;
        dd += v * v;
        double w = (double)gg[a] * c->h[a] - C[3 * i + a];
        w -= L[a] * (double)nint_away(w / L[a]);
        o[a] = w;
    }
    const double dist = std::sqrt(dd);
    double f = 0.0, rho;                 // lens centre at C_i + f (C_j - C_i)
    if (i == j) {
        rho = Ri;
    } else if (dist >= Ri + Rj) {
        return 0.0;
    } else if (dist == 0.0) {
        rho = std::min(Ri, Rj);
    } else {
        const double x = (dd + Ri * Ri - Rj * Rj) / (2.0 * dist);
        if (x <= 0.0) {
            rho = Ri;
        } else if (x >= dist) {
            f = 1.0;
            rho = Rj;
        } else {
            f = x / dist;
            rho = std::sqrt(Ri * Ri - x * x);
        }
    }
    double e2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double u = o[a] - f * d[a];
        e2 += u * u;
    }
    return std::sqrt(e2) + rho;
}

exx_status pairs_common(exx_ctx *c, int32_t n_orb, const double *C, const double *spreads, int64_t *n_pairs)
{
    if (c->state < 1) return fail(c, EXX_ESTATE, "exx_pairs before exx_setup");
    if (n_orb < 1 || !C) return fail(c, EXX_EINVAL, "exx_pairs: need n_orb >= 1 and centers");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, EXX_EDEVICE, "hipSetDevice failed");
    const double *L = c->prm.cell;
    const int *N = c->prm.n_grid;
    for (int i = 0; i < 3 * n_orb; ++i)
        if (!std::isfinite(C[i])) return fail(c, EXX_EINVAL, "centre coordinate %d is not finite", i);
    c->out_off.clear();
    c->rhs_off.clear();
    c->owner.clear();
    c->centers.assign(C, C + 3 * (size_t)n_orb);
    {
        exx_status st = build_pair_list(c, n_orb, C);
        if (st != EXX_OK) return st;
    }
    c->n_self = n_orb;
    c->n_pairs = (int64_t)c->ij.size();
    c->class_capped = 0;
    if (spreads) {
        // per-pair classes: the smallest class whose PE sphere covers Omega_ij
        for (size_t p = 0; p < c->ij.size(); ++p) {
            const double r = pair_domain_radius(c, c->ij[p].x, c->ij[p].y, c->gc[p], C, spreads);
            int k = 0;
            while (k < c->n_cls && c->cls[k].r_pe < r) ++k;
            if (k == c->n_cls) {
                k = c->n_cls - 1;
                ++c->class_capped;
            }
            c->gc[p].w = k;
        }
        if (c->tune_on_pairs) {
            std::vector<int64_t> mix(KMAX, 0);
            for (const int4 &q : c->gc) ++mix[q.w];
            exx_status st = select_variant(c, mix.data());
            if (st != EXX_OK) return st;
        }
    }
    c->n_orb = n_orb;
    // orbital boxes: origin = nearest grid point of the centre minus half the
    // box; a box as wide as the grid has origin 0
    c->box_org.assign((size_t)n_orb, int4{0, 0, 0, 0});
    for (int i = 0; i < n_orb; ++i) {
        int o[3];
        for (int a = 0; a < 3; ++a) {
            if (c->box[a] >= N[a]) { o[a] = 0; continue; }
            double m = C[3 * i + a] - L[a] * std::floor(C[3 * i + a] / L[a]);
            o[a] = mod_pos(nint_away(m / c->h[a]) - c->box[a] / 2, N[a]);
        }
        c->box_org[i] = int4{o[0], o[1], o[2], 0};
    }
    // every ME sphere must lie inside the boxes of both its orbitals, or D
    // would be cut off
    for (size_t p = 0; p < c->ij.size(); ++p) {
        const HostClass &k = c->cls[c->gc[p].w];
        const int lo[3] = {k.mxlo, k.mylo, k.mzlo}, ext[3] = {k.mxhi - k.mxlo + 1, k.myhi - k.mylo + 1, k.mzhi - k.mzlo + 1};
        const int gp[3] = {c->gc[p].x, c->gc[p].y, c->gc[p].z};
        for (int side = 0; side < 2; ++side) {
            const int orb = side ? c->ij[p].y : c->ij[p].x;
            const int oo[3] = {c->box_org[orb].x, c->box_org[orb].y, c->box_org[orb].z};
            for (int a = 0; a < 3; ++a) {
                if (c->box[a] >= N[a]) continue;
                const int start = mod_pos((long)gp[a] + lo[a] - oo[a], N[a]);
                if (start + ext[a] > c->box[a])
                    return fail(c, EXX_EINVAL,
                                "box_dims[%d] = %d is too small: the ME sphere of pair (%d, %d) leaves the box of "
                                "orbital %d",
                                a, c->box[a], c->ij[p].x, c->ij[p].y, orb);
            }
        }
    }
    c->orb_ptr.assign(n_orb + 1, 0);
    for (auto &q : c->ij) {
        c->orb_ptr[q.x + 1]++;
        if (q.y != q.x) c->orb_ptr[q.y + 1]++;
    }
    for (int i = 0; i < n_orb; ++i) c->orb_ptr[i + 1] += c->orb_ptr[i];
    c->orb_pairs.assign(c->orb_ptr[n_orb], 0);
    {
        std::vector<int> fill(c->orb_ptr.begin(), c->orb_ptr.end() - 1);
        for (int p = 0; p < (int)c->ij.size(); ++p) {
            c->orb_pairs[fill[c->ij[p].x]++] = p;
            if (c->ij[p].y != c->ij[p].x) c->orb_pairs[fill[c->ij[p].y]++] = p;
        }
    }
    exx_status st;
    if ((st = upload(c, c->d_ij, c->ij)) != EXX_OK) return st;
    if ((st = upload(c, c->d_gc, c->gc)) != EXX_OK) return st;
    if ((st = upload(c, c->d_orb_ptr, c->orb_ptr)) != EXX_OK) return st;
    if ((st = upload(c, c->d_orb_pairs, c->orb_pairs)) != EXX_OK) return st;
    if ((st = upload(c, c->d_box_org, c->box_org)) != EXX_OK) return st;
    const size_t np = (size_t)c->n_pairs;
    if ((st = dev_reserve(c, c->d_q, np * NLM)) != EXX_OK) return st;
    if ((st = dev_reserve(c, c->d_e, np)) != EXX_OK) return st;
    if ((st = dev_reserve(c, c->d_relres, np)) != EXX_OK) return st;
    if ((st = dev_reserve(c, c->d_iters, np)) != EXX_OK) return st;
    if ((st = dev_reserve(c, c->d_outer, np)) != EXX_OK) return st;
    if ((st = dev_reserve(c, c->d_conv, np)) != EXX_OK) return st;
    if ((st = dev_reserve(c, c->d_counter, 1)) != EXX_OK) return st;
    if ((st = dev_reserve(c, c->d_E, 1)) != EXX_OK) return st;
    // persistent grid and per-slot scratch
    int per_cu = 0;
    HIPCHK(c, cg_occupancy(c->var, cg_mode(c->prm.precision, c->prm.guess != EXX_GUESS_ZERO, c->prm.precond == EXX_PRECOND_MG), c->lds_bytes, &per_cu));
    per_cu = std::max(per_cu, 1);
    c->grid = (int)std::min<int64_t>(c->n_pairs, (int64_t)per_cu * c->n_cu);
    c->grid = std::max(c->grid, 1);
    c->slots = c->grid;
    // one spare element past the largest PE vector: the z-march kernels store
    // the values of unused lanes there
    c->slot_n = ((long long)c->cls[big_class(c)].n_pe + 1 + 63) / 64 * 64;
    if (c->prm.precision == EXX_FP32_REFINE) {
        if (!c->var.zmarch) return fail(c, EXX_EINVAL, "FP32 refinement needs a z-march CG kernel");
        if ((st = dev_reserve(c, c->d_scratch32, (size_t)c->slots * 4 * c->slot_n)) != EXX_OK) return st;
    }
    const bool mg = c->prm.precond == EXX_PRECOND_MG;
    if (mg && !c->var.zmarch) return fail(c, EXX_EINVAL, "the multigrid preconditioner needs a z-march CG kernel");
    if ((st = dev_reserve(c, c->d_scratch, (size_t)c->slots * (mg ? 4 : 3) * c->slot_n)) != EXX_OK) return st;
    if (mg && (st = dev_reserve(c, c->d_mg_scratch, (size_t)c->slots * mg_slot_doubles(c))) != EXX_OK)
        return st;
    // Waves of pairs: each wave holds its pairs' right-hand sides and
    // potentials, each pair at its own class's size.  One wave when
    // everything fits; otherwise D is summed wave by wave into FP64 partial
    // sums (so the result does not depend on the split) and the waves are as
    // large as the device allows.
    {
        size_t freeb = 0, totalb = 0;
        HIPCHK(c, hipMemGetInfo(&freeb, &totalb));
        // a pair's b takes its n_pe rounded up to 64 elements (512-byte aligned)
        auto rhs_len = [&](int64_t p) -> long long { return ((long long)c->cls[c->gc[p].w].n_pe + 63) / 64 * 64; };
        std::vector<size_t> pre((size_t)c->n_pairs + 1, 0);   // bytes of pairs [0, p)
        size_t small = SIZE_MAX;
        for (int64_t p = 0; p < c->n_pairs; ++p) {
            const HostClass &k = c->cls[c->gc[p].w];
            const size_t b = (size_t)(rhs_len(p) + k.n_pe + k.n_sh) * sizeof(double);
            pre[p + 1] = pre[p] + b;
            small = std::min(small, b);
        }
        // every wave of w consecutive pairs (the last may hold fewer) within cap
        auto fits = [&](int64_t w, size_t cap) {
            for (int64_t w0 = 0; w0 < c->n_pairs; w0 += w)
                if (pre[std::min<int64_t>(w0 + w, c->n_pairs)] - pre[w0] > cap) return false;
            return true;
        };
        const size_t have = (c->d_rhs.n + c->d_vout.n + c->d_dacc.n) * sizeof(double);
        // keep 2 GiB free, and room for the model or the guess history
        size_t keep = (size_t)2 << 30;
        if (c->prm.guess == EXX_GUESS_LEARNED) keep += (size_t)3 << 29;   // net activations
        if (c->prm.guess == EXX_GUESS_PREVIOUS || c->prm.guess == EXX_GUESS_EXTRAP) {
            size_t hist = 0;
            for (auto &q : c->gc) hist += (size_t)c->cls[q.w].n_pe * sizeof(float);
            size_t held = c->hist_next.v.n * sizeof(float);
            for (auto &h : c->hist) held += h.v.n * sizeof(float);
            const size_t levels = c->prm.guess == EXX_GUESS_PREVIOUS ? 2 : 4;   // kept + the one being written
            keep += levels * hist > held ? levels * hist - held : 0;
        }
        // dev_reserve adds 1/33 to large buffers: potentials, right-hand
        // sides and partial sums together get budget * 34/33 at most
        const size_t budget = freeb + have > keep ? (freeb + have - keep) / 34 * 33 : 0;
        const size_t dacc = (size_t)c->n_orb * c->box_vol * sizeof(double);
        int64_t w = c->n_pairs;
        if (!fits(w, budget)) {
            // from an upper bound down: w no larger than cap over the largest
            // pair's bytes fits, so this ends
            const size_t cap = budget > dacc ? budget - dacc : 0;
            w = std::min<int64_t>(c->n_pairs - 1, (int64_t)(cap / small));
            while (w > 0 && !fits(w, cap)) w = std::min<int64_t>(w - 1, w * 127 / 128);
        }
        if (c->prm.wave_pairs > 0) w = std::min<int64_t>(w, c->prm.wave_pairs);
        if (c->prm.keep_intermediates) w = c->n_pairs;
        w = std::min<int64_t>(w, c->n_pairs);
        if (w < 1) return fail(c, EXX_ENOMEM, "no device memory left for a wave of pairs");
        c->wave_n = (int)w;
        // potentials and right-hand sides: offsets relative to the pair's wave
        c->out_off.assign((size_t)c->n_pairs, 0);
        c->rhs_off.assign((size_t)c->n_pairs, 0);
        long long vmax = 0, bmax = 0;
        for (int64_t w0 = 0; w0 < c->n_pairs; w0 += w) {
            long long o = 0, ob = 0;
            for (int64_t p = w0; p < std::min<int64_t>(w0 + w, c->n_pairs); ++p) {
                c->out_off[p] = o;
                c->rhs_off[p] = ob;
                o += (long long)c->cls[c->gc[p].w].n_pe + c->cls[c->gc[p].w].n_sh;
                ob += rhs_len(p);
            }
            vmax = std::max(vmax, o);
            bmax = std::max(bmax, ob);
        }
        c->vout_n = vmax;
        if ((st = upload(c, c->d_off, c->out_off)) != EXX_OK) return st;
        if ((st = upload(c, c->d_rhs_off, c->rhs_off)) != EXX_OK) return st;
        // CG queue: within each wave the pairs of the larger classes first, so
        // that the longest solves do not start last and leave a tail where
        // most of the GPU idles.  Each pair's result does not depend on when
        // or where it is solved, so the order changes no value.
        c->queue.clear();
        bool mixed_sizes = false;
        for (int k = 1; k < c->n_cls; ++k) mixed_sizes |= c->cls[k].n_pe != c->cls[0].n_pe;
        if (mixed_sizes) {
            c->queue.resize((size_t)c->n_pairs);
            for (int64_t p = 0; p < c->n_pairs; ++p) c->queue[p] = (int)p;
            for (int64_t w0 = 0; w0 < c->n_pairs; w0 += w)
                std::stable_sort(c->queue.begin() + w0, c->queue.begin() + std::min<int64_t>(w0 + w, c->n_pairs),
                                 [&](int u, int v) { return c->cls[c->gc[u].w].n_pe > c->cls[c->gc[v].w].n_pe; });
            if ((st = upload(c, c->d_queue, c->queue)) != EXX_OK) return st;
        } else {
            dev_free(c->d_queue);
        }
        if ((st = dev_reserve(c, c->d_clock, (size_t)2 * ((c->n_pairs + w - 1) / w))) != EXX_OK) return st;
        if ((st = dev_reserve(c, c->d_vout, (size_t)vmax)) != EXX_OK) return st;
        if ((st = dev_reserve(c, c->d_rhs, (size_t)bmax)) != EXX_OK) return st;
        if (w < c->n_pairs) {
            if ((st = dev_reserve(c, c->d_dacc, (size_t)c->n_orb * c->box_vol)) != EXX_OK) return st;
        } else {
            dev_free(c->d_dacc);
        }
        if (c->prm.keep_intermediates &&
            (st = dev_reserve(c, c->d_rho_keep, (size_t)c->n_pairs * c->slot_n)) != EXX_OK)
            return st;
    }
    c->state = 2;
    ++c->pairs_gen;
    if (n_pairs) *n_pairs = c->n_pairs;
    return EXX_OK;
}

static exx_status exx_pairs_body(exx_ctx *c, int32_t n_orb, const double *C, int64_t *n_pairs)
{
    if (!c) return fail(nullptr, EXX_EINVAL, "exx_pairs: ctx is NULL");
    if (c->prm.n_classes >= 2) return fail(c, EXX_EINVAL, "n_classes >= 2: the pair classes need exx_pairs_spread");
    return pairs_common(c, n_orb, C, nullptr, n_pairs);
}

static exx_status exx_pairs_spread_body(exx_ctx *c, int32_t n_orb, const double *C, const double *spreads, int64_t *n_pairs)
{
    if (!c) return fail(nullptr, EXX_EINVAL, "exx_pairs_spread: ctx is NULL");
    if (c->prm.n_classes < 2) return fail(c, EXX_EINVAL, "exx_pairs_spread needs n_classes >= 2");
    if (!spreads || n_orb < 1) return fail(c, EXX_EINVAL, "exx_pairs_spread: need n_orb >= 1 and spreads");
    for (int i = 0; i < n_orb; ++i)
        if (!(spreads[i] >= 0.0) || !std::isfinite(spreads[i]))
            return fail(c, EXX_EINVAL, "spread %d is negative or not finite", i);
    return pairs_common(c, n_orb, C, spreads, n_pairs);
}

// exx_solve, or with fixed_scratch the allocation-free exx_solve_static: the
// CG work vectors in the device's fixed scratch array, the CG grid cut to the
// slots it holds, eager launches only, zero initial guess only.
static exx_status solve_impl(exx_ctx *c, const void *phi, void *stream, bool fixed_scratch)
{
    const char *who = fixed_scratch ? "exx_solve_static" : "exx_solve";
    if (!c) return fail(nullptr, EXX_EINVAL, "%s: ctx is NULL", who);
    if (c->state < 2) return fail(c, EXX_ESTATE, "%s before exx_pairs", who);
    if (!phi) return fail(c, EXX_EINVAL, "%s: phi is NULL", who);
    if (fixed_scratch && c->prm.guess != EXX_GUESS_ZERO)
        return fail(c, EXX_EINVAL, "exx_solve_static: only the zero initial guess (the other guesses allocate)");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    int cg_grid = c->grid;
    double *scr64 = c->d_scratch.p, *scr_mg = c->d_mg_scratch.p;
    float *scr32 = c->d_scratch32.p;
    if (fixed_scratch) {
        // per CG slot: the FP64 vectors, the FP32 vectors, the coarse levels,
        // each region 256-byte aligned
        const bool mg = c->prm.precond == EXX_PRECOND_MG;
        const bool mixed = c->prm.precision == EXX_FP32_REFINE;
        auto up256 = [](size_t b) { return (b + 255) / 256 * 256; };
        const size_t b64 = (size_t)(mg ? 4 : 3) * c->slot_n * sizeof(double);
        const size_t b32 = mixed ? (size_t)4 * c->slot_n * sizeof(float) : 0;
        const size_t bmg = mg ? (size_t)mg_slot_doubles(c) * sizeof(double) : 0;
        const size_t cap = static_scratch_bytes();
        const size_t need1 = up256(b64) + up256(b32) + up256(bmg);
        if (need1 > cap)
            return fail(c, EXX_EINVAL, "exx_solve_static: one CG slot needs %zu bytes, the fixed scratch holds %zu",
                        need1, cap);
        int slots = (int)std::min<size_t>((size_t)c->grid, cap / need1);
        while (slots > 1 && up256((size_t)slots * b64) + up256((size_t)slots * b32) + up256((size_t)slots * bmg) > cap)
            --slots;
        void *base = nullptr;
        if (static_scratch_for(c->device, &base) != hipSuccess || !base)
            return fail(c, EXX_EDEVICE, "exx_solve_static: no fixed scratch address on device %d", c->device);
        char *b = static_cast<char *>(base);
        scr64 = reinterpret_cast<double *>(b);
        scr32 = reinterpret_cast<float *>(b + up256((size_t)slots * b64));
        scr_mg = reinterpret_cast<double *>(b + up256((size_t)slots * b64) + up256((size_t)slots * b32));
        cg_grid = slots;
    }
    SolveArgs a{};
    for (int k = 0; k < c->n_cls; ++k) a.cls[k] = class_dev(c->cls[k]);
    a.pair_gc = c->d_gc.p;
    a.pair_ij = c->d_ij.p;
    a.out_off = c->d_off.p;
    a.queue = c->queue.empty() ? nullptr : c->d_queue.p;
    a.phi = phi;
    a.box = orb_box(c);
    a.phi_f32 = c->prm.orbital_dtype == EXX_F32;
    a.nx = c->prm.n_grid[0];
    a.ny = c->prm.n_grid[1];
    a.nz = c->prm.n_grid[2];
    a.ngrid = (long long)a.nx * a.ny * a.nz;
    a.vout = c->d_vout.p;
    a.scratch = scr64;
    a.scratch32 = scr32;
    a.rhs = c->d_rhs.p;
    a.rhs_off = c->d_rhs_off.p;
    a.rho_keep = c->prm.keep_intermediates ? c->d_rho_keep.p : nullptr;
    a.slot_n = c->slot_n;
    a.q_out = c->d_q.p;
    a.e_out = c->d_e.p;
    a.iters_out = c->d_iters.p;
    a.outer_out = c->d_outer.p;
    a.conv_out = c->d_conv.p;
    a.relres_out = c->d_relres.p;
    a.counter = c->d_counter.p;
    a.static_sched = 0;
    a.precision = c->prm.precision;
    for (int k = 0; k < 3; ++k) a.h[k] = c->h[k];
    for (int k = 0; k < 4; ++k) a.wfd[k] = kFD[k];
    a.tol = c->prm.cg_rtol;
    a.inner_tol = c->prm.inner_rtol;
    a.maxit = c->prm.cg_max_iter;
    ylm_norms(a.ylm_norm);
    mg_args(c, a, scr_mg);
    // initial guess from earlier steps: constant, linear or quadratic
    // extrapolation over the consecutive levels that hold the same (i, j);
    // or from the learned model
    const bool use_guess = c->prm.guess == EXX_GUESS_PREVIOUS || c->prm.guess == EXX_GUESS_EXTRAP;
    const bool learned = c->prm.guess == EXX_GUESS_LEARNED;
    if (learned && !c->net) return fail(c, EXX_ESTATE, "guess = EXX_GUESS_LEARNED needs a model (exx_model_init or exx_load_model)");
    a.guess = use_guess || learned ? 1 : 0;
    c->guess_pairs = learned ? (int)c->n_pairs : 0;
    NetPairArgs na{};
    if (learned) na = net_args(c);
    GuessArgs ga{};
    if (use_guess) {
        std::vector<PairGuess> tab((size_t)c->n_pairs);
        const int max_levels = c->prm.guess == EXX_GUESS_PREVIOUS ? 1 : 3;
        static const double coef[4][3] = {{0, 0, 0}, {1, 0, 0}, {2, -1, 0}, {3, -3, 1}};
        for (int64_t p = 0; p < c->n_pairs; ++p) {
            PairGuess &t = tab[p];
            const long long key = (long long)c->ij[p].x * c->n_orb + c->ij[p].y;
            int n = 0;
            for (int k = 0; k < max_levels; ++k) {
                t.off[k] = -1;
                t.shift[k] = int4{0, 0, 0, 0};
            }
            for (int k = 0; k < max_levels; ++k) {
                const exx_ctx::Hist &h = c->hist[k];
                if (!h.valid) break;
                auto it = h.index.find(key);
                if (it == h.index.end()) break;
                const int q = it->second;
                if (h.gc[q].w != c->gc[p].w) break;   // another class: another PE sphere
                t.off[k] = h.off[q];
                int sh[3] = {c->gc[p].x - h.gc[q].x, c->gc[p].y - h.gc[q].y, c->gc[p].z - h.gc[q].z};
                for (int d = 0; d < 3; ++d) {
                    const int N = c->prm.n_grid[d];
                    if (sh[d] > N / 2) sh[d] -= N;
                    if (sh[d] < -N / 2) sh[d] += N;
                }
                t.shift[k] = int4{sh[0], sh[1], sh[2], 1};
                ++n;
            }
            for (int k = max_levels; k < 3; ++k) {
                t.off[k] = -1;
                t.shift[k] = int4{0, 0, 0, 0};
            }
            for (int k = 0; k < 3; ++k) t.coef[k] = coef[n][k];
            if (n) ++c->guess_pairs;
        }
        exx_status st2 = upload_async(c, c->d_guess, tab, s, true);
        if (st2 != EXX_OK) return st2;
        for (int k = 0; k < c->n_cls; ++k) ga.cls[k] = a.cls[k];
        ga.pair_gc = c->d_gc.p;
        ga.out_off = c->d_off.p;
        ga.guess = c->d_guess.p;
        for (int k = 0; k < 3; ++k) ga.hist[k] = c->hist[k].valid ? c->hist[k].v.p : nullptr;
        ga.vout = c->d_vout.p;
    }
    c->n_waves = (int)((c->n_pairs + c->wave_n - 1) / c->wave_n);
    // the level this step's potentials go to (saved wave by wave)
    exx_ctx::Hist &nx = c->hist_next;
    if (use_guess) {
        nx.valid = false;
        nx.index.clear();
        nx.gc = c->gc;
        nx.off.assign((size_t)c->n_pairs, 0);
        long long tot = 0;
        for (int64_t p = 0; p < c->n_pairs; ++p) {
            nx.off[p] = tot;
            tot += c->cls[c->gc[p].w].n_pe;
            nx.index[(long long)c->ij[p].x * c->n_orb + c->ij[p].y] = (int)p;
        }
        exx_status st2 = dev_reserve(c, nx.v, (size_t)tot);
        if (st2 != EXX_OK) return st2;
        // nx.off lives until this level is recycled, after the copy completes
        if ((st2 = upload_async(c, c->d_hist_off, nx.off, s, false)) != EXX_OK) return st2;
    }
    const bool multi = c->n_waves > 1;
    DxxArgs dacc{};
    if (multi) dacc = dxx_args(c, phi, nullptr);
    // every launch of the solve, wave by wave; phase events only when eager
    auto enqueue = [&](hipStream_t st, bool events) -> hipError_t {
        hipError_t e;
        for (int64_t w0 = 0; w0 < c->n_pairs; w0 += c->wave_n) {
            a.wave_begin = (int)w0;
            a.wave_n = (int)std::min<int64_t>(c->wave_n, c->n_pairs - w0);
            if ((e = launch_prep(a, st)) != hipSuccess) return e;
            if (events && w0 == 0 && (e = hipEventRecord(c->ev[6], st)) != hipSuccess) return e;
            if (use_guess) {
                ga.wave_begin = a.wave_begin;
                if ((e = launch_guess(ga, a.wave_n, st)) != hipSuccess) return e;
            }
            if (learned) {
                na.wave_begin = a.wave_begin;
                if ((e = net_infer(c->net, na, a.wave_n, c->net_D, nullptr, st)) != hipSuccess) return e;
            }
            const size_t wi = (size_t)(w0 / c->wave_n);
            a.clock = c->d_clock.p + 2 * wi;
            if ((e = launch_wave_reset(c->d_counter.p, a.clock, st)) != hipSuccess) return e;
            if (events && w0 == 0 && (e = hipEventRecord(c->ev[5], st)) != hipSuccess) return e;
            if (events && (e = hipEventRecord(c->ev_cg[2 * wi], st)) != hipSuccess) return e;
            if ((e = launch_cg(c->var, a, std::min(cg_grid, a.wave_n), c->lds_bytes, st)) != hipSuccess) return e;
            if (events && (e = hipEventRecord(c->ev_cg[2 * wi + 1], st)) != hipSuccess) return e;
            if ((e = launch_pair_energy(a, st)) != hipSuccess) return e;
            if (use_guess &&
                (e = launch_save_history(c->d_vout.p, c->d_off.p, c->d_hist_off.p, c->d_gc.p,
                                         int4{c->cls[0].n_pe, c->cls[1].n_pe, c->cls[2].n_pe, c->cls[3].n_pe},
                                         a.wave_begin, a.wave_n, nx.v.p, st)) != hipSuccess)
                return e;
            if (multi) {
                // this wave's share of D, added to the partial sums in pair order
                dacc.pair_lo = a.wave_begin;
                dacc.pair_hi = a.wave_begin + a.wave_n;
                dacc.acc_first = w0 == 0;
                if ((e = launch_dxx(dacc, c->n_orb, 1, st)) != hipSuccess) return e;
            }
        }
        return hipSuccess;
    };
    // Graph mode (zero or learned guess): the launches are captured once on
    // the context's own stream and replayed while the pairs, phi and the
    // model's buffers are unchanged; the caller's stream and the graph
    // stream are ordered by events.
    c->last_graph = c->prm.graph && !use_guess && !fixed_scratch;
    if (c->last_graph) {
        if (!c->gstream) HIPCHK(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
        if (learned) HIPCHK(c, net_reserve(c->net, (int)std::min<int64_t>(c->wave_n, c->n_pairs), c->net_D));
        const unsigned long long net_gen = c->net ? net_generation(c->net) : 0;
        if (!c->gexec || c->g_pairs_gen != c->pairs_gen || c->g_phi != phi || c->g_net_gen != net_gen ||
            c->g_learned != learned) {
            if (c->gexec) { (void)hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
            HIPCHK(c, hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
            const hipError_t e1 = enqueue(c->gstream, false);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(c->gstream, &g);
            HIPCHK(c, e1);
            HIPCHK(c, e2);
            const hipError_t e3 = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIPCHK(c, e3);
            c->g_pairs_gen = c->pairs_gen;
            c->g_phi = phi;
            c->g_net_gen = net_gen;
            c->g_learned = learned;
            ++c->graph_builds;
        }
        HIPCHK(c, hipEventRecord(c->ev[0], s));
        HIPCHK(c, hipStreamWaitEvent(c->gstream, c->ev[0], 0));
        HIPCHK(c, hipGraphLaunch(c->gexec, c->gstream));
        HIPCHK(c, hipEventRecord(c->ev[1], c->gstream));
        HIPCHK(c, hipStreamWaitEvent(s, c->ev[1], 0));
        ++c->graph_launches;
    } else {
        // per-wave CG events (created once; the allocation-free solve uses
        // them only when an earlier exx_solve has created enough)
        const bool cg_events = !fixed_scratch || c->ev_cg.size() >= (size_t)2 * c->n_waves;
        while (!fixed_scratch && c->ev_cg.size() < (size_t)2 * c->n_waves) {
            hipEvent_t e = nullptr;
            HIPCHK(c, hipEventCreate(&e));
            c->ev_cg.push_back(e);
        }
        HIPCHK(c, hipEventRecord(c->ev[0], s));
        HIPCHK(c, enqueue(s, cg_events));
        HIPCHK(c, hipEventRecord(c->ev[1], s));
    }
    c->last_grid = cg_grid;
    c->last_cg_timed = !c->last_graph && (!fixed_scratch || c->ev_cg.size() >= (size_t)2 * c->n_waves);
    if (use_guess) {
        // rotate the ring: this step's level becomes the most recent; the
        // PREVIOUS guess keeps one level, the extrapolations three
        const int levels = c->prm.guess == EXX_GUESS_PREVIOUS ? 1 : 3;
        exx_ctx::Hist spare = std::move(c->hist[levels - 1]);
        for (int k = levels - 1; k > 0; --k) c->hist[k] = std::move(c->hist[k - 1]);
        c->hist[0] = std::move(nx);
        c->hist[0].valid = true;
        c->hist_next = std::move(spare);
        c->hist_next.valid = false;
    }
    c->phi = phi;
    c->state = 3;
    c->solved_once = true;
    return EXX_OK;
}

static exx_status exx_energy_potential_body(exx_ctx *c, double *e_xx, void *dxx, void *stream)
{
    if (!c) return fail(nullptr, EXX_EINVAL, "exx_energy_potential: ctx is NULL");
    if (c->state < 3) return fail(c, EXX_ESTATE, "exx_energy_potential before exx_solve");
    if (!e_xx || !dxx) return fail(c, EXX_EINVAL, "exx_energy_potential: e_xx and dxx are required");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const DxxArgs d = dxx_args(c, c->phi, dxx);
    HIPCHK(c, hipEventRecord(c->ev[2], s));
    if (c->n_waves > 1)
        HIPCHK(c, launch_dxx_final(d, c->n_orb, s));   // D was summed wave by wave during the solve
    else
        HIPCHK(c, launch_dxx(d, c->n_orb, 0, s));
    HIPCHK(c, hipEventRecord(c->ev[3], s));
    HIPCHK(c, launch_energy(c->d_e.p, c->d_ij.p, (int)c->n_pairs, c->d_E.p, s));
    HIPCHK(c, hipEventRecord(c->ev[4], s));
    HIPCHK(c, hipMemcpyAsync(e_xx, c->d_E.p, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    // convergence flags
    std::vector<int> conv((size_t)c->n_pairs);
    HIPCHK(c, hipMemcpy(conv.data(), c->d_conv.p, conv.size() * sizeof(int), hipMemcpyDeviceToHost));
    for (size_t k = 0; k < conv.size(); ++k)
        if (!conv[k]) return fail(c, EXX_ENOCONV, "pair %zu did not converge in %d iterations", k, c->prm.cg_max_iter);
    return EXX_OK;
}

static exx_status exx_stats_body(exx_ctx *c, exx_stats_t *st)
{
    if (!c || !st) return fail(c, EXX_EINVAL, "exx_stats: null argument");
    std::memset(st, 0, sizeof *st);
    st->n_pairs = c->n_pairs;
    st->n_self = c->n_self;
    st->solve_grid = c->solved_once ? c->last_grid : c->grid;
    st->solve_block = c->block;
    st->cg_cols = c->var.zmarch ? c->var.cols : 0;
    st->cg_inflight[0] = c->var.pf64;
    st->cg_inflight[1] = c->var.pf32;
    st->cg_cols32 = c->var.zmarch ? c->var.cols32 : 0;
    st->cg_bands[0] = (int)c->cls[0].bands.size() / 12;
    st->cg_bands[1] = (int)c->cls[1].bands.size() / 12;
    for (int k = 0; k < 2; ++k) {
        st->n_pe[k] = c->cls[k].n_pe;
        st->n_me[k] = c->cls[k].n_pe + c->cls[k].n_sh;
    }
    st->n_classes = c->n_cls;
    for (int k = 0; k < c->n_cls; ++k) {
        st->class_n_pe[k] = c->cls[k].n_pe;
        st->class_n_me[k] = c->cls[k].n_pe + c->cls[k].n_sh;
    }
    for (const int4 &q : c->gc) st->class_pairs[q.w]++;
    st->class_capped = c->class_capped;
    st->device_bytes = (int64_t)(c->d_vout.n * 8 + c->d_scratch.n * 8 + c->d_scratch32.n * 4 + c->d_q.n * 8 +
                                 c->d_rhs.n * 8 + c->d_rho_keep.n * 8);
    if (c->state < 3) return EXX_OK;
    HIPCHK(c, hipSetDevice(c->device));
    const size_t np = (size_t)c->n_pairs;
    std::vector<int> it(np), cv(np), ou(np);
    std::vector<double> rr(np);
    HIPCHK(c, hipMemcpy(it.data(), c->d_iters.p, np * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(ou.data(), c->d_outer.p, np * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(cv.data(), c->d_conv.p, np * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(rr.data(), c->d_relres.p, np * sizeof(double), hipMemcpyDeviceToHost));
    st->iters_min = np ? it[0] : 0;
    const int sphi = c->prm.orbital_dtype == EXX_F32 ? 4 : 8;
    const int scg = c->prm.precision == EXX_FP32_REFINE ? 4 : 8;
    const bool mg = c->prm.precond == EXX_PRECOND_MG;
    for (size_t p = 0; p < np; ++p) {
        const HostClass &k = c->cls[c->gc[p].w];
        st->iters_total += it[p];
        st->outer_total += ou[p];
        st->iters_min = std::min(st->iters_min, it[p]);
        st->iters_max = std::max(st->iters_max, it[p]);
        st->n_not_converged += cv[p] ? 0 : 1;
        st->relres_max = std::max(st->relres_max, rr[p]);
        // algorithmic bytes per unknown: 8 vector passes per CG iteration,
        // 32 B per FP64 residual pass (x, b, d in; x, r out) and 16 B for the
        // closing residual pass (x, b in); the pair energy reads x and the
        // two orbitals, the preparation the two orbitals (and writes b and
        // the shell potential)
        // With the multigrid preconditioner an iteration moves 72 B per
        // unknown (r, x FP64; the dense residual, z, p FP32): smoothing
        // passes 12 (r in, the dense residual out) and 12 (r in, z out; r at
        // the output plane is recovered from the cached coarse correction),
        // direction 12 (z, p in, p out), update 36 (p, x, r in, x, r out; the
        // kernel pairs the iterate updates and moves 30 on average); plus the
        // V-cycle's bytes per coarse cell in the domain.
        // In FP32 (FP32_REFINE) the preconditioned iteration moves 50 B per
        // unknown: smoothing passes 8 (r in, the dense residual out) and 8
        // (r in, z out; r at the output plane is kept in registers),
        // direction 12, update 22 (p, r in, r out FP32; x FP64 every other
        // iteration; the previous p every other); the V-cycle in FP32; each
        // residual replacement 20 (x, b in, r out) and the owed step it folds
        // into x first 20 (x in and out, p in), counted on every replacement.
        int64_t per_it, per_outer;
        if (mg && scg == 4) {
            per_it = (int64_t)k.n_pe * 50 + k.mg_cells_bytes32;
            per_outer = 40;
        } else if (mg) {
            per_it = (int64_t)k.n_pe * 72 + k.mg_cells_bytes;
            per_outer = 32;
        } else {
            per_it = (int64_t)k.n_pe * 8 * scg;
            per_outer = 32;
        }
        const int64_t cg = (int64_t)it[p] * per_it + (int64_t)k.n_pe * ((int64_t)ou[p] * per_outer + 16);
        st->cg_bytes += cg;
        st->solve_bytes += cg + (int64_t)k.n_pe * (2 * sphi + 8) + (int64_t)k.n_sh * 8 + (int64_t)k.n_pe * (8 + 2 * sphi);
        const int m = c->ij[p].x == c->ij[p].y ? 1 : 2;
        st->dxx_bytes += (int64_t)m * (k.n_pe + k.n_sh) * (8 + sphi);
    }
    st->dxx_bytes += (int64_t)c->n_orb * c->box_vol * sphi;
    float ms = 0.f;
    st->n_waves = c->n_waves;
    st->wave_n = c->wave_n;
    if (hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess) st->solve_ms = ms;
    st->prep_ms = st->cg_ms = st->guess_ms = -1.0;
    st->guess_pairs = c->guess_pairs;
    st->tuned = c->tuned;
    st->tune_ms = c->tune_ms;
    st->graph_builds = c->graph_builds;
    st->graph_launches = c->graph_launches;
    if (c->n_waves == 1 && !c->last_graph) {
        if (hipEventElapsedTime(&ms, c->ev[0], c->ev[6]) == hipSuccess) st->prep_ms = ms;
        if (hipEventElapsedTime(&ms, c->ev[6], c->ev[5]) == hipSuccess) st->guess_ms = ms;
    }
    if (c->last_cg_timed && c->ev_cg.size() >= (size_t)2 * c->n_waves) {
        double tot = 0.0;
        bool ok = true;
        for (int w = 0; w < c->n_waves && ok; ++w) {
            ok = hipEventElapsedTime(&ms, c->ev_cg[2 * w], c->ev_cg[2 * w + 1]) == hipSuccess;
            tot += ms;
        }
        if (ok) st->cg_ms = tot;   // the persistent CG kernel alone, summed over waves
    }
    st->cg_clock_ms = -1.0;
    if (c->clock_khz > 0 && c->d_clock.p && c->n_waves > 0) {
        std::vector<unsigned long long> ck((size_t)2 * c->n_waves);
        if (hipMemcpy(ck.data(), c->d_clock.p, ck.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost) ==
            hipSuccess) {
            double tot = 0.0;
            bool ok = true;
            for (int w = 0; w < c->n_waves; ++w) {
                ok = ok && ck[2 * w + 1] >= ck[2 * w];
                tot += (double)(ck[2 * w + 1] - ck[2 * w]);
            }
            if (ok) st->cg_clock_ms = tot / c->clock_khz;
        }
    }
    if (hipEventElapsedTime(&ms, c->ev[2], c->ev[3]) == hipSuccess) st->dxx_ms = ms;
    if (hipEventElapsedTime(&ms, c->ev[3], c->ev[4]) == hipSuccess) st->energy_ms = ms;
    // a timing that is not available (an event not recorded in this mode)
    // must not leave its error behind for the next launch check
    (void)hipGetLastError();
    return EXX_OK;
}

static exx_status exx_pair_class_body(exx_ctx *c, int32_t *cls)
{
    if (!c) return fail(nullptr, EXX_EINVAL, "exx_pair_class: ctx is NULL");
    if (c->state < 2) return fail(c, EXX_ESTATE, "exx_pair_class before exx_pairs");
    if (!cls) return fail(c, EXX_EINVAL, "exx_pair_class: cls is NULL");
    for (size_t p = 0; p < c->gc.size(); ++p) cls[p] = c->gc[p].w;
    return EXX_OK;
}

static exx_status exx_pair_owners_body(exx_ctx *c, int32_t *owner, int32_t *sweeps)
{
    if (!c) return fail(nullptr, EXX_EINVAL, "exx_pair_owners: ctx is NULL");
    if (c->state < 2) return fail(c, EXX_ESTATE, "exx_pair_owners before exx_pairs");
    if (!owner) return fail(c, EXX_EINVAL, "exx_pair_owners: owner is NULL");
    if (c->owner.size() != c->ij.size()) unique_pair_owners(c);
    std::copy(c->owner.begin(), c->owner.end(), owner);
    if (sweeps) *sweeps = c->owner_sweeps;
    return EXX_OK;
}

static exx_status exx_pair_info_body(exx_ctx *c, int32_t *pi, int32_t *pj, int32_t *origin, double *e, int32_t *iters,
                         int32_t *converged, double *relres)
{
    if (!c) return fail(nullptr, EXX_EINVAL, "exx_pair_info: ctx is NULL");
    if (c->state < 2) return fail(c, EXX_ESTATE, "exx_pair_info before exx_pairs");
    const size_t np = (size_t)c->n_pairs;
    for (size_t p = 0; p < np; ++p) {
        if (pi) pi[p] = c->ij[p].x;
        if (pj) pj[p] = c->ij[p].y;
        if (origin) { origin[3 * p] = c->gc[p].x; origin[3 * p + 1] = c->gc[p].y; origin[3 * p + 2] = c->gc[p].z; }
    }
    if (e || iters || converged || relres) {
        if (c->state < 3) return fail(c, EXX_ESTATE, "exx_pair_info: no solve yet");
        HIPCHK(c, hipSetDevice(c->device));
        HIPCHK(c, hipDeviceSynchronize());
        if (e) HIPCHK(c, hipMemcpy(e, c->d_e.p, np * sizeof(double), hipMemcpyDeviceToHost));
        if (iters) HIPCHK(c, hipMemcpy(iters, c->d_iters.p, np * sizeof(int), hipMemcpyDeviceToHost));
        if (converged) HIPCHK(c, hipMemcpy(converged, c->d_conv.p, np * sizeof(int), hipMemcpyDeviceToHost));
        if (relres) HIPCHK(c, hipMemcpy(relres, c->d_relres.p, np * sizeof(double), hipMemcpyDeviceToHost));
    }
    return EXX_OK;
}

static exx_status exx_debug_pair_body(exx_ctx *c, int64_t pair, double *v_pe, double *v_shell, double *q_lm, double *rho,
                          double *rhs)
{
    if (!c) return fail(nullptr, EXX_EINVAL, "exx_debug_pair: ctx is NULL");
    if (c->state < 3) return fail(c, EXX_ESTATE, "exx_debug_pair: no solve yet");
    if (pair < 0 || pair >= c->n_pairs) return fail(c, EXX_EINVAL, "pair %lld out of range", (long long)pair);
    if ((rho || rhs) && !c->prm.keep_intermediates)
        return fail(c, EXX_ESTATE, "exx_debug_pair: intermediates were not kept (keep_intermediates = 0)");
    if ((v_pe || v_shell) && c->n_waves > 1 && pair < (int64_t)(c->n_waves - 1) * c->wave_n)
        return fail(c, EXX_ESTATE, "exx_debug_pair: the potentials of pair %lld were released with its wave",
                    (long long)pair);
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipDeviceSynchronize());
    const HostClass &k = c->cls[c->gc[pair].w];
    const double *v = c->d_vout.p + c->out_off[pair];
    if (v_pe) HIPCHK(c, hipMemcpy(v_pe, v, (size_t)k.n_pe * 8, hipMemcpyDeviceToHost));
    if (v_shell) HIPCHK(c, hipMemcpy(v_shell, v + k.n_pe, (size_t)k.n_sh * 8, hipMemcpyDeviceToHost));
    if (q_lm) HIPCHK(c, hipMemcpy(q_lm, c->d_q.p + pair * NLM, NLM * 8, hipMemcpyDeviceToHost));
    if (rho) HIPCHK(c, hipMemcpy(rho, c->d_rho_keep.p + (size_t)pair * c->slot_n, (size_t)k.n_pe * 8, hipMemcpyDeviceToHost));
    if (rhs) HIPCHK(c, hipMemcpy(rhs, c->d_rhs.p + c->rhs_off[pair], (size_t)k.n_pe * 8, hipMemcpyDeviceToHost));
    return EXX_OK;
}

static exx_status exx_model_init_body(exx_ctx *c, int32_t coarsen, uint64_t seed)
{
    if (!c) return fail(nullptr, EXX_EINVAL, "exx_model_init: ctx is NULL");
    if (coarsen != 2 && coarsen != 4 && coarsen != 8)
        return fail(c, EXX_EINVAL, "coarsen must be 2, 4 or 8 (got %d)", coarsen);
    HIPCHK(c, hipSetDevice(c->device));
    net_destroy(c->net);
    c->net = nullptr;
    hipError_t e = hipSuccess;
    ExxNet *net = net_create(coarsen, (unsigned long long)seed, &e);
    if (e != hipSuccess) {
        net_destroy(net);
        return fail(c, e == hipErrorOutOfMemory ? EXX_ENOMEM : EXX_EDEVICE, "model allocation: %s", hipGetErrorString(e));
    }
    c->net = net;
    c->net_D = net_edge(coarsen, pe_rmax(c));
    for (int k = 0; k < c->n_cls; ++k)
        if (!c->d_bnd[k].p) {
            exx_status st = dev_reserve(c, c->d_bnd[k], (size_t)c->cls[k].n_pe);
            if (st != EXX_OK) return st;
            HIPCHK(c, net_boundary_flags(class_dev(c->cls[k]), c->d_bnd[k].p, 0));
        }
    HIPCHK(c, hipDeviceSynchronize());
    return EXX_OK;
}

static exx_status exx_load_model_body(exx_ctx *c, const void *weights, size_t bytes)
{
    if (!c) return fail(nullptr, EXX_EINVAL, "exx_load_model: ctx is NULL");
    const int f = net_blob_coarsen(weights, bytes);
    if (f < 0)
        return fail(c, EXX_EINVAL, "exx_load_model: not a model blob of %zu bytes (got %zu)", net_model_bytes(), bytes);
    exx_status st = exx_model_init(c, f, 0);
    if (st != EXX_OK) return st;
    hipError_t e = hipSuccess;
    if (net_load(c->net, weights, bytes, &e) != 0)
        return fail(c, EXX_EDEVICE, "exx_load_model: %s", hipGetErrorString(e));
    return EXX_OK;
}

static exx_status exx_model_save_body(exx_ctx *c, void *buf, size_t *bytes)
{
    if (!c) return fail(nullptr, EXX_EINVAL, "exx_model_save: ctx is NULL");
    if (!bytes) return fail(c, EXX_EINVAL, "exx_model_save: bytes is NULL");
    if (!c->net) return fail(c, EXX_ESTATE, "exx_model_save: no model");
    const size_t need = net_model_bytes();
    if (!buf) {
        *bytes = need;
        return EXX_OK;
    }
    if (*bytes < need) return fail(c, EXX_EINVAL, "exx_model_save: buffer of %zu bytes, need %zu", *bytes, need);
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipDeviceSynchronize());
    HIPCHK(c, net_save(c->net, buf));
    *bytes = need;
    return EXX_OK;
}

static exx_status exx_model_train_body(exx_ctx *c, int32_t epochs, int32_t batch, double lr, uint64_t seed, double *loss,
                           void *stream)
{
    if (!c) return fail(nullptr, EXX_EINVAL, "exx_model_train: ctx is NULL");
    if (!c->net) return fail(c, EXX_ESTATE, "exx_model_train: no model (exx_model_init or exx_load_model)");
    if (c->state < 3) return fail(c, EXX_ESTATE, "exx_model_train before exx_solve");
    // the pairs whose right-hand sides and potentials are still resident:
    // every pair, or the last wave's when the solve ran in waves
    const int64_t w0 = c->n_waves > 1 ? (int64_t)(c->n_waves - 1) * c->wave_n : 0;
    const int64_t nt = c->n_pairs - w0;
    if (epochs < 0 || batch < 1 || batch > nt || !(lr > 0.0 || epochs == 0) || !loss)
        return fail(c, EXX_EINVAL, "exx_model_train: need epochs >= 0, 1 <= batch <= %lld (resident pairs), lr > 0, loss",
                    (long long)nt);
    HIPCHK(c, hipSetDevice(c->device));
    std::vector<int> pairs((size_t)nt);
    for (int64_t p = 0; p < nt; ++p) pairs[p] = (int)(w0 + p);
    NetPairArgs na = net_args(c);
    na.wave_begin = (int)w0;
    HIPCHK(c, net_train(c->net, na, pairs.data(), (int)nt, c->net_D, epochs, batch, (float)lr,
                        (unsigned long long)seed, loss, (hipStream_t)stream));
    return EXX_OK;
}

static exx_status exx_model_conv_body(exx_ctx *c, int32_t layer, int32_t transposed, const void *x, float *y, int32_t n,
                          int32_t edge, void *stream)
{
    if (!c) return fail(nullptr, EXX_EINVAL, "exx_model_conv: ctx is NULL");
    if (!c->net) return fail(c, EXX_ESTATE, "exx_model_conv: no model");
    int cin = 0, cout = 0;
    if (net_layer_dims(layer, &cin, &cout) != 0) return fail(c, EXX_EINVAL, "layer %d out of range", layer);
    if (!x || !y || n < 1 || edge < 1 || (long long)n * edge * edge * edge > (1LL << 30))
        return fail(c, EXX_EINVAL, "exx_model_conv: need x, y, n >= 1, 1 <= edge, n edge^3 <= 2^30");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, net_conv_test(c->net, layer, transposed, x, y, n, edge, (hipStream_t)stream));
    return EXX_OK;
}

static exx_status exx_model_wgrad_body(exx_ctx *c, int32_t layer, const void *x, const void *dy, float *dw, int32_t n,
                           int32_t edge, void *stream)
{
    if (!c) return fail(nullptr, EXX_EINVAL, "exx_model_wgrad: ctx is NULL");
    if (!c->net) return fail(c, EXX_ESTATE, "exx_model_wgrad: no model");
    int cin = 0, cout = 0;
    if (net_layer_dims(layer, &cin, &cout) != 0) return fail(c, EXX_EINVAL, "layer %d out of range", layer);
    if (!x || !dy || !dw || n < 1 || edge < 1 || (long long)n * edge * edge * edge > (1LL << 30))
        return fail(c, EXX_EINVAL, "exx_model_wgrad: need x, dy, dw, n >= 1, 1 <= edge, n edge^3 <= 2^30");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, net_wgrad_test(c->net, layer, x, dy, dw, n, edge, (hipStream_t)stream));
    return EXX_OK;
}

static exx_status exx_box_origins_body(exx_ctx *c, int32_t *origins)
{
    if (!c) return fail(nullptr, EXX_EINVAL, "exx_box_origins: ctx is NULL");
    if (!origins) return fail(c, EXX_EINVAL, "exx_box_origins: origins is NULL");
    if (c->state < 2) return fail(c, EXX_ESTATE, "exx_box_origins before exx_pairs");
    for (int i = 0; i < c->n_orb; ++i) {
        origins[3 * i] = c->box_org[i].x;
        origins[3 * i + 1] = c->box_org[i].y;
        origins[3 * i + 2] = c->box_org[i].z;
    }
    return EXX_OK;
}

// Every entry point that takes a context: nothing thrown inside (a host
// allocation that fails, say) crosses the C ABI; it becomes a status.
exx_status exx_pairs(exx_ctx *c, int32_t n_orb, const double *C, int64_t *n_pairs)
{
    EXX_GUARDED(c, exx_pairs_body(c, n_orb, C, n_pairs));
}

exx_status exx_pairs_spread(exx_ctx *c, int32_t n_orb, const double *C, const double *spreads, int64_t *n_pairs)
{
    EXX_GUARDED(c, exx_pairs_spread_body(c, n_orb, C, spreads, n_pairs));
}

exx_status exx_solve(exx_ctx *c, const void *phi, void *stream)
{
    EXX_GUARDED(c, solve_impl(c, phi, stream, false));
}

exx_status exx_solve_static(exx_ctx *c, const void *phi, void *stream)
{
    EXX_GUARDED(c, solve_impl(c, phi, stream, true));
}

exx_status exx_energy_potential(exx_ctx *c, double *e_xx, void *dxx, void *stream)
{
    EXX_GUARDED(c, exx_energy_potential_body(c, e_xx, dxx, stream));
}

exx_status exx_stats(exx_ctx *c, exx_stats_t *st)
{
    EXX_GUARDED(c, exx_stats_body(c, st));
}

exx_status exx_pair_class(exx_ctx *c, int32_t *cls)
{
    EXX_GUARDED(c, exx_pair_class_body(c, cls));
}

exx_status exx_pair_owners(exx_ctx *c, int32_t *owner, int32_t *sweeps)
{
    EXX_GUARDED(c, exx_pair_owners_body(c, owner, sweeps));
}

exx_status exx_pair_info(exx_ctx *c, int32_t *pi, int32_t *pj, int32_t *origin, double *e, int32_t *iters,
                         int32_t *converged, double *relres)
{
    EXX_GUARDED(c, exx_pair_info_body(c, pi, pj, origin, e, iters, converged, relres));
}

exx_status exx_debug_pair(exx_ctx *c, int64_t pair, double *v_pe, double *v_shell, double *q_lm, double *rho,
                          double *rhs)
{
    EXX_GUARDED(c, exx_debug_pair_body(c, pair, v_pe, v_shell, q_lm, rho, rhs));
}

exx_status exx_model_init(exx_ctx *c, int32_t coarsen, uint64_t seed)
{
    EXX_GUARDED(c, exx_model_init_body(c, coarsen, seed));
}

exx_status exx_load_model(exx_ctx *c, const void *weights, size_t bytes)
{
    EXX_GUARDED(c, exx_load_model_body(c, weights, bytes));
}

exx_status exx_model_save(exx_ctx *c, void *buf, size_t *bytes)
{
    EXX_GUARDED(c, exx_model_save_body(c, buf, bytes));
}

exx_status exx_model_train(exx_ctx *c, int32_t epochs, int32_t batch, double lr, uint64_t seed, double *loss,
                           void *stream)
{
    EXX_GUARDED(c, exx_model_train_body(c, epochs, batch, lr, seed, loss, stream));
}

exx_status exx_model_conv(exx_ctx *c, int32_t layer, int32_t transposed, const void *x, float *y, int32_t n,
                          int32_t edge, void *stream)
{
    EXX_GUARDED(c, exx_model_conv_body(c, layer, transposed, x, y, n, edge, stream));
}

exx_status exx_model_wgrad(exx_ctx *c, int32_t layer, const void *x, const void *dy, float *dw, int32_t n,
                           int32_t edge, void *stream)
{
    EXX_GUARDED(c, exx_model_wgrad_body(c, layer, x, dy, dw, n, edge, stream));
}

exx_status exx_box_origins(exx_ctx *c, int32_t *origins)
{
    EXX_GUARDED(c, exx_box_origins_body(c, origins));
}

int32_t exx_model_edge(const exx_ctx *c) { return c && c->net ? c->net_D : 0; }

const char *exx_last_error(const exx_ctx *c) { return c ? c->err : g_setup_error; }

void exx_destroy(exx_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto &k : c->cls) free_class(k);
    dev_free(c->d_ij); dev_free(c->d_gc); dev_free(c->d_off); dev_free(c->d_rhs_off); dev_free(c->d_queue); dev_free(c->d_orb_ptr); dev_free(c->d_orb_pairs);
    dev_free(c->d_vout); dev_free(c->d_q); dev_free(c->d_e); dev_free(c->d_relres); dev_free(c->d_scratch);
    dev_free(c->d_rhs); dev_free(c->d_rho_keep);
    dev_free(c->d_guess); dev_free(c->d_hist_off);
    for (auto &h : c->hist) dev_free(h.v);
    dev_free(c->hist_next.v);
    dev_free(c->d_box_org); dev_free(c->d_dacc);
    net_destroy(c->net);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    for (auto &b : c->d_bnd) dev_free(b);
    dev_free(c->d_pC); dev_free(c->d_cell_of); dev_free(c->d_cell_start); dev_free(c->d_cell_items);
    dev_free(c->d_pcount); dev_free(c->d_pstart); dev_free(c->d_pij); dev_free(c->d_pgc);
    dev_free(c->d_mg_scratch);
    dev_free(c->d_E); dev_free(c->d_iters); dev_free(c->d_outer); dev_free(c->d_conv); dev_free(c->d_counter); dev_free(c->d_scratch32);
    dev_free(c->d_clock);
    if (c->have_events)
        for (auto &e : c->ev)
            if (e) (void)hipEventDestroy(e);
    for (auto &e : c->ev_cg) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"
