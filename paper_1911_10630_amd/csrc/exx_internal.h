// exx_internal.h -- structures shared by the host code and the HIP kernels of
// the pair-Poisson exact-exchange library (library-internal, not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace exx {

constexpr int LMAX = 6;                      // multipole order (Eq. me)
constexpr int NLM = (LMAX + 1) * (LMAX + 1); // 49 real harmonics
constexpr int FD_N = 3;                      // stencil half-width (Eq. d2_1)
constexpr int KMAX = 4;                      // subdomain classes (pair.w indexes them)

// Local offsets (grid units, |o| < 512) packed into one int: 10 bits per axis.
__host__ __device__ inline int pack_xyz(int x, int y, int z)
{
    return (x + 512) | ((y + 512) << 10) | ((z + 512) << 20);
}
__host__ __device__ inline void unpack_xyz(int v, int &x, int &y, int &z)
{
    x = (v & 1023) - 512;
    y = ((v >> 10) & 1023) - 512;
    z = ((v >> 20) & 1023) - 512;
}

// Device view of one proto-subdomain class (PE sphere + ME shell).
//
// PE storage ("row-packed"): rows (z, y) of the sphere in z-major, y-minor
// order, each row the contiguous x run [xlo, xhi]; element (x, y, z) lives
// at base(z, y) + x - xlo(z, y).  This is exactly the z, y, x lexicographic
// order of Alg. 2, so local index q of Eq. rbar equals the packed index.
// Shell storage: the same lexicographic order over shell points; a shell
// row (z, y) holds the run [mlo, plo-1] then [phi+1, mhi].
struct ClassDev {
    const int4 *pe_rows;   // [pnz][pny] {base, xlo, xhi, 0}; empty row: xlo > xhi
    const int4 *me_rows;   // [mnz][mny][2] {pe_base, plo, phi, sh_base}, {mlo, mhi, 0, 0};
                           // a row outside ME has mlo > mhi
    const int *pe_xyz;     // [n_pe] packed offsets
    const int *sh_xyz;     // [n_sh] packed offsets
    const int *cols;       // [n_cols] packed (x, y, 0) of the PE projection, sorted (y, x)
    int n_cols;
    const int *colz;       // [n_cols] z range of each column: (zlo + 512) | (zhi + 512) << 16
    const int *pe_off;     // [pnz][pny] base(z, y) - xlo(z, y): packed index of (x, y, z) = pe_off + x
    const int *bnd_q;      // [n_bnd] PE points with a stencil neighbour on the shell, ascending
    const int *bnd_ptr;    // [n_bnd + 1] their runs in bnd_ent
    const int *bnd_ent;    // shell neighbours: (shell index << 4) | (axis * 3 + s - 1)
    int n_bnd;
    const int *bands;      // [n_bands][12] z-march bands: own cols [c0,c1), halo cols
                           // [h0,h1) u [h2,h3), planes [zlo, zhi], first own row ya
    int n_bands;
    const int *bands32;    // bands of the FP32 passes (more columns per thread)
    int n_bands32;
    int tbl_ints;          // LDS ints holding pe_off (pnz * pny rounded up to 4)
    int lds_w, lds_plane;  // z-march LDS plane: row pitch pnx + 6, plane_rows * lds_w
    int plane_rows;        // own rows of the widest band + 6
    int lds_plane32;       // plane size of the FP32 bands
    int pxlo, pylo, pzlo, pnx, pny, pnz;   // PE bounding box
    int mxlo, mylo, mzlo, mnx, mny, mnz;   // ME bounding box
    int n_pe, n_sh;
};

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

// Orbital storage: orbital k lives on the periodic box [org_k, org_k + b)
// of the grid, layout [n_orb][bz][by][bx], x fastest; outside its box an
// orbital is zero.  The whole grid is the box with org = 0, b = N.
// v in [-n, 2n) wrapped into [0, n)
__device__ __forceinline__ int wrap_n(int v, int n)
{
    v = v < 0 ? v + n : v;
    return v >= n ? v - n : v;
}

struct OrbBox {
    const int4 *org;            // [n_orb] box origin (grid point)
    int bx, by, bz;
    long long vol;              // bx * by * bz
};

// Value of orbital k (base = k * vol, origin o) at grid point (gx, gy, gz).
// Branch-free: points outside the box load element 0 and select zero.
__device__ __forceinline__ double load_orb(const void *phi, int f32, const OrbBox &B, long long base, int4 o, int gx,
                                           int gy, int gz, int nx, int ny, int nz)
{
    int lx = gx - o.x, ly = gy - o.y, lz = gz - o.z;
    lx += lx < 0 ? nx : 0;
    ly += ly < 0 ? ny : 0;
    lz += lz < 0 ? nz : 0;
    const bool in = lx < B.bx && ly < B.by && lz < B.bz;
    const long long idx = in ? base + ((long long)lz * B.by + ly) * B.bx + lx : 0;
    const double v = f32 ? (double)static_cast<const float *>(phi)[idx] : static_cast<const double *>(phi)[idx];
    return in ? v : 0.0;
}

// Multigrid preconditioner: coarse levels of one subdomain class, each a
// dense box of cells (level 1 cell c covers the fine offsets
// plo + 2c + {0, 1} per axis, level l + 1 cell C the level-l cells
// 2C + {0, 1}).  cm[c] has bit kx + 2 ky + 4 kz set when child (kx, ky, kz)
// lies in the domain of the finer level (PE for level 1); a cell is in the
// domain when cm[c] != 0.
constexpr int MG_MAX = 6;
struct MgLevel {
    int nx, ny, nz;
    const unsigned char *cm;    // [nz][ny][nx] child bits
    long long off;              // f, e, t at off, off + n, off + 2n of a slot's coarse scratch
};
struct MgClass {
    int levels;
    MgLevel lv[MG_MAX];
    long long dense_off;        // the fine residual on the PE box padded to even
                                // edges, [2 nz1][2 ny1][2 nx1], then one sink element
};

struct SolveArgs {
    ClassDev cls[KMAX];
    const int4 *pair_gc;        // [n_pairs] {gx, gy, gz, class}
    const int2 *pair_ij;        // [n_pairs] {i, j}
    const long long *out_off;   // [n_pairs] offset of the pair's v in vout (relative to its wave)
    const int *queue;           // [n_pairs] pair taken at each CG queue position (a permutation
                                // within each wave, largest class first), or null: pair order
    const void *phi;            // [n_orb][bz][by][bx] on the orbital boxes
    OrbBox box;
    int phi_f32;
    int nx, ny, nz;
    long long ngrid;
    double *vout;               // per pair: v on PE (n_pe) then v on shell (n_sh)
    double *rhs;                // per wave pair: right-hand side b (n_pe, padded)
    const long long *rhs_off;   // [n_pairs] offset of the pair's b in rhs (relative to its wave)
    double *rho_keep;           // optional per pair: pair density (slot_n each)
    double *scratch;            // per CG slot: r, p, Ap (slot_n each)
    long long slot_n;           // elements per array (max n_pe, padded)
    float *scratch32;           // per CG slot: FP32 work vectors (refinement)
    double *q_out;              // [n_pairs][NLM]
    double *e_out;              // [n_pairs]
    int *iters_out;             // [n_pairs] CG iterations (FP32 refinement: inner total)
    int *outer_out;             // [n_pairs] FP64 residual passes (refinement)
    int *conv_out;              // [n_pairs]
    double *relres_out;         // [n_pairs]
    int *counter;               // dynamic pair queue (wave-relative)
    unsigned long long *clock;  // or null: {first start, last end} of the CG launch,
                                // device wall clock (k_wave_reset initializes it)
    int wave_begin, wave_n;     // pairs [wave_begin, wave_begin + wave_n)
    int static_sched;           // 1: pair = block + k*grid, slot = block
    int guess;                  // 0 zero, 1 v already in vout (previous step)
    int precision;              // 0 FP64, 1 FP32 inner + FP64 refinement
    double h[3];
    double wfd[4];              // central-difference weights w_0..w_3
    double tol;                 // relative residual target
    double inner_tol;           // FP32 inner solve target
    int maxit;
    double ylm_norm[NLM];       // normalization of the real solid harmonics
    // multigrid-preconditioned CG (FP64): two more fine vectors per slot
    // (scratch holds 5 per slot) and per-slot coarse arrays
    int mg;
    MgClass mgc[KMAX];          // coarse levels per class
    double *mg_scratch;         // per slot: mg_slot_n doubles
    long long mg_slot_n;
    double mg_omega;            // damping of the fine Jacobi smoother
    double mg_omega_c;          // damping of the coarse Jacobi smoother
    int mg_coarse_sweeps;       // Jacobi sweeps on the coarsest level
    double mg_coarse_scale;     // scale of the coarse correction reaching the fine level
};

// Initial guess of one pair from up to three earlier steps (Sec. III.C Step IV:
// polynomial extrapolation of the potential from previous MD steps).
struct PairGuess {
    long long off[3];   // offset of the earlier PE solution in its history level, or -1
    int4 shift[3];      // origin(now) - origin(then), minimum image, in grid points
    double coef[3];     // extrapolation weights
};

struct GuessArgs {
    ClassDev cls[KMAX];
    const int4 *pair_gc;
    const long long *out_off;
    const PairGuess *guess;    // [n_pairs]
    const float *hist[3];      // history levels (most recent first)
    double *vout;
    int wave_begin;
};

struct DxxArgs {
    ClassDev cls[KMAX];
    const int4 *pair_gc;
    const int2 *pair_ij;
    const long long *out_off;
    const int *orb_ptr;         // [n_orb + 1] CSR over orbitals
    const int *orb_pairs;       // pair indices, ascending per orbital
    const void *phi;
    OrbBox box;
    void *dxx;                  // [n_orb][bz][by][bx]
    double *acc;                // FP64 partial sums across waves (accumulating form)
    int acc_first;              // 1: the first wave (partial sums start at 0)
    int pair_lo, pair_hi;       // pairs of this wave
    int f32;
    int nx, ny, nz;
    long long ngrid;
    const double *vout;
};

// Launchers (exx_kernels.hip).
hipError_t launch_prep(const SolveArgs &a, hipStream_t s);
// e_ij = h^3 sum rho x for the pairs of the wave (after their CG).
hipError_t launch_pair_energy(const SolveArgs &a, hipStream_t s);

// Pair list (exx_pairs.hip): centres binned into a periodic cell list with
// cells at least R_pair wide; count[i] = 1 + partners j > i within R_pair;
// the fill writes, from start[i], the self pair and the partners in
// ascending j with their origins and classes.
struct PairArgs {
    const double *C;            // [n_orb][3] centres
    int n_orb;
    double L[3], h[3];
    double r2;                  // R_pair^2
    int N[3];
    int nc[3];                  // cells per axis
    const int *cell_of;         // [n_orb]
    const int *cell_start;      // [cells + 1]
    const int *cell_items;      // orbital indices grouped by cell
    int *count;                 // [n_orb]
    const long long *start;     // [n_orb]
    int2 *ij;                   // [n_pairs]
    int4 *gc;                   // [n_pairs] {gx, gy, gz, class}
};
hipError_t launch_pair_count(const PairArgs &a, hipStream_t s);
hipError_t launch_pair_fill(const PairArgs &a, hipStream_t s);
// Persistent CG kernels: "flat" (any sphere) and "zmarch" (register queue,
// needs the LDS plane to fit).  Variants are (block, columns per thread).
struct CgVariant {
    int zmarch;   // 0 flat, 1 z-march
    int block;    // threads per work-group
    int cols;     // FP64 columns per thread per band (z-march)
    int halo;     // FP64 halo columns per thread (z-march)
    int cols32;   // FP32 columns per thread (refinement passes)
    int halo32;   // FP32 halo columns per thread
    int wpe;      // minimum resident waves per SIMD the kernel is compiled for
    int pf64;     // planes of loads in flight in the FP64 passes (1 or 2)
    int pf32;     // planes of loads in flight in the FP32 passes (1 or 2)
    int modes;    // bit mask of the kernel modes it is built for
};
int cg_variants(CgVariant *out, int max_n);
// Whether a variant is built for a mode.
bool cg_variant_applies(const CgVariant &v, int mode);
// Kernel mode for a precision (EXX_FP64 / EXX_FP32_REFINE), whether CG
// starts from a guess in vout, and the multigrid preconditioner (in FP64, or
// in FP32 with FP64 residual replacement under EXX_FP32_REFINE).
int cg_mode(int precision, int guess, int mg);
hipError_t cg_occupancy(const CgVariant &v, int mode, size_t lds_bytes, int *blocks_per_cu);
hipError_t launch_cg(const CgVariant &v, const SolveArgs &a, int grid, size_t lds_bytes, hipStream_t s);
// D from the pairs [pair_lo, pair_hi): written to dxx (accumulate = 0) or
// added to the FP64 partial sums acc (accumulate = 1); launch_dxx_final
// converts acc to dxx.
hipError_t launch_dxx(const DxxArgs &a, int n_orb, int accumulate, hipStream_t s);
hipError_t launch_dxx_final(const DxxArgs &a, int n_orb, hipStream_t s);
hipError_t launch_energy(const double *e, const int2 *ij, int n_pairs, double *out, hipStream_t s);
hipError_t launch_zero_int(int *p, int n, hipStream_t s);
// Before a CG launch: its queue counter to 0 and its clock pair to
// {max, 0} (a kernel, so that it can be captured into a graph).
hipError_t launch_wave_reset(int *counter, unsigned long long *clock, hipStream_t s);
hipError_t launch_guess(const GuessArgs &a, int n_pairs, hipStream_t s);
hipError_t launch_save_history(const double *vout, const long long *out_off, const long long *hist_off,
                               const int4 *pair_gc, int4 n_pe, int wave_begin, int wave_n, float *hist,
                               hipStream_t s);

// Fixed device scratch of the allocation-free solve (exx_kernels.hip): its
// size, and its device address on the current device.
size_t static_scratch_bytes();
hipError_t static_scratch_address(void **ptr);

// Learned initial guess (exx_net.hip).  The net reads a pair's right-hand
// side on a coarse cube (coarsening factor f, edge D coarse cells, fine
// offsets [-fD/2, fD/2) per axis) and writes its PE guess into vout.
struct NetPairArgs {
    ClassDev cls[KMAX];         // subdomain classes (unused ones have n_pe = 0)
    const int4 *pair_gc;
    const long long *out_off;
    const double *rhs;          // right-hand sides of the wave
    const long long *rhs_off;   // [n_pairs] offset of the pair's b in rhs (relative to its wave)
    int wave_begin;
    double *vout;               // read (training targets) or written (guess)
    double h2;                  // output scale: RMS(v) ~ RMS(b) h^2
    const unsigned char *bnd[KMAX];// per class, per PE point: 1 if the stencil leaves PE
};

struct ExxNet;
// Fresh net with He-initialized weights; coarsening factor f (2, 4 or 8).
ExxNet *net_create(int f, unsigned long long seed, hipError_t *err);
void net_destroy(ExxNet *net);
int net_coarsen(const ExxNet *net);
// Coarse edge for PE offsets |o| <= r_max: f D / 2 >= r_max + 1, D a multiple of 8.
int net_edge(int f, int r_max);
// flag[q] = 1 for PE points whose stencil leaves PE (n_pe bytes).
hipError_t net_boundary_flags(const ClassDev &g, unsigned char *flag, hipStream_t s);
// Device bytes of the activation buffers for `batch` samples of edge D
// (training adds the gradient buffers).
size_t net_buffer_bytes(int batch, int D, bool training);
// Allocates the inference buffers for waves of n pairs (nothing if they exist).
hipError_t net_reserve(ExxNet *net, int n, int D);
// Changes whenever the model's device buffers are reallocated.
unsigned long long net_generation(const ExxNet *net);
// Guess for pairs [wave_begin, wave_begin + n) of the wave in a.
hipError_t net_infer(ExxNet *net, const NetPairArgs &a, int n, int D, double *ms, hipStream_t s);
// Adam epochs over the given pairs (their rhs and solutions must be resident).
hipError_t net_train(ExxNet *net, const NetPairArgs &a, const int *pairs, int n_pairs, int D, int epochs, int batch,
                     float lr, unsigned long long seed, double *loss, hipStream_t s);
size_t net_model_bytes();
hipError_t net_save(ExxNet *net, void *host);
// Returns 0, or -1 for a malformed blob (header or size), or -2 on a device error (*err).
int net_load(ExxNet *net, const void *host, size_t bytes, hipError_t *err);
int net_blob_coarsen(const void *host, size_t bytes);
// One forward convolution of layer l (or its input-gradient form) on given
// bf16 input [N][D^3][Cin], FP32 output [N][D^3][Cout]; for tests.
hipError_t net_conv_test(ExxNet *net, int l, int transposed, const void *x, float *y, int N, int D, hipStream_t s);
// Weight gradient of layer l for given bf16 x and dy, FP32 [27][Cout][Cin]; for tests.
hipError_t net_wgrad_test(ExxNet *net, int l, const void *x, const void *dy, float *dw, int N, int D, hipStream_t s);
int net_layer_dims(int l, int *cin, int *cout);

}  // namespace exx
