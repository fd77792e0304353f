/*
 * exx_oracle.c -- plain, slow, FP64 CPU oracle for the pair-Poisson path of
 * the localized-orbital exact-exchange method of Ko, Jia, Santra, Wu, Car and
 * DiStasio, "Enabling large-scale condensed-phase hybrid DFT based AIMD I"
 * (arXiv:1911.10630).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP library.
 *
 * Every step follows the paper in its own order and notation, with no
 * blocking, fusion or reordering:
 *   - pair criterion |C_i - C_j| < R_pair under the minimum image (Sec. III.C
 *     Step II, and the parameter definitions opening Sec. IV);
 *   - proto-subdomains PE and ME around the grid point C_0 nearest the cell
 *     centre, built by looping over the grid (Alg. 2, Eqs. rbar and g0);
 *   - pair origin C_ij = (C_i + C_j)/2 snapped to the nearest grid point and
 *     local-to-global index map g = MOD(g0 + tau, N) (Sec. III.C Step III,
 *     Eq. l2g);
 *   - pair density on PE, multipole moments Q_lm with complex Y_lm, l <= 6
 *     (Eq. mepole), far-field potential on the ME shell (Eq. me);
 *   - 6th-order central-difference Laplacian (Eq. d2_1) restricted to PE with
 *     the shell values folded into the right-hand side as a boundary charge
 *     (Eq. pe_mat_red), solved by unpreconditioned conjugate gradient;
 *   - pair energy integrated over PE (Sec. III.C Step V, Eq. exx_omega) and
 *     D^ij = v_ij phi_j, D^ji = v_ij phi_i accumulated over the whole ME
 *     sphere (Eq. Dxx_mlwf_omega, Step V).
 *
 * Readings where the paper is silent (listed with reasons in the design
 * notes): unordered pairs weighted 2 in E for i != j; NINT rounds half away
 * from zero; MOD is the non-negative modulo; a grid point is inside radius R
 * iff sum_a (o_a h_a)^2 <= R^2 (1 + 1e-12); CG stops on the relative 2-norm
 * of the recursive residual ||r|| <= tol ||b|| starting from x = 0.
 *
 * Units: bohr and hartree.  Grid layout: [Nz][Ny][Nx], x fastest, 0-based.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define O_LMAX 6
#define O_NLM ((O_LMAX + 1) * (O_LMAX + 1))

/* Central-difference weights for the second derivative, n = 3 (Eq. d2_1). */
static const double W_FD[4] = {-49.0 / 18.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0};

typedef struct {
    int n[3];
    double cell[3], h[3];
    double r_pe, r_me;
    int c0[3];
    int n_pe, n_me;
    int *off;            /* [n_me][3] local offsets (x,y,z) in grid units    */
    int blo[3], bhi[3];  /* bounding box of the offsets                      */
    int *box;            /* dense map offset -> local index q, or -1         */
    int *nbr;            /* [n_pe][18] local index of each stencil neighbour */
} osub;

/* ---- small helpers ------------------------------------------------------ */

/* Fortran NINT: nearest integer, halves rounded away from zero. */
static long o_nint(double v) { return (long)(v >= 0.0 ? floor(v + 0.5) : -floor(-v + 0.5)); }

/* Mathematical (non-negative) modulo. */
static int o_mod(long a, int n) { long r = a % n; return (int)(r < 0 ? r + n : r); }

static int o_inside(const double h[3], int ox, int oy, int oz, double R)
{
    double dx = ox * h[0], dy = oy * h[1], dz = oz * h[2];
    return dx * dx + dy * dy + dz * dz <= R * R * (1.0 + 1e-12);
}

double o_fd_weight(int s) { return W_FD[s < 0 ? -s : s]; }

/* ---- pair list (Step II) -------------------------------------------------- */

/* Unique pairs i <= j with |C_j - C_i|_min-image < r_pair (self pairs always
 * kept), ordered by i then j.  Returns the number of pairs; writes at most
 * max_pairs of them. */
int o_pair_list(int n_orb, const double *C, const double cell[3], double r_pair,
                int max_pairs, int *pi, int *pj)
{
    int np = 0;
    for (int i = 0; i < n_orb; ++i)
        for (int j = i; j < n_orb; ++j) {
            double d2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double d = C[3 * j + a] - C[3 * i + a];
                d -= cell[a] * (double)o_nint(d / cell[a]);
                d2 += d * d;
            }
            if (i == j || d2 < r_pair * r_pair) {
                if (np < max_pairs) { pi[np] = i; pj[np] = j; }
                ++np;
            }
        }
    return np;
}

/* Pair origin: midpoint of the two centres under the minimum image, wrapped
 * into the cell and snapped to the nearest grid point (Step III). */
void o_pair_origin(const double ci[3], const double cj[3], const double cell[3],
                   const int n[3], int gc[3])
{
    for (int a = 0; a < 3; ++a) {
        double d = cj[a] - ci[a];
        d -= cell[a] * (double)o_nint(d / cell[a]);
        double m = ci[a] + 0.5 * d;
        m -= cell[a] * floor(m / cell[a]);
        double h = cell[a] / n[a];
        gc[a] = o_mod(o_nint(m / h), n[a]);
    }
}

/* ---- proto-subdomains (Alg. 2) ------------------------------------------ */

void o_sub_free(osub *s)
{
    if (!s) return;
    free(s->off); free(s->box); free(s->nbr); free(s);
}

/* Returns 0 on success, -1 on bad arguments, -2 when some stencil neighbour
 * of a PE point falls outside PE u shell (R_ME - R_PE too small or the ME
 * sphere clipped by the cell too close to PE). */
int o_sub_build(const int n[3], const double cell[3], double r_pe, double r_me, osub **out)
{
    *out = NULL;
    if (!(r_pe > 0.0) || !(r_me > r_pe)) return -1;
    osub *s = (osub *)calloc(1, sizeof(osub));
    for (int a = 0; a < 3; ++a) {
        s->n[a] = n[a]; s->cell[a] = cell[a]; s->h[a] = cell[a] / n[a];
        s->c0[a] = (int)o_nint(0.5 * n[a]);
    }
    s->r_pe = r_pe; s->r_me = r_me;
    /* Loop over every grid point of the cell; classify its offset from C_0. */
    int cap = 1024, npe = 0, nsh = 0;
    int *pe = (int *)malloc(sizeof(int) * 3 * cap), *sh = (int *)malloc(sizeof(int) * 3 * cap);
    int capsh = cap;
    for (int iz = 0; iz < n[2]; ++iz)
        for (int iy = 0; iy < n[1]; ++iy)
            for (int ix = 0; ix < n[0]; ++ix) {
                int ox = ix - s->c0[0], oy = iy - s->c0[1], oz = iz - s->c0[2];
                if (o_inside(s->h, ox, oy, oz, r_pe)) {
                    if (npe == cap) { cap *= 2; pe = (int *)realloc(pe, sizeof(int) * 3 * cap); }
                    pe[3 * npe] = ox; pe[3 * npe + 1] = oy; pe[3 * npe + 2] = oz; ++npe;
                } else if (o_inside(s->h, ox, oy, oz, r_me)) {
                    if (nsh == capsh) { capsh *= 2; sh = (int *)realloc(sh, sizeof(int) * 3 * capsh); }
                    sh[3 * nsh] = ox; sh[3 * nsh + 1] = oy; sh[3 * nsh + 2] = oz; ++nsh;
                }
            }
    /* Concatenate: PE block first, then the shell (Eqs. rbar, g0). */
    s->n_pe = npe; s->n_me = npe + nsh;
    if (npe == 0) { free(pe); free(sh); free(s); return -1; }
    s->off = (int *)malloc(sizeof(int) * 3 * (size_t)s->n_me);
    memcpy(s->off, pe, sizeof(int) * 3 * (size_t)npe);
    memcpy(s->off + 3 * npe, sh, sizeof(int) * 3 * (size_t)nsh);
    free(pe); free(sh);
    for (int a = 0; a < 3; ++a) { s->blo[a] = 1 << 30; s->bhi[a] = -(1 << 30); }
    for (int q = 0; q < s->n_me; ++q)
        for (int a = 0; a < 3; ++a) {
            int o = s->off[3 * q + a];
            if (o < s->blo[a]) s->blo[a] = o;
            if (o > s->bhi[a]) s->bhi[a] = o;
        }
    int ibx = s->bhi[0] - s->blo[0] + 1, iby = s->bhi[1] - s->blo[1] + 1, ibz = s->bhi[2] - s->blo[2] + 1;
    if (ibx < 1 || iby < 1 || ibz < 1 || ibx > 4096 || iby > 4096 || ibz > 4096) { o_sub_free(s); return -1; }
    size_t bx = (size_t)ibx, by = (size_t)iby, bz = (size_t)ibz;
    s->box = (int *)malloc(sizeof(int) * bx * by * bz);
    for (size_t t = 0; t < bx * by * bz; ++t) s->box[t] = -1;
    for (int q = 0; q < s->n_me; ++q) {
        size_t t = ((size_t)(s->off[3 * q + 2] - s->blo[2]) * by + (s->off[3 * q + 1] - s->blo[1])) * bx
                   + (s->off[3 * q] - s->blo[0]);
        s->box[t] = q;
    }
    /* Stencil neighbours of every PE point: 3 axes x offsets +-1..+-3. */
    s->nbr = (int *)malloc(sizeof(int) * 18 * (size_t)npe);
    int bad = 0;
    for (int q = 0; q < npe; ++q) {
        int k = 0;
        for (int a = 0; a < 3; ++a)
            for (int st = -3; st <= 3; ++st) {
                if (st == 0) continue;
                int o[3] = {s->off[3 * q], s->off[3 * q + 1], s->off[3 * q + 2]};
                o[a] += st;
                int idx = -1;
                if (o[0] >= s->blo[0] && o[0] <= s->bhi[0] && o[1] >= s->blo[1] && o[1] <= s->bhi[1] &&
                    o[2] >= s->blo[2] && o[2] <= s->bhi[2])
                    idx = s->box[((size_t)(o[2] - s->blo[2]) * by + (o[1] - s->blo[1])) * bx + (o[0] - s->blo[0])];
                if (idx < 0) bad = 1;
                s->nbr[18 * q + k++] = idx;
            }
    }
    if (bad) { o_sub_free(s); return -2; }
    *out = s;
    return 0;
}

void o_sub_info(const osub *s, int *n_pe, int *n_me, int blo[3], int bhi[3])
{
    *n_pe = s->n_pe; *n_me = s->n_me;
    for (int a = 0; a < 3; ++a) { blo[a] = s->blo[a]; bhi[a] = s->bhi[a]; }
}

void o_sub_offsets(const osub *s, int *off) { memcpy(off, s->off, sizeof(int) * 3 * (size_t)s->n_me); }

/* ---- discrete operator and right-hand side (Eqs. d2_1, pe_mat_red) -------- */

/* y = A x with A = -Laplacian restricted to PE (neighbours outside PE dropped). */
void o_apply_A(const osub *s, const double *x, double *y)
{
    for (int q = 0; q < s->n_pe; ++q) {
        double acc = 0.0;
        int k = 0;
        for (int a = 0; a < 3; ++a) {
            double inv_h2 = 1.0 / (s->h[a] * s->h[a]);
            double t = W_FD[0] * x[q];
            for (int st = -3; st <= 3; ++st) {
                if (st == 0) continue;
                int nb = s->nbr[18 * q + k++];
                if (nb < s->n_pe) t += W_FD[abs(st)] * x[nb];
            }
            acc += t * inv_h2;
        }
        y[q] = -acc;
    }
}

/* b = 4 pi rho + (stencil part reaching the shell) applied to the shell
 * potential vsh[0 .. n_me-n_pe).  Equals 4 pi (rho - rho^b). */
void o_rhs(const osub *s, const double *rho, const double *vsh, double *b)
{
    for (int q = 0; q < s->n_pe; ++q) {
        double acc = 4.0 * M_PI * rho[q];
        int k = 0;
        for (int a = 0; a < 3; ++a) {
            double inv_h2 = 1.0 / (s->h[a] * s->h[a]);
            for (int st = -3; st <= 3; ++st) {
                if (st == 0) continue;
                int nb = s->nbr[18 * q + k++];
                if (nb >= s->n_pe) acc += W_FD[abs(st)] * inv_h2 * vsh[nb - s->n_pe];
            }
        }
        b[q] = acc;
    }
}

/* ---- spherical harmonics and the multipole expansion (Eqs. mepole, me) ---- */

/* Associated Legendre function P_l^m(t), 0 <= m <= l, Condon-Shortley phase. */
static double o_plm(int l, int m, double t)
{
    double pmm = 1.0, somx2 = sqrt((1.0 - t) * (1.0 + t)), f = 1.0;
    for (int i = 1; i <= m; ++i) { pmm *= -f * somx2; f += 2.0; }
    if (l == m) return pmm;
    double pm1 = t * (2 * m + 1) * pmm;
    if (l == m + 1) return pm1;
    double pll = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pll = (t * (2 * ll - 1) * pm1 - (ll + m - 1) * pmm) / (ll - m);
        pmm = pm1; pm1 = pll;
    }
    return pll;
}

static double o_fact(int k) { double f = 1.0; for (int i = 2; i <= k; ++i) f *= i; return f; }

/* Orthonormal complex spherical harmonic Y_lm(theta, phi). */
double complex o_ylm(int l, int m, double theta, double phi)
{
    int am = m < 0 ? -m : m;
    double nlm = sqrt((2 * l + 1) / (4.0 * M_PI) * o_fact(l - am) / o_fact(l + am));
    double complex y = nlm * o_plm(l, am, cos(theta)) * cexp(I * am * phi);
    if (m < 0) y = ((am & 1) ? -1.0 : 1.0) * conj(y);
    return y;
}

void o_ylm_reim(int l, int m, double theta, double phi, double *re, double *im)
{
    double complex y = o_ylm(l, m, theta, phi);
    *re = creal(y); *im = cimag(y);
}

static void o_polar(const osub *s, int q, double *r, double *theta, double *phi)
{
    double x = s->off[3 * q] * s->h[0], y = s->off[3 * q + 1] * s->h[1], z = s->off[3 * q + 2] * s->h[2];
    *r = sqrt(x * x + y * y + z * z);
    *theta = (*r > 0.0) ? acos(z / *r) : 0.0;
    *phi = atan2(y, x);
}

/* Q_lm = h^3 sum_{q in PE} rho_q r_q^l conj(Y_lm(rhat_q)), index l*l + l + m. */
void o_moments(const osub *s, const double *rho, double *Qre, double *Qim)
{
    double dv = s->h[0] * s->h[1] * s->h[2];
    double complex Q[O_NLM];
    for (int t = 0; t < O_NLM; ++t) Q[t] = 0.0;
    for (int q = 0; q < s->n_pe; ++q) {
        double r, th, ph;
        o_polar(s, q, &r, &th, &ph);
        if (r == 0.0) { Q[0] += dv * rho[q] / sqrt(4.0 * M_PI); continue; }
        for (int l = 0; l <= O_LMAX; ++l) {
            double rl = pow(r, l);
            for (int m = -l; m <= l; ++m)
                Q[l * l + l + m] += dv * rho[q] * rl * conj(o_ylm(l, m, th, ph));
        }
    }
    for (int t = 0; t < O_NLM; ++t) { Qre[t] = creal(Q[t]); Qim[t] = cimag(Q[t]); }
}

/* v(r) = sum_lm 4 pi/(2l+1) Q_lm Y_lm(rhat) / r^(l+1) on every shell point. */
void o_shell_potential(const osub *s, const double *Qre, const double *Qim, double *vsh)
{
    for (int q = s->n_pe; q < s->n_me; ++q) {
        double r, th, ph;
        o_polar(s, q, &r, &th, &ph);
        double complex v = 0.0;
        for (int l = 0; l <= O_LMAX; ++l) {
            double f = 4.0 * M_PI / (2 * l + 1) / pow(r, l + 1);
            for (int m = -l; m <= l; ++m)
                v += f * (Qre[l * l + l + m] + I * Qim[l * l + l + m]) * o_ylm(l, m, th, ph);
        }
        vsh[q - s->n_pe] = creal(v);
    }
}

/* ---- conjugate gradient --------------------------------------------------- */

static double o_dot(int n, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Solves A x = b from x = 0.  Returns the number of iterations; *converged
 * is 1 if ||r|| <= tol ||b|| was reached within maxit; *relres receives the
 * true relative residual ||b - A x|| / ||b|| recomputed at the end. */
int o_cg(const osub *s, const double *b, double *x, double tol, int maxit, int *converged, double *relres)
{
    int n = s->n_pe;
    double *r = (double *)malloc(sizeof(double) * n), *p = (double *)malloc(sizeof(double) * n),
           *Ap = (double *)malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; p[i] = b[i]; }
    double rr = o_dot(n, r, r), bb = rr;
    int k = 0;
    *converged = 0;
    for (;;) {
        if (sqrt(rr) <= tol * sqrt(bb)) { *converged = 1; break; }
        if (k >= maxit) break;
        o_apply_A(s, p, Ap);
        double alpha = rr / o_dot(n, p, Ap);
        for (int i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * Ap[i]; }
        double rr_new = o_dot(n, r, r);
        double beta = rr_new / rr;
        for (int i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rr = rr_new;
        ++k;
    }
    o_apply_A(s, x, Ap);
    double res = 0.0;
    for (int i = 0; i < n; ++i) { double d = b[i] - Ap[i]; res += d * d; }
    *relres = bb > 0.0 ? sqrt(res / bb) : 0.0;
    free(r); free(p); free(Ap);
    return k;
}

/* ---- one pair, end to end ---------------------------------------------- */

typedef struct {
    double e;        /* h^3 sum_PE rho x */
    int iters;
    int converged;
    double relres;
} o_pair_result;

static size_t o_gidx(const osub *s, const int gc[3], int q)
{
    int gx = o_mod((long)gc[0] + s->off[3 * q], s->n[0]);
    int gy = o_mod((long)gc[1] + s->off[3 * q + 1], s->n[1]);
    int gz = o_mod((long)gc[2] + s->off[3 * q + 2], s->n[2]);
    return ((size_t)gz * s->n[1] + gy) * s->n[0] + gx;
}

/* Gather, density, moments, shell potential, RHS, CG, energy for one pair.
 * Outputs (optional, may be NULL): x [n_pe], vsh [n_me - n_pe], Q (re/im 49),
 * rho [n_pe], b [n_pe]. */
int o_solve_pair(const osub *s, const double *phi_i, const double *phi_j, const int gc[3],
                 double tol, int maxit, double *x_out, double *vsh_out, double *Qre_out,
                 double *Qim_out, double *rho_out, double *b_out, double *e, int *iters,
                 int *converged, double *relres)
{
    int npe = s->n_pe, nsh = s->n_me - s->n_pe;
    double *rho = (double *)malloc(sizeof(double) * npe), *b = (double *)malloc(sizeof(double) * npe),
           *x = (double *)malloc(sizeof(double) * npe), *vsh = (double *)malloc(sizeof(double) * (nsh > 0 ? nsh : 1));
    double Qre[O_NLM], Qim[O_NLM];
    for (int q = 0; q < npe; ++q) {
        size_t g = o_gidx(s, gc, q);
        rho[q] = phi_i[g] * phi_j[g];
    }
    o_moments(s, rho, Qre, Qim);
    o_shell_potential(s, Qre, Qim, vsh);
    o_rhs(s, rho, vsh, b);
    *iters = o_cg(s, b, x, tol, maxit, converged, relres);
    double dv = s->h[0] * s->h[1] * s->h[2];
    *e = dv * o_dot(npe, rho, x);
    if (x_out) memcpy(x_out, x, sizeof(double) * npe);
    if (vsh_out) memcpy(vsh_out, vsh, sizeof(double) * nsh);
    if (Qre_out) memcpy(Qre_out, Qre, sizeof(Qre));
    if (Qim_out) memcpy(Qim_out, Qim, sizeof(Qim));
    if (rho_out) memcpy(rho_out, rho, sizeof(double) * npe);
    if (b_out) memcpy(b_out, b, sizeof(double) * npe);
    free(rho); free(b); free(x); free(vsh);
    return 0;
}

/* D^i += v phi_j and (i != j) D^j += v phi_i over the whole ME sphere. */
static void o_accumulate_D(const osub *s, const int gc[3], int i, int j, const double *x, const double *vsh,
                           const double *phi, double *D, size_t ngrid)
{
    for (int q = 0; q < s->n_me; ++q) {
        size_t g = o_gidx(s, gc, q);
        double v = q < s->n_pe ? x[q] : vsh[q - s->n_pe];
        D[(size_t)i * ngrid + g] += v * phi[(size_t)j * ngrid + g];
        if (i != j) D[(size_t)j * ngrid + g] += v * phi[(size_t)i * ngrid + g];
    }
}

/* Whole step: pair list, every pair solve (OpenMP over pairs, in batches),
 * E_xx = -sum_pairs w_ij e_ij with w = 1 (i == j) or 2, and D (if non-NULL,
 * zeroed here) accumulated in pair order.  Per-pair outputs are optional.
 * r_pe, r_me: [0] self pairs, [1] non-self pairs.  Returns the number of
 * pairs, or a negative error. */
long o_exx(const int n[3], const double cell[3], double r_pair, const double r_pe[2], const double r_me[2],
           int n_orb, const double *C, const double *phi, double tol, int maxit, int nthreads,
           double *E, double *D, long max_pairs, int *pi_out, int *pj_out, double *e_out,
           int *iters_out, int *conv_out, double *relres_out)
{
    osub *cls[2] = {NULL, NULL};
    for (int c = 0; c < 2; ++c) {
        int rc = o_sub_build(n, cell, r_pe[c], r_me[c], &cls[c]);
        if (rc) { o_sub_free(cls[0]); return rc - 10; }
    }
    int np = o_pair_list(n_orb, C, cell, r_pair, 0, NULL, NULL);
    int *pi = (int *)malloc(sizeof(int) * np), *pj = (int *)malloc(sizeof(int) * np);
    o_pair_list(n_orb, C, cell, r_pair, np, pi, pj);
    size_t ngrid = (size_t)n[0] * n[1] * n[2];
    if (D) memset(D, 0, sizeof(double) * ngrid * n_orb);
    double Exx = 0.0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    int batch = nthreads;
    double **xs = (double **)calloc(batch, sizeof(double *)), **vs = (double **)calloc(batch, sizeof(double *));
    for (int t = 0; t < batch; ++t) {
        xs[t] = (double *)malloc(sizeof(double) * cls[0]->n_me + sizeof(double) * cls[1]->n_me);
        vs[t] = (double *)malloc(sizeof(double) * cls[0]->n_me + sizeof(double) * cls[1]->n_me);
    }
    o_pair_result *res = (o_pair_result *)malloc(sizeof(o_pair_result) * batch);
    for (int p0 = 0; p0 < np; p0 += batch) {
        int nb = np - p0 < batch ? np - p0 : batch;
#pragma omp parallel for schedule(static, 1) num_threads(nthreads)
        for (int t = 0; t < nb; ++t) {
            int p = p0 + t, i = pi[p], j = pj[p];
            const osub *s = cls[i == j ? 0 : 1];
            int gc[3];
            o_pair_origin(C + 3 * i, C + 3 * j, cell, n, gc);
            o_solve_pair(s, phi + (size_t)i * ngrid, phi + (size_t)j * ngrid, gc, tol, maxit, xs[t], vs[t],
                         NULL, NULL, NULL, NULL, &res[t].e, &res[t].iters, &res[t].converged, &res[t].relres);
        }
        for (int t = 0; t < nb; ++t) {   /* pair order: deterministic sums */
            int p = p0 + t, i = pi[p], j = pj[p];
            const osub *s = cls[i == j ? 0 : 1];
            Exx -= (i == j ? 1.0 : 2.0) * res[t].e;
            if (D) {
                int gc[3];
                o_pair_origin(C + 3 * i, C + 3 * j, cell, n, gc);
                o_accumulate_D(s, gc, i, j, xs[t], vs[t], phi, D, ngrid);
            }
            if (p < max_pairs) {
                if (pi_out) pi_out[p] = i;
                if (pj_out) pj_out[p] = j;
                if (e_out) e_out[p] = res[t].e;
                if (iters_out) iters_out[p] = res[t].iters;
                if (conv_out) conv_out[p] = res[t].converged;
                if (relres_out) relres_out[p] = res[t].relres;
            }
        }
    }
    for (int t = 0; t < batch; ++t) { free(xs[t]); free(vs[t]); }
    free(xs); free(vs); free(res); free(pi); free(pj);
    o_sub_free(cls[0]); o_sub_free(cls[1]);
    *E = Exx;
    return np;
}

/* Solves an explicit list of pairs in parallel (timing / sampled checks).
 * Orbitals are addressed through phi_ptrs[orbital] so callers can pass only
 * the orbitals the sample touches.  Returns the number of threads used. */
int o_solve_pairs(const int n[3], const double cell[3], const double r_pe[2], const double r_me[2],
                  const double *C, const double *const *phi_ptrs, int n_list, const int *pi, const int *pj,
                  double tol, int maxit, int nthreads, double *e_out, int *iters_out, int *conv_out,
                  double *relres_out)
{
    osub *cls[2] = {NULL, NULL};
    for (int c = 0; c < 2; ++c)
        if (o_sub_build(n, cell, r_pe[c], r_me[c], &cls[c])) { o_sub_free(cls[0]); return -1; }
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int t = 0; t < n_list; ++t) {
        int i = pi[t], j = pj[t];
        const osub *s = cls[i == j ? 0 : 1];
        int gc[3];
        o_pair_origin(C + 3 * i, C + 3 * j, cell, n, gc);
        o_solve_pair(s, phi_ptrs[i], phi_ptrs[j], gc, tol, maxit, NULL, NULL, NULL, NULL, NULL, NULL,
                     &e_out[t], &iters_out[t], &conv_out[t], &relres_out[t]);
    }
    o_sub_free(cls[0]); o_sub_free(cls[1]);
    return nthreads;
}

/* An explicit list of pairs, each on its own subdomain class k = cls[t]
 * (radii r_pe[k], r_me[k], k < n_cls): the per-pair subdomains of the
 * paper's outlook (Sec. IV A), each class built by Alg. 2 as the two fixed
 * ones are.  Returns the number of threads used, or -1. */
int o_solve_pairs_classed(const int n[3], const double cell[3], int n_cls, const double *r_pe, const double *r_me,
                          const double *C, const double *const *phi_ptrs, int n_list, const int *pi, const int *pj,
                          const int *cls, double tol, int maxit, int nthreads, double *e_out, int *iters_out,
                          int *conv_out, double *relres_out)
{
    if (n_cls < 1 || n_cls > 8) return -1;
    osub *sub[8] = {NULL};
    for (int k = 0; k < n_cls; ++k)
        if (o_sub_build(n, cell, r_pe[k], r_me[k], &sub[k])) {
            for (int q = 0; q < k; ++q) o_sub_free(sub[q]);
            return -1;
        }
    for (int t = 0; t < n_list; ++t)
        if (cls[t] < 0 || cls[t] >= n_cls) {
            for (int k = 0; k < n_cls; ++k) o_sub_free(sub[k]);
            return -1;
        }
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int t = 0; t < n_list; ++t) {
        int i = pi[t], j = pj[t];
        int gc[3];
        o_pair_origin(C + 3 * i, C + 3 * j, cell, n, gc);
        o_solve_pair(sub[cls[t]], phi_ptrs[i], phi_ptrs[j], gc, tol, maxit, NULL, NULL, NULL, NULL, NULL, NULL,
                     &e_out[t], &iters_out[t], &conv_out[t], &relres_out[t]);
    }
    for (int k = 0; k < n_cls; ++k) o_sub_free(sub[k]);
    return nthreads;
}

/* D^k (Eq. Dxx_mlwf_omega) over an explicit list of pairs that involve
 * orbital k, each on its class cls[t]: the pairs are solved in parallel and
 * their contributions v phi_other added in list order (so, for the list of
 * every pair of k in pair order, the sum runs as the whole step's does).
 * Dk: [Nz][Ny][Nx], overwritten.  Returns 0, or -1. */
int o_dxx_orbital(const int n[3], const double cell[3], int n_cls, const double *r_pe, const double *r_me,
                  const double *C, const double *const *phi_ptrs, int n_list, const int *pi, const int *pj,
                  const int *cls, int k, double tol, int maxit, int nthreads, double *Dk)
{
    if (n_cls < 1 || n_cls > 8) return -1;
    for (int t = 0; t < n_list; ++t)
        if ((pi[t] != k && pj[t] != k) || cls[t] < 0 || cls[t] >= n_cls) return -1;
    osub *sub[8] = {NULL};
    int max_me = 0;
    for (int q = 0; q < n_cls; ++q) {
        if (o_sub_build(n, cell, r_pe[q], r_me[q], &sub[q])) {
            for (int u = 0; u < q; ++u) o_sub_free(sub[u]);
            return -1;
        }
        if (sub[q]->n_me > max_me) max_me = sub[q]->n_me;
    }
    size_t ngrid = (size_t)n[0] * n[1] * n[2];
    memset(Dk, 0, sizeof(double) * ngrid);
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    int batch = nthreads;
    double **xs = (double **)calloc(batch, sizeof(double *)), **vs = (double **)calloc(batch, sizeof(double *));
    for (int t = 0; t < batch; ++t) {
        xs[t] = (double *)malloc(sizeof(double) * max_me);
        vs[t] = (double *)malloc(sizeof(double) * max_me);
    }
    for (int p0 = 0; p0 < n_list; p0 += batch) {
        int nb = n_list - p0 < batch ? n_list - p0 : batch;
#pragma omp parallel for schedule(static, 1) num_threads(nthreads)
        for (int t = 0; t < nb; ++t) {
            int p = p0 + t, i = pi[p], j = pj[p];
            int gc[3], it, cv;
            double e, rr;
            o_pair_origin(C + 3 * i, C + 3 * j, cell, n, gc);
            o_solve_pair(sub[cls[p]], phi_ptrs[i], phi_ptrs[j], gc, tol, maxit, xs[t], vs[t], NULL, NULL, NULL, NULL,
                         &e, &it, &cv, &rr);
        }
        for (int t = 0; t < nb; ++t) {   /* list order */
            int p = p0 + t, i = pi[p], j = pj[p];
            const osub *s = sub[cls[p]];
            int gc[3];
            o_pair_origin(C + 3 * i, C + 3 * j, cell, n, gc);
            const double *other = phi_ptrs[i == k ? j : i];
            for (int q = 0; q < s->n_me; ++q) {
                size_t g = o_gidx(s, gc, q);
                double v = q < s->n_pe ? xs[t][q] : vs[t][q - s->n_pe];
                Dk[g] += v * other[g];
            }
        }
    }
    for (int t = 0; t < batch; ++t) { free(xs[t]); free(vs[t]); }
    free(xs); free(vs);
    for (int q = 0; q < n_cls; ++q) o_sub_free(sub[q]);
    return 0;
}
