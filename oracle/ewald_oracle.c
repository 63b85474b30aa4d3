/*
 * Plain FP64 CPU oracle for classical Ewald summation -- TEST INFRASTRUCTURE.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header, table or constant generator
 * with the HIP path; it is the reference the GPU results are checked against.
 *
 * What it computes (Saunders, Grant & Mueller, "Long range forces in a
 * performance portable Molecular Dynamics framework", section 3):
 *
 *   N point charges q_j at r_j in a periodic cube of side L, V = L^3,
 *   Gaussian units (Coulomb potential q/r, section 2.1).  The splitting
 *   Gaussian S_alpha ~ exp(-alpha r^2) (section 3.1.1) fixes the convention:
 *   real-space kernel erfc(sqrt(alpha) d)/d, reciprocal damping
 *   exp(-k^2/(4 alpha)), k = 2 pi n / L with integer n (section 3.1.2).
 *
 *   E_real  = 1/2 sum_i sum_{(j,s) != (i,0), |d|<r_c} q_i q_j erfc(sqrt(alpha)|d|)/|d|,
 *             d = r_i - r_j + s, s in L Z^3        (truncated sum of section 3.2.1)
 *   F_real,i = sum (same set) q_i q_j d/|d|^2 [erfc(sqrt(alpha)|d|)/|d|
 *                                             + 2 sqrt(alpha/pi) exp(-alpha |d|^2)]
 *   S_k      = sum_j q_j exp(i k.r_j)   (the paper's rho-hat is its conjugate, Eq. perf_mod1)
 *   C_k      = 4 pi / (V k^2) exp(-k^2 / (4 alpha))                 (Eq. perf_mod1)
 *   E_recip  = 1/2 sum_{k in K} C_k |S_k|^2, K = {n != 0 : |n|^2 <= k_max^2}
 *   F_recip,i = q_i sum_{k in K} C_k k Im(exp(i k.r_i) conj(S_k))     (Algorithm 2)
 *   phi_recip,i = sum_{k in K} C_k Re(exp(i k.r_i) conj(S_k))
 *   E_self   = -sqrt(alpha/pi) sum_i q_i^2      (self term of section 3.2.2, not printed
 *                                               in the paper; potential of a Gaussian at
 *                                               its own centre)
 *   E_bg     = -pi Q^2 / (2 V alpha), Q = sum q  (uniform neutralising background; zero
 *                                               for the neutral systems the paper assumes)
 *   dE/dq_i  = phi_real,i + phi_recip,i - 2 sqrt(alpha/pi) q_i - pi Q/(V alpha)
 *
 * Readings where the paper is silent or inconsistent:
 *   - the reciprocal energy carries the factor 1/2 over the full k set (equal to the
 *     sum over a half space); Algorithm 2 prints the energy line without it, but its
 *     force line is the gradient of the halved sum;
 *   - the k set is the sphere |n|^2 <= k_max^2 (inclusive, exact integer test);
 *   - the real-space cutoff is strict, tested as |d|^2 < r_c^2 on the FP64 displacement;
 *   - every periodic image with |d| < r_c is summed, also when r_c > L/2;
 *   - conducting ("tin-foil") boundary: no dipole surface term.
 *
 * Two independent evaluation routes exist for each part so that tests can play
 * them against each other:
 *   real space : ORACLE_BRUTE  -- every pair (i, j) and every shift |a|,|b|,|c| <= A
 *                ORACLE_CELLS  -- a plain cell list of side >= r_c with unwrapped offsets
 *   reciprocal : ORACLE_BRUTE  -- full k set, direct sin/cos of k.r per (particle, k)
 *                ORACLE_TABLES -- half space k set, exp(i k.r) as the product of per-axis
 *                                 exp(i n_a theta_a) evaluated directly with libm
 * Sums over particles run in index order, so results do not depend on the number of
 * OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_BRUTE 0
#define ORACLE_CELLS 1
#define ORACLE_TABLES 1

static const double ORACLE_PI = 3.14159265358979323846264338327950288;

/* Reduce one coordinate into [0, L). */
static double wrap_coord(double x, double L)
{
    double w = x - L * floor(x / L);
    if (w < 0.0) w += L;
    if (w >= L) w -= L;
    if (!(w >= 0.0 && w < L)) w = 0.0;
    return w;
}

static double *wrapped_copy(int64_t n, const double *pos, double L)
{
    double *w = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!w) return NULL;
    for (int64_t i = 0; i < 3 * n; ++i) w[i] = wrap_coord(pos[i], L);
    return w;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ------------------------------------------------------------------ k sets */

static int in_half_space(int nx, int ny, int nz)
{
    return nx > 0 || (nx == 0 && ny > 0) || (nx == 0 && ny == 0 && nz > 0);
}

/* Count (out == NULL) or list the integer vectors n != 0 with |n|^2 <= k_max^2.
 * half != 0 keeps only the half space above.  Order: nx, then ny, then nz ascending. */
int64_t oracle_kset(int k_max, int half, int32_t *out)
{
    int64_t c = 0;
    const int K2 = k_max * k_max;
    for (int nx = -k_max; nx <= k_max; ++nx)
        for (int ny = -k_max; ny <= k_max; ++ny)
            for (int nz = -k_max; nz <= k_max; ++nz) {
                int m2 = nx * nx + ny * ny + nz * nz;
                if (m2 == 0 || m2 > K2) continue;
                if (half && !in_half_space(nx, ny, nz)) continue;
                if (out) {
                    out[3 * c + 0] = nx;
                    out[3 * c + 1] = ny;
                    out[3 * c + 2] = nz;
                }
                ++c;
            }
    return c;
}

/* C_k for integer n in a box of side L. */
static double coef_ck(int m2, double L, double alpha)
{
    const double V = L * L * L;
    const double g = 2.0 * ORACLE_PI / L;
    const double k2 = g * g * (double)m2;
    return 4.0 * ORACLE_PI / (V * k2) * exp(-k2 / (4.0 * alpha));
}

/* ---------------------------------------------------- structure factor S_k */

/* S_k = sum_j q_j exp(i k.r_j) for the listed k (integer triples), by direct
 * cos/sin of the full phase.  Positions are wrapped first (S_k is periodic). */
int oracle_structure_factor(int64_t n, const double *pos, const double *q, double L,
                            int64_t nk, const int32_t *kn, double *re, double *im)
{
    double *w = wrapped_copy(n, pos, L);
    if (!w) return -3;
    const double g = 2.0 * ORACLE_PI / L;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nk; ++k) {
        const double kx = g * kn[3 * k], ky = g * kn[3 * k + 1], kz = g * kn[3 * k + 2];
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double ph = kx * w[3 * j] + ky * w[3 * j + 1] + kz * w[3 * j + 2];
            sr += q[j] * cos(ph);
            si += q[j] * sin(ph);
        }
        re[k] = sr;
        im[k] = si;
    }
    free(w);
    return 0;
}

/* ------------------------------------------------------------- real space */

/* Contribution of one image pair to phi_i and F_i (strict cutoff on |d|^2). */
static inline void real_pair(double dx, double dy, double dz, double qj, double rc2,
                             double sqrt_alpha, double alpha, double two_sqrt_a_pi,
                             double *phi, double *fx, double *fy, double *fz)
{
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 < rc2)) return;
    const double r = sqrt(r2);
    const double ec = erfc(sqrt_alpha * r) / r;          /* erfc(sqrt(a) r)/r */
    const double f = qj * (ec + two_sqrt_a_pi * exp(-alpha * r2)) / r2;
    *phi += qj * ec;
    *fx += f * dx;
    *fy += f * dy;
    *fz += f * dz;
}

/* Real-space potential phi_real and force F_real for the targets (all particles
 * when targets == NULL).  forces/phi are indexed like the targets list.  When
 * targets == NULL, *e_real = 1/2 sum_i q_i phi_i (index order). */
int oracle_real_space(int64_t n, const double *pos, const double *q, double L, double alpha,
                      double r_c, int method, int64_t n_targets, const int64_t *targets,
                      double *e_real, double *forces, double *phi)
{
    if (n < 0 || L <= 0 || alpha <= 0 || r_c <= 0) return -1;
    double *w = wrapped_copy(n, pos, L);
    if (!w) return -3;
    const int64_t nt = targets ? n_targets : n;
    double *ph = (double *)calloc((size_t)(nt > 0 ? nt : 1), sizeof(double));
    double *fo = (double *)calloc((size_t)(nt > 0 ? nt : 1) * 3, sizeof(double));
    if (!ph || !fo) { free(w); free(ph); free(fo); return -3; }
    const double rc2 = r_c * r_c;
    const double sa = sqrt(alpha);
    const double tsap = 2.0 * sqrt(alpha / ORACLE_PI);

    if (method == ORACLE_BRUTE) {
        /* positions in [0,L): |r_i - r_j| < L per axis, so |a| <= ceil(r_c/L) + 1 suffices */
        const int A = (int)ceil(r_c / L) + 1;
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t t = 0; t < nt; ++t) {
            const int64_t i = targets ? targets[t] : t;
            double p = 0, fx = 0, fy = 0, fz = 0;
            for (int64_t j = 0; j < n; ++j)
                for (int a = -A; a <= A; ++a)
                    for (int b = -A; b <= A; ++b)
                        for (int c = -A; c <= A; ++c) {
                            if (j == i && a == 0 && b == 0 && c == 0) continue;
                            real_pair(w[3 * i] - w[3 * j] + a * L, w[3 * i + 1] - w[3 * j + 1] + b * L,
                                      w[3 * i + 2] - w[3 * j + 2] + c * L, q[j], rc2, sa, alpha, tsap,
                                      &p, &fx, &fy, &fz);
                        }
            ph[t] = p;
            fo[3 * t] = q[i] * fx;
            fo[3 * t + 1] = q[i] * fy;
            fo[3 * t + 2] = q[i] * fz;
        }
    } else {
        /* Cell list: nc = floor(L / r_c) cells per axis (side h >= r_c), so every image
         * within r_c of particle i lies in the 27 cells around its own, taken as
         * unwrapped offsets: each offset names one (cell, image shift) pair, which stays
         * correct when nc < 3 (the same cell then appears under different shifts). */
        if (r_c > L) { free(w); free(ph); free(fo); return -1; }
        int nc = (int)floor(L / r_c);
        if (nc < 1) nc = 1;
        const double h = L / nc;
        const int64_t ncell = (int64_t)nc * nc * nc;
        int64_t *head = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell + 1));
        int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        int64_t *cid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        if (!head || !list || !cid) { free(w); free(ph); free(fo); free(head); free(list); free(cid); return -3; }
        memset(head, 0, sizeof(int64_t) * (size_t)(ncell + 1));
        for (int64_t j = 0; j < n; ++j) {
            int c3[3];
            for (int a = 0; a < 3; ++a) {
                int c = (int)(w[3 * j + a] / h);
                if (c >= nc) c = nc - 1;
                if (c < 0) c = 0;
                c3[a] = c;
            }
            cid[j] = ((int64_t)c3[0] * nc + c3[1]) * nc + c3[2];
            head[cid[j] + 1]++;
        }
        for (int64_t c = 0; c < ncell; ++c) head[c + 1] += head[c];
        {
            int64_t *fill = (int64_t *)calloc((size_t)ncell, sizeof(int64_t));
            if (!fill) { free(w); free(ph); free(fo); free(head); free(list); free(cid); return -3; }
            for (int64_t j = 0; j < n; ++j) list[head[cid[j]] + fill[cid[j]]++] = j;
            free(fill);
        }
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t t = 0; t < nt; ++t) {
            const int64_t i = targets ? targets[t] : t;
            const int64_t ci = cid[i];
            const int cx = (int)(ci / ((int64_t)nc * nc)), cy = (int)((ci / nc) % nc), cz = (int)(ci % nc);
            double p = 0, fx = 0, fy = 0, fz = 0;
            for (int ox = -1; ox <= 1; ++ox)
                for (int oy = -1; oy <= 1; ++oy)
                    for (int oz = -1; oz <= 1; ++oz) {
                        int vx = cx + ox, vy = cy + oy, vz = cz + oz;
                        double sx = 0, sy = 0, sz = 0; /* image shift added to r_j */
                        if (vx < 0) { vx += nc; sx = -L; } else if (vx >= nc) { vx -= nc; sx = L; }
                        if (vy < 0) { vy += nc; sy = -L; } else if (vy >= nc) { vy -= nc; sy = L; }
                        if (vz < 0) { vz += nc; sz = -L; } else if (vz >= nc) { vz -= nc; sz = L; }
                        const int64_t cn = ((int64_t)vx * nc + vy) * nc + vz;
                        const int zero_shift = (sx == 0 && sy == 0 && sz == 0);
                        for (int64_t e = head[cn]; e < head[cn + 1]; ++e) {
                            const int64_t j = list[e];
                            if (j == i && zero_shift) continue;
                            real_pair(w[3 * i] - (w[3 * j] + sx), w[3 * i + 1] - (w[3 * j + 1] + sy),
                                      w[3 * i + 2] - (w[3 * j + 2] + sz), q[j], rc2, sa, alpha, tsap,
                                      &p, &fx, &fy, &fz);
                        }
                    }
            ph[t] = p;
            fo[3 * t] = q[i] * fx;
            fo[3 * t + 1] = q[i] * fy;
            fo[3 * t + 2] = q[i] * fz;
        }
        free(head);
        free(list);
        free(cid);
    }
    if (e_real) {
        double e = 0.0;
        if (!targets)
            for (int64_t i = 0; i < n; ++i) e += 0.5 * q[i] * ph[i];
        *e_real = e;
    }
    if (phi) memcpy(phi, ph, sizeof(double) * (size_t)nt);
    if (forces) memcpy(forces, fo, sizeof(double) * 3 * (size_t)nt);
    free(w);
    free(ph);
    free(fo);
    return 0;
}

/* ------------------------------------------------------- reciprocal space */

/* exp(i n theta) for one axis from per-axis tables of n >= 0 (n < 0: conjugate). */
static inline void axis_phase(const double *c, const double *s, int nabs_max, int n, double *re, double *im)
{
    (void)nabs_max;
    if (n >= 0) { *re = c[n]; *im = s[n]; }
    else { *re = c[-n]; *im = -s[-n]; }
}

/* Reciprocal energy, and phi_recip / F_recip for the targets (all when NULL).
 * method ORACLE_BRUTE: full k set, direct cos/sin of k.r everywhere.
 * method ORACLE_TABLES: half-space k set (E = sum_{K+} C|S|^2, forces and phi with
 * the factor 2 of the folded sum), exp(i k.r) from per-axis libm cos/sin tables.
 * When sk_re/sk_im are given, the half-space S_k (oracle_kset order, half=1) is
 * written there (ORACLE_TABLES only). */
int oracle_recip_space(int64_t n, const double *pos, const double *q, double L, double alpha,
                       int k_max, int method, int64_t n_targets, const int64_t *targets,
                       double *e_recip, double *forces, double *phi, double *sk_re, double *sk_im)
{
    if (n < 0 || L <= 0 || alpha <= 0 || k_max < 1) return -1;
    double *w = wrapped_copy(n, pos, L);
    if (!w) return -3;
    const int half = (method != ORACLE_BRUTE);
    const int64_t nk = oracle_kset(k_max, half, NULL);
    int32_t *kn = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)nk);
    double *Sr = (double *)malloc(sizeof(double) * (size_t)nk);
    double *Si = (double *)malloc(sizeof(double) * (size_t)nk);
    double *Ck = (double *)malloc(sizeof(double) * (size_t)nk);
    const int64_t nt = targets ? n_targets : n;
    if (!kn || !Sr || !Si || !Ck) { free(w); free(kn); free(Sr); free(Si); free(Ck); return -3; }
    oracle_kset(k_max, half, kn);
    for (int64_t k = 0; k < nk; ++k) {
        const int m2 = kn[3 * k] * kn[3 * k] + kn[3 * k + 1] * kn[3 * k + 1] + kn[3 * k + 2] * kn[3 * k + 2];
        Ck[k] = coef_ck(m2, L, alpha);
    }
    const double g = 2.0 * ORACLE_PI / L;
    const int K1 = k_max + 1;
    double *tc = NULL, *ts = NULL;

    if (method == ORACLE_BRUTE) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t k = 0; k < nk; ++k) {
            const double kx = g * kn[3 * k], ky = g * kn[3 * k + 1], kz = g * kn[3 * k + 2];
            double sr = 0, si = 0;
            for (int64_t j = 0; j < n; ++j) {
                const double ph = kx * w[3 * j] + ky * w[3 * j + 1] + kz * w[3 * j + 2];
                sr += q[j] * cos(ph);
                si += q[j] * sin(ph);
            }
            Sr[k] = sr;
            Si[k] = si;
        }
    } else {
        /* per-axis tables: cos(n theta_a), sin(n theta_a), theta_a = 2 pi x_a / L, n = 0..k_max */
        tc = (double *)malloc(sizeof(double) * 3 * (size_t)K1 * (size_t)(n > 0 ? n : 1));
        ts = (double *)malloc(sizeof(double) * 3 * (size_t)K1 * (size_t)(n > 0 ? n : 1));
        if (!tc || !ts) { free(w); free(kn); free(Sr); free(Si); free(Ck); free(tc); free(ts); return -3; }
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; ++j)
            for (int a = 0; a < 3; ++a) {
                const double th = g * w[3 * j + a];
                for (int m = 0; m <= k_max; ++m) {
                    tc[(j * 3 + a) * K1 + m] = cos(m * th);
                    ts[(j * 3 + a) * K1 + m] = sin(m * th);
                }
            }
        /* Each thread owns a contiguous range of k and walks the particles in index order. */
#pragma omp parallel
        {
            int nth = 1, tid = 0;
#ifdef _OPENMP
            nth = omp_get_num_threads();
            tid = omp_get_thread_num();
#endif
            const int64_t k0 = nk * tid / nth, k1 = nk * (tid + 1) / nth;
            for (int64_t k = k0; k < k1; ++k) Sr[k] = Si[k] = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                const double *cx = tc + (j * 3 + 0) * K1, *sx = ts + (j * 3 + 0) * K1;
                const double *cy = tc + (j * 3 + 1) * K1, *sy = ts + (j * 3 + 1) * K1;
                const double *cz = tc + (j * 3 + 2) * K1, *sz = ts + (j * 3 + 2) * K1;
                for (int64_t k = k0; k < k1; ++k) {
                    double xr, xi, yr, yi, zr, zi;
                    axis_phase(cx, sx, k_max, kn[3 * k], &xr, &xi);
                    axis_phase(cy, sy, k_max, kn[3 * k + 1], &yr, &yi);
                    axis_phase(cz, sz, k_max, kn[3 * k + 2], &zr, &zi);
                    const double ar = xr * yr - xi * yi, ai = xr * yi + xi * yr;
                    const double er = ar * zr - ai * zi, ei = ar * zi + ai * zr;
                    Sr[k] += q[j] * er;
                    Si[k] += q[j] * ei;
                }
            }
        }
    }

    /* energy: 1/2 sum over the full set, or sum over the half space */
    double e = 0.0;
    for (int64_t k = 0; k < nk; ++k) e += Ck[k] * (Sr[k] * Sr[k] + Si[k] * Si[k]);
    if (!half) e *= 0.5;
    if (e_recip) *e_recip = e;
    if (half && sk_re && sk_im) {
        memcpy(sk_re, Sr, sizeof(double) * (size_t)nk);
        memcpy(sk_im, Si, sizeof(double) * (size_t)nk);
    }

    if (forces || phi) {
        const double fold = half ? 2.0 : 1.0;
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t t = 0; t < nt; ++t) {
            const int64_t i = targets ? targets[t] : t;
            double fx = 0, fy = 0, fz = 0, p = 0;
            for (int64_t k = 0; k < nk; ++k) {
                const double kx = g * kn[3 * k], ky = g * kn[3 * k + 1], kz = g * kn[3 * k + 2];
                double c, s;
                if (tc) {
                    double xr, xi, yr, yi, zr, zi;
                    axis_phase(tc + (i * 3 + 0) * K1, ts + (i * 3 + 0) * K1, k_max, kn[3 * k], &xr, &xi);
                    axis_phase(tc + (i * 3 + 1) * K1, ts + (i * 3 + 1) * K1, k_max, kn[3 * k + 1], &yr, &yi);
                    axis_phase(tc + (i * 3 + 2) * K1, ts + (i * 3 + 2) * K1, k_max, kn[3 * k + 2], &zr, &zi);
                    const double ar = xr * yr - xi * yi, ai = xr * yi + xi * yr;
                    c = ar * zr - ai * zi;
                    s = ar * zi + ai * zr;
                } else {
                    const double ph = kx * w[3 * i] + ky * w[3 * i + 1] + kz * w[3 * i + 2];
                    c = cos(ph);
                    s = sin(ph);
                }
                /* exp(i k.r_i) conj(S_k) = (c + i s)(Sr - i Si) */
                const double re = c * Sr[k] + s * Si[k];
                const double im = s * Sr[k] - c * Si[k];
                p += Ck[k] * re;
                fx += Ck[k] * kx * im;
                fy += Ck[k] * ky * im;
                fz += Ck[k] * kz * im;
            }
            if (phi) phi[t] = fold * p;
            if (forces) {
                forces[3 * t] = fold * q[i] * fx;
                forces[3 * t + 1] = fold * q[i] * fy;
                forces[3 * t + 2] = fold * q[i] * fz;
            }
        }
    }
    free(tc);
    free(ts);
    free(w);
    free(kn);
    free(Sr);
    free(Si);
    free(Ck);
    return 0;
}

/* ------------------------------------------------------------- full result */

/* energy[5] = {total, real, recip, self, background}; forces (n x 3) and dEdq (n)
 * optional.  method selects the route for both real and reciprocal space. */
int oracle_energy_forces(int64_t n, const double *pos, const double *q, double L, double alpha,
                         double r_c, int k_max, int method, double *energy, double *forces,
                         double *dEdq)
{
    if (n < 1 || !pos || !q || !energy) return -1;
    double *fr = NULL, *fk = NULL, *pr = NULL, *pk = NULL;
    fr = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    fk = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    pr = (double *)malloc(sizeof(double) * (size_t)n);
    pk = (double *)malloc(sizeof(double) * (size_t)n);
    if (!fr || !fk || !pr || !pk) { free(fr); free(fk); free(pr); free(pk); return -3; }
    double er = 0, ek = 0;
    int st = oracle_real_space(n, pos, q, L, alpha, r_c, method, 0, NULL, &er, fr, pr);
    if (st == 0) st = oracle_recip_space(n, pos, q, L, alpha, k_max, method, 0, NULL, &ek, fk, pk, NULL, NULL);
    if (st != 0) { free(fr); free(fk); free(pr); free(pk); return st; }
    double q2 = 0, Q = 0;
    for (int64_t i = 0; i < n; ++i) { q2 += q[i] * q[i]; Q += q[i]; }
    const double V = L * L * L;
    const double es = -sqrt(alpha / ORACLE_PI) * q2;
    const double eb = -ORACLE_PI * Q * Q / (2.0 * V * alpha);
    energy[1] = er;
    energy[2] = ek;
    energy[3] = es;
    energy[4] = eb;
    energy[0] = er + ek + es + eb;
    if (forces)
        for (int64_t i = 0; i < 3 * n; ++i) forces[i] = fr[i] + fk[i];
    if (dEdq) {
        const double c_self = 2.0 * sqrt(alpha / ORACLE_PI);
        const double c_bg = ORACLE_PI * Q / (V * alpha);
        for (int64_t i = 0; i < n; ++i) dEdq[i] = pr[i] + pk[i] - c_self * q[i] - c_bg;
    }
    free(fr);
    free(fk);
    free(pr);
    free(pk);
    return 0;
}

/* Same quantities as oracle_energy_forces, with the per-particle outputs
 * restricted to a list of targets (all particles when targets == NULL):
 *   energy[5]      total, real, reciprocal, self, background (all particles)
 *   forces[t][3]   F_i = F_real,i + F_recip,i of particle i = targets[t]
 *   dEdq[t]        phi_real,i + phi_recip,i - 2 sqrt(alpha/pi) q_i - pi Q / (V alpha)
 *   sk_re, sk_im   optional half-space S_k in oracle_kset(k_max, 1) order
 *                  (table route only)
 * The real-space part is evaluated for every particle (E_real needs every
 * phi_i); the reciprocal forces and potentials only for the targets. */
int oracle_energy_forces_targets(int64_t n, const double *pos, const double *q, double L, double alpha,
                                 double r_c, int k_max, int method, int64_t n_targets,
                                 const int64_t *targets, double *energy, double *forces, double *dEdq,
                                 double *sk_re, double *sk_im)
{
    if (n < 1 || !pos || !q || !energy) return -1;
    if ((sk_re || sk_im) && method == ORACLE_BRUTE) return -1;
    const int64_t nt = targets ? n_targets : n;
    if (nt < 0) return -1;
    for (int64_t t = 0; targets && t < nt; ++t)
        if (targets[t] < 0 || targets[t] >= n) return -1;
    double *fr = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *pr = (double *)malloc(sizeof(double) * (size_t)n);
    double *fk = (double *)malloc(sizeof(double) * 3 * (size_t)(nt > 0 ? nt : 1));
    double *pk = (double *)malloc(sizeof(double) * (size_t)(nt > 0 ? nt : 1));
    if (!fr || !fk || !pr || !pk) { free(fr); free(fk); free(pr); free(pk); return -3; }
    double er = 0, ek = 0;
    int st = oracle_real_space(n, pos, q, L, alpha, r_c, method, 0, NULL, &er, fr, pr);
    if (st == 0)
        st = oracle_recip_space(n, pos, q, L, alpha, k_max, method, nt, targets, &ek, fk, pk, sk_re, sk_im);
    if (st != 0) { free(fr); free(fk); free(pr); free(pk); return st; }
    double q2 = 0, Q = 0;
    for (int64_t i = 0; i < n; ++i) { q2 += q[i] * q[i]; Q += q[i]; }
    const double V = L * L * L;
    const double es = -sqrt(alpha / ORACLE_PI) * q2;
    const double eb = -ORACLE_PI * Q * Q / (2.0 * V * alpha);
    energy[1] = er;
    energy[2] = ek;
    energy[3] = es;
    energy[4] = eb;
    energy[0] = er + ek + es + eb;
    const double c_self = 2.0 * sqrt(alpha / ORACLE_PI);
    const double c_bg = ORACLE_PI * Q / (V * alpha);
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = targets ? targets[t] : t;
        if (forces)
            for (int a = 0; a < 3; ++a) forces[3 * t + a] = fr[3 * i + a] + fk[3 * t + a];
        if (dEdq) dEdq[t] = pr[i] + pk[t] - c_self * q[i] - c_bg;
    }
    free(fr);
    free(fk);
    free(pr);
    free(pk);
    return 0;
}
