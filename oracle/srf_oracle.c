/*
 * srf_oracle.c -- plain FP64 CPU reference of the short-range TreePM step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header or constant table with the GPU
 * library; every rule below is written out again from the paper
 * (Ishiyama, Nitadori & Makino, SC12, "4.45 Pflops Astrophysical N-Body
 * Simulation on K computer") and from the readings listed beside each
 * function where the paper is silent.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC.  No FMA
 * contraction anywhere: the tree decisions must be the literal expressions.
 *
 * Conventions
 *   - box [0,1)^3, periodic; minimum image per axis: d -= rint(d);
 *   - "sorted" arrays are indexed by sorted position s; perm[s] is the
 *     original index of the particle at sorted position s;
 *   - node arrays are in DFS preorder (parent before children, children in
 *     octant order), i.e. ordered by (first, level) ascending;
 *   - G multiplies every force and gradient.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KEY_BITS 21          /* bits per axis of the Morton key */
#define MAX_LEVEL 21         /* deepest tree level */

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ================================================================== */
/* Cutoff function and pair kernel                                     */
/* ================================================================== */

/* g_P3M(xi) exactly as printed in Sec. 2, eq. (cutoff): the degree-8
 * polynomial with the zeta = max(0, xi - 1) branch term, 0 for xi > 2.
 * Kept for the transcription pins; near xi = 2 its two terms cancel. */
double or_gcut_printed(double xi) {
    if (xi > 2.0) return 0.0;
    double zeta = xi - 1.0 > 0.0 ? xi - 1.0 : 0.0;
    double x2 = xi * xi, x3 = x2 * xi, x5 = x3 * x2, x6 = x5 * xi, x7 = x6 * xi, x8 = x7 * xi;
    double first = 1.0 - (8.0 / 5.0) * x3 + (8.0 / 5.0) * x5 - 0.5 * x6
                 - (12.0 / 35.0) * x7 + (3.0 / 20.0) * x8;
    double second = pow(zeta, 6.0) * (3.0 / 35.0 + (18.0 / 35.0) * xi + (1.0 / 5.0) * x2);
    return first - second;
}

/* g_P3M(xi), the function of eq. (cutoff).  On [0,1] the printed
 * polynomial (zeta = 0 there).  On [1,2] the same polynomial, expanded
 * and factored: first - zeta^6 (...) = -(xi-2)^5 (7 xi^3 + 22 xi^2 + 10 xi + 4)/140,
 * which keeps full relative accuracy as g -> 0 at xi = 2 (the printed
 * difference of two O(1) terms does not).  0 beyond xi = 2. */
double or_gcut(double xi) {
    if (xi > 2.0) return 0.0;
    if (xi <= 1.0) {
        double x2 = xi * xi, x3 = x2 * xi, x5 = x3 * x2, x6 = x5 * xi, x7 = x6 * xi, x8 = x7 * xi;
        return 1.0 - (8.0 / 5.0) * x3 + (8.0 / 5.0) * x5 - 0.5 * x6 - (12.0 / 35.0) * x7 + (3.0 / 20.0) * x8;
    }
    double t = 2.0 - xi;
    return pow(t, 5.0) * (7.0 * xi * xi * xi + 22.0 * xi * xi + 10.0 * xi + 4.0) / 140.0;
}

/* dg/dxi.  On [0,1] term by term from the monomials; on [1,2] the
 * derivative of the factored form, -xi (xi-2)^4 (2 xi^2 + 4 xi - 1) / 5. */
double or_gcut_deriv(double xi) {
    if (xi > 2.0) return 0.0;
    if (xi <= 1.0) {
        double x2 = xi * xi, x4 = x2 * x2, x5 = x4 * xi, x6 = x5 * xi, x7 = x6 * xi;
        return -(24.0 / 5.0) * x2 + 8.0 * x4 - 3.0 * x5 - (12.0 / 5.0) * x6 + (6.0 / 5.0) * x7;
    }
    double t = 2.0 - xi;
    return -xi * pow(t, 4.0) * (2.0 * xi * xi + 4.0 * xi - 1.0) / 5.0;
}

/* d^2g/dxi^2: on [0,1] term by term from the monomials of g'; on [1,2] the
 * derivative of the factored g' = -xi t^4 P / 5 (t = 2 - xi,
 * P = 2 xi^2 + 4 xi - 1): -t^3 (t P - 4 xi P + xi t P') / 5, P' = 4 xi + 4. */
double or_gcut_deriv2(double xi) {
    if (xi > 2.0) return 0.0;
    if (xi <= 1.0) {
        double x2 = xi * xi, x3 = x2 * xi, x4 = x3 * xi, x5 = x4 * xi, x6 = x5 * xi;
        return -(48.0 / 5.0) * xi + 32.0 * x3 - 15.0 * x4 - (72.0 / 5.0) * x5 + (42.0 / 5.0) * x6;
    }
    double t = 2.0 - xi;
    double P = 2.0 * xi * xi + 4.0 * xi - 1.0, dP = 4.0 * xi + 4.0;
    return -t * t * t * (t * P - 4.0 * xi * P + xi * t * dP) / 5.0;
}

void or_gcut_deriv2_vec(int64_t n, const double* xi, double* out) {
    for (int64_t k = 0; k < n; ++k) out[k] = or_gcut_deriv2(xi[k]);
}

/* Potential factor q of the split: a source of mass m at distance r has the
 * short-range potential -G m q(xi) / r, xi = 2 r / r_cut, the antiderivative
 * of the Sec. 2 pair force (g = q - xi q', q(2) = 0):
 *   q(xi) = xi * integral_xi^2 g(t) / t^2 dt
 *         = 1 - 52/35 xi + 4/5 xi^3 - 2/5 xi^5 + 1/10 xi^6 + 2/35 xi^7 - 3/140 xi^8   (xi <= 1)
 *         = (2 - xi)^6 (xi^2 + 4 xi + 2) / 140                                       (1 <= xi <= 2)
 * and 0 beyond 2.  (1 - q)/r -> (52/35)(2/r_cut) as r -> 0: the potential of
 * a particle's own S2 cloud at its centre is -G m (104/35) / r_cut. */
double or_qcut(double xi) {
    if (xi > 2.0) return 0.0;
    if (xi <= 1.0) {
        double x2 = xi * xi, x3 = x2 * xi, x5 = x3 * x2, x6 = x5 * xi, x7 = x6 * xi, x8 = x7 * xi;
        return 1.0 - (52.0 / 35.0) * xi + 0.8 * x3 - 0.4 * x5 + 0.1 * x6 + (2.0 / 35.0) * x7 - (3.0 / 140.0) * x8;
    }
    double t = 2.0 - xi;
    return pow(t, 6.0) * (xi * xi + 4.0 * xi + 2.0) / 140.0;
}

void or_qcut_vec(int64_t n, const double* xi, double* q) {
    for (int64_t k = 0; k < n; ++k) q[k] = or_qcut(xi[k]);
}

void or_gcut_vec(int64_t n, const double* xi, double* g, double* dg) {
    for (int64_t k = 0; k < n; ++k) {
        g[k] = or_gcut(xi[k]);
        if (dg) dg[k] = or_gcut_deriv(xi[k]);
    }
}

void or_gcut_printed_vec(int64_t n, const double* xi, double* g) {
    for (int64_t k = 0; k < n; ++k) g[k] = or_gcut_printed(xi[k]);
}

/* phi(r) = (r^2 + eps^2)^(-3/2) * g(2 r / r_cut) for r < r_cut, else 0.
 * Sec. 2 force sum; the Plummer form replaces the delta function by a small
 * kernel (the paper's "small softening"), and the cutoff argument uses the
 * unsoftened distance, as in the force sum. */
static double phi_of(double r2, double rc, double eps) {
    if (!(r2 < rc * rc)) return 0.0;
    double r = sqrt(r2);
    double s2 = r2 + eps * eps;
    return or_gcut(2.0 * r / rc) / (s2 * sqrt(s2));
}

/* (d phi / d r) / r for 0 < r < r_cut (0 beyond).  Only used with r > 0. */
static double dphi_over_r(double r2, double rc, double eps) {
    if (!(r2 < rc * rc)) return 0.0;
    double r = sqrt(r2);
    double s2 = r2 + eps * eps;
    double s = sqrt(s2);
    double xi = 2.0 * r / rc;
    double dphidr = -3.0 * r / (s2 * s2 * s) * or_gcut(xi) + or_gcut_deriv(xi) * (2.0 / rc) / (s2 * s);
    return dphidr / r;
}

/* Pair force F(d) = d * phi(|d|) (the attraction of a unit source at offset d). */
void or_pair_force(double dx, double dy, double dz, double rc, double eps, double* f) {
    double p = phi_of(dx * dx + dy * dy + dz * dz, rc, eps);
    f[0] = dx * p; f[1] = dy * p; f[2] = dz * p;
}

/* J(d) w with J = dF/dd = phi I + (phi'/r) d d^T; at d = 0 only phi I. */
static void jac_times(double dx, double dy, double dz, double rc, double eps,
                      const double* w, double* out) {
    double r2 = dx * dx + dy * dy + dz * dz;
    double p = phi_of(r2, rc, eps);
    out[0] = p * w[0]; out[1] = p * w[1]; out[2] = p * w[2];
    if (r2 > 0.0) {
        double q = dphi_over_r(r2, rc, eps) * (dx * w[0] + dy * w[1] + dz * w[2]);
        out[0] += q * dx; out[1] += q * dy; out[2] += q * dz;
    }
}

void or_pair_jac(double dx, double dy, double dz, double rc, double eps, const double* w, double* out) {
    jac_times(dx, dy, dz, rc, eps, w, out);
}

/* Minimum image of one coordinate difference (periodic unit box). */
static double mimage(double d) { return d - rint(d); }

/* The periodic image of coordinate v nearest the reference point ref. */
static double near_image(double v, double ref) { return v - rint(v - ref); }

/* ================================================================== */
/* Brute force (the plain definition of the short-range sum)           */
/* ================================================================== */

/* O(N^2) minimum-image sum over all pairs; j = i contributes 0 (d = 0). */
void or_bf_n2(int64_t n, const double* x, const double* y, const double* z, const double* m,
              double G, double rc, double eps, double* ax, double* ay, double* az) {
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double a[3] = {0, 0, 0};
        for (int64_t j = 0; j < n; ++j) {
            double d[3] = {mimage(x[j] - x[i]), mimage(y[j] - y[i]), mimage(z[j] - z[i])};
            double p = phi_of(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], rc, eps);
            a[0] += m[j] * d[0] * p; a[1] += m[j] * d[1] * p; a[2] += m[j] * d[2] * p;
        }
        ax[i] = G * a[0]; ay[i] = G * a[1]; az[i] = G * a[2];
    }
}

/* Short-range potential of a unit source at squared distance r2: q(2r/r_cut)
 * over the softened distance (r^2 + eps^2)^(1/2), 0 at and beyond r_cut. */
static double pot_of(double r2, double rc, double eps) {
    if (!(r2 < rc * rc)) return 0.0;
    return or_qcut(2.0 * sqrt(r2) / rc) / sqrt(r2 + eps * eps);
}

/* O(N^2) short-range potential phi_i = -G sum_{j != i} m_j pot(d_ij). */
void or_bf_potential_n2(int64_t n, const double* x, const double* y, const double* z, const double* m,
                        double G, double rc, double eps, double* phi) {
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double a = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3] = {mimage(x[j] - x[i]), mimage(y[j] - y[i]), mimage(z[j] - z[i])};
            a += m[j] * pot_of(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], rc, eps);
        }
        phi[i] = -G * a;
    }
}

/* Cell list with cell side >= r_cut: every partner within r_cut lies in the
 * 27 cells around a particle's own cell.  Needs at least 3 cells per axis. */
typedef struct { int nc; int64_t* start; int64_t* idx; } cells_t;

static int cell_coord(double v, int nc) {
    double u = v - floor(v);
    if (u >= 1.0) u = 0.0;
    int c = (int)floor(u * nc);
    return c >= nc ? nc - 1 : c;
}

static int cells_build(int64_t n, const double* x, const double* y, const double* z, double rc, cells_t* cl) {
    int nc = (int)floor(1.0 / rc);
    if (nc > 256) nc = 256;
    if (nc < 3) return 0;
    int64_t ncell = (int64_t)nc * nc * nc;
    int64_t* cnt = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t* cid = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = ((int64_t)cell_coord(x[i], nc) * nc + cell_coord(y[i], nc)) * nc + cell_coord(z[i], nc);
        cid[i] = c; cnt[c + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) cnt[c + 1] += cnt[c];
    int64_t* fill = (int64_t*)malloc((size_t)ncell * sizeof(int64_t));
    memcpy(fill, cnt, (size_t)ncell * sizeof(int64_t));
    int64_t* idx = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) idx[fill[cid[i]]++] = i;
    free(fill); free(cid);
    cl->nc = nc; cl->start = cnt; cl->idx = idx;
    return 1;
}

static void cells_free(cells_t* cl) { free(cl->start); free(cl->idx); }

/* Exact short-range accelerations by brute force over the cell list.
 * Returns 0 on success, 1 if the box has fewer than 3 cells per axis
 * (then the O(N^2) routine is used instead). */
int or_bf_cells(int64_t n, const double* x, const double* y, const double* z, const double* m,
                double G, double rc, double eps, double* ax, double* ay, double* az) {
    cells_t cl;
    if (!cells_build(n, x, y, z, rc, &cl)) {
        or_bf_n2(n, x, y, z, m, G, rc, eps, ax, ay, az);
        return 1;
    }
    int nc = cl.nc;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int cx = cell_coord(x[i], nc), cy = cell_coord(y[i], nc), cz = cell_coord(z[i], nc);
        double a[3] = {0, 0, 0};
        for (int ox = -1; ox <= 1; ++ox)
        for (int oy = -1; oy <= 1; ++oy)
        for (int oz = -1; oz <= 1; ++oz) {
            int64_t c = ((int64_t)((cx + ox + nc) % nc) * nc + (cy + oy + nc) % nc) * nc + (cz + oz + nc) % nc;
            for (int64_t q = cl.start[c]; q < cl.start[c + 1]; ++q) {
                int64_t j = cl.idx[q];
                double d[3] = {mimage(x[j] - x[i]), mimage(y[j] - y[i]), mimage(z[j] - z[i])};
                double p = phi_of(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], rc, eps);
                a[0] += m[j] * d[0] * p; a[1] += m[j] * d[1] * p; a[2] += m[j] * d[2] * p;
            }
        }
        ax[i] = G * a[0]; ay[i] = G * a[1]; az[i] = G * a[2];
    }
    cells_free(&cl);
    return 0;
}

/* The same brute-force sum for a subset of target particles sel[0..nsel).
 * If `pairs` is not NULL it receives the number of (target, source) pairs
 * with 0 < r < r_cut that were summed. */
int or_bf_cells_sel(int64_t n, const double* x, const double* y, const double* z, const double* m,
                    double G, double rc, double eps, const int64_t* sel, int64_t nsel,
                    double* ax, double* ay, double* az, int64_t* pairs) {
    cells_t cl;
    int have = cells_build(n, x, y, z, rc, &cl);
    int nc = have ? cl.nc : 0;
    int64_t np = 0;
    #pragma omp parallel for schedule(dynamic, 16) reduction(+ : np)
    for (int64_t q = 0; q < nsel; ++q) {
        int64_t i = sel[q];
        double a[3] = {0, 0, 0};
        if (have) {
            int cx = cell_coord(x[i], nc), cy = cell_coord(y[i], nc), cz = cell_coord(z[i], nc);
            for (int ox = -1; ox <= 1; ++ox)
            for (int oy = -1; oy <= 1; ++oy)
            for (int oz = -1; oz <= 1; ++oz) {
                int64_t c = ((int64_t)((cx + ox + nc) % nc) * nc + (cy + oy + nc) % nc) * nc + (cz + oz + nc) % nc;
                for (int64_t t = cl.start[c]; t < cl.start[c + 1]; ++t) {
                    int64_t j = cl.idx[t];
                    double d[3] = {mimage(x[j] - x[i]), mimage(y[j] - y[i]), mimage(z[j] - z[i])};
                    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                    double p = phi_of(r2, rc, eps);
                    if (r2 > 0.0 && r2 < rc * rc) ++np;
                    a[0] += m[j] * d[0] * p; a[1] += m[j] * d[1] * p; a[2] += m[j] * d[2] * p;
                }
            }
        } else {
            for (int64_t j = 0; j < n; ++j) {
                double d[3] = {mimage(x[j] - x[i]), mimage(y[j] - y[i]), mimage(z[j] - z[i])};
                double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                double p = phi_of(r2, rc, eps);
                if (r2 > 0.0 && r2 < rc * rc) ++np;
                a[0] += m[j] * d[0] * p; a[1] += m[j] * d[1] * p; a[2] += m[j] * d[2] * p;
            }
        }
        ax[q] = G * a[0]; ay[q] = G * a[1]; az[q] = G * a[2];
    }
    if (pairs) *pairs = np;
    if (have) cells_free(&cl);
    return have ? 0 : 1;
}

/* Number of ordered pairs (i, j != i) closer than r_cut (cell list). */
int64_t or_bf_pair_count(int64_t n, const double* x, const double* y, const double* z, double rc) {
    cells_t cl;
    int64_t total = 0;
    if (!cells_build(n, x, y, z, rc, &cl)) {
        #pragma omp parallel for reduction(+:total)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double d[3] = {mimage(x[j] - x[i]), mimage(y[j] - y[i]), mimage(z[j] - z[i])};
                if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < rc * rc) total++;
            }
        return total;
    }
    int nc = cl.nc;
    #pragma omp parallel for schedule(dynamic, 64) reduction(+:total)
    for (int64_t i = 0; i < n; ++i) {
        int cx = cell_coord(x[i], nc), cy = cell_coord(y[i], nc), cz = cell_coord(z[i], nc);
        for (int ox = -1; ox <= 1; ++ox)
        for (int oy = -1; oy <= 1; ++oy)
        for (int oz = -1; oz <= 1; ++oz) {
            int64_t c = ((int64_t)((cx + ox + nc) % nc) * nc + (cy + oy + nc) % nc) * nc + (cz + oz + nc) % nc;
            for (int64_t q = cl.start[c]; q < cl.start[c + 1]; ++q) {
                int64_t j = cl.idx[q];
                if (j == i) continue;
                double d[3] = {mimage(x[j] - x[i]), mimage(y[j] - y[i]), mimage(z[j] - z[i])};
                if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < rc * rc) total++;
            }
        }
    }
    cells_free(&cl);
    return total;
}

/* Brute-force gradient of L = sum_i w_i . a_i:
 *   dL/dx_k = G sum_j J(x_j - x_k) (m_k w_j - m_j w_k)
 *   dL/dm_k = G sum_i w_i . F(x_k - x_i)
 * (J is even in d, so both the "i = k" and "j = k" terms use d = x_j - x_k.) */
void or_bf_adjoint(int64_t n, const double* x, const double* y, const double* z, const double* m,
                   const double* wx, const double* wy, const double* wz,
                   double G, double rc, double eps, double* gx, double* gy, double* gz, double* gm) {
    cells_t cl;
    int have_cells = cells_build(n, x, y, z, rc, &cl);
    int nc = have_cells ? cl.nc : 0;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < n; ++k) {
        double g3[3] = {0, 0, 0}, gmk = 0.0;
        int cx = 0, cy = 0, cz = 0;
        if (have_cells) { cx = cell_coord(x[k], nc); cy = cell_coord(y[k], nc); cz = cell_coord(z[k], nc); }
        int span = have_cells ? 1 : 0;
        for (int ox = -span; ox <= span; ++ox)
        for (int oy = -span; oy <= span; ++oy)
        for (int oz = -span; oz <= span; ++oz) {
            int64_t q0, q1;
            int64_t c = 0;
            if (have_cells) {
                c = ((int64_t)((cx + ox + nc) % nc) * nc + (cy + oy + nc) % nc) * nc + (cz + oz + nc) % nc;
                q0 = cl.start[c]; q1 = cl.start[c + 1];
            } else { q0 = 0; q1 = n; }
            for (int64_t q = q0; q < q1; ++q) {
                int64_t j = have_cells ? cl.idx[q] : q;
                if (j == k) continue;   /* j != i in the force sum */
                double d[3] = {mimage(x[j] - x[k]), mimage(y[j] - y[k]), mimage(z[j] - z[k])};
                double v[3] = {m[k] * wx[j] - m[j] * wx[k], m[k] * wy[j] - m[j] * wy[k], m[k] * wz[j] - m[j] * wz[k]};
                double jv[3];
                jac_times(d[0], d[1], d[2], rc, eps, v, jv);
                g3[0] += jv[0]; g3[1] += jv[1]; g3[2] += jv[2];
                /* F(x_k - x_j) = -F(d) */
                double p = phi_of(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], rc, eps);
                gmk -= (wx[j] * d[0] + wy[j] * d[1] + wz[j] * d[2]) * p;
            }
        }
        gx[k] = G * g3[0]; gy[k] = G * g3[1]; gz[k] = G * g3[2]; gm[k] = G * gmk;
    }
    if (have_cells) cells_free(&cl);
}

/* ================================================================== */
/* Morton keys and the stable sort                                     */
/* ================================================================== */

/* Wrap into [0,1): u = v - floor(v), and u == 1.0 (a tiny negative v)
 * becomes 0.0. */
double or_wrap(double v) {
    double u = v - floor(v);
    return u == 1.0 ? 0.0 : u;
}

/* Integer cell coordinate of a wrapped coordinate on the 2^21 grid. */
static uint32_t grid_coord(double u) {
    double c = floor(u * 2097152.0);       /* 2^21; the product is exact */
    if (c > 2097151.0) c = 2097151.0;
    return (uint32_t)c;
}

/* 63-bit Morton key: bit 3b+2 is bit b of the x coordinate, 3b+1 of y,
 * 3b of z (x most significant within each triple).  Written as a plain
 * loop over the 21 bit positions. */
uint64_t or_morton3(uint32_t ix, uint32_t iy, uint32_t iz) {
    uint64_t k = 0;
    for (int b = 0; b < KEY_BITS; ++b) {
        k |= (uint64_t)((ix >> b) & 1u) << (3 * b + 2);
        k |= (uint64_t)((iy >> b) & 1u) << (3 * b + 1);
        k |= (uint64_t)((iz >> b) & 1u) << (3 * b);
    }
    return k;
}

/* Keys of all particles in input order, and the wrapped positions. */
void or_morton_keys(int64_t n, const double* x, const double* y, const double* z,
                    uint64_t* keys, double* ux, double* uy, double* uz) {
    for (int64_t i = 0; i < n; ++i) {
        double a = or_wrap(x[i]), b = or_wrap(y[i]), c = or_wrap(z[i]);
        if (ux) { ux[i] = a; uy[i] = b; uz[i] = c; }
        keys[i] = or_morton3(grid_coord(a), grid_coord(b), grid_coord(c));
    }
}

typedef struct { uint64_t key; int64_t idx; } keyidx_t;

static int cmp_keyidx(const void* a, const void* b) {
    const keyidx_t* p = (const keyidx_t*)a;
    const keyidx_t* q = (const keyidx_t*)b;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    if (p->idx != q->idx) return p->idx < q->idx ? -1 : 1;
    return 0;
}

/* Order by (key, original index): a total order, so the permutation is
 * unique (the same as a stable sort by key). */
void or_sort(int64_t n, const uint64_t* keys, uint64_t* keys_sorted, int64_t* perm) {
    keyidx_t* t = (keyidx_t*)malloc((size_t)n * sizeof(keyidx_t));
    for (int64_t i = 0; i < n; ++i) { t[i].key = keys[i]; t[i].idx = i; }
    qsort(t, (size_t)n, sizeof(keyidx_t), cmp_keyidx);
    for (int64_t i = 0; i < n; ++i) { keys_sorted[i] = t[i].key; perm[i] = t[i].idx; }
    free(t);
}

/* ================================================================== */
/* Octree (Barnes-Hut cells over the Morton order)                     */
/* ================================================================== */

/* A cell at level L is the set of particles whose keys share the top 3L
 * bits (the prefix).  The root (level 0) is always split; any other cell
 * is split iff it holds more than n_leaf particles and L < 21.  Children
 * are the non-empty sub-cells, visited in octant order. */
typedef struct {
    const uint64_t* keys;
    int64_t n_leaf;
    int64_t next;
    int fill;
    int32_t* level; uint64_t* prefix; int64_t* first; int64_t* count;
    int64_t* parent; int64_t* child; uint8_t* leaf;
} tree_ctx;

static int64_t tree_rec(tree_ctx* c, int level, uint64_t prefix, int64_t first, int64_t count, int64_t parent) {
    int64_t id = c->next++;
    int split = (level == 0) || (level < MAX_LEVEL && count > c->n_leaf);
    if (c->fill) {
        c->level[id] = level; c->prefix[id] = prefix; c->first[id] = first; c->count[id] = count;
        c->parent[id] = parent; c->leaf[id] = (uint8_t)!split;
        for (int o = 0; o < 8; ++o) c->child[id * 8 + o] = -1;
    }
    if (!split) return id;
    int shift = 3 * (MAX_LEVEL - (level + 1));
    int64_t s = first, end = first + count;
    for (int o = 0; o < 8; ++o) {
        uint64_t cp = prefix * 8 + (uint64_t)o;
        int64_t e = s;
        while (e < end && (c->keys[e] >> shift) == cp) ++e;
        if (e > s) {
            int64_t cid = tree_rec(c, level + 1, cp, s, e - s, id);
            if (c->fill) c->child[id * 8 + o] = cid;
        }
        s = e;
    }
    return id;
}

int64_t or_tree_count(int64_t n, const uint64_t* keys_sorted, int64_t n_leaf) {
    tree_ctx c; memset(&c, 0, sizeof c);
    c.keys = keys_sorted; c.n_leaf = n_leaf;
    tree_rec(&c, 0, 0, 0, n, -1);
    return c.next;
}

void or_tree_fill(int64_t n, const uint64_t* keys_sorted, int64_t n_leaf,
                  int32_t* level, uint64_t* prefix, int64_t* first, int64_t* count,
                  int64_t* parent, int64_t* child, uint8_t* leaf) {
    tree_ctx c; memset(&c, 0, sizeof c);
    c.keys = keys_sorted; c.n_leaf = n_leaf; c.fill = 1;
    c.level = level; c.prefix = prefix; c.first = first; c.count = count;
    c.parent = parent; c.child = child; c.leaf = leaf;
    tree_rec(&c, 0, 0, 0, n, -1);
}

/* Monopole moments, directly from the definition: M = sum m, X = sum m x / M
 * over the particles of the cell (Sec. 1 multipole expansion of a cell,
 * truncated at the monopole with the centre of mass as expansion point).
 * Each position is taken at its periodic image nearest the cell's dyadic
 * centre: in a freshly built tree every particle lies inside its cell and
 * this is the position itself; in a tree reused after its particles moved
 * (refitted) a cell's particles may sit on both sides of a face of the unit
 * box, and the centre of mass is that of the images which lie together. */
static void cell_geom(int level, uint64_t prefix, double cen[3], double* side);

void or_moments(int64_t nn, const int32_t* level, const uint64_t* prefix, const int64_t* first,
                const int64_t* count, const double* ux, const double* uy, const double* uz, const double* m,
                double* M, double* X, double* Y, double* Z) {
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t c = 0; c < nn; ++c) {
        double cref[3], side, sm = 0, sx = 0, sy = 0, sz = 0;
        cell_geom(level[c], prefix[c], cref, &side);
        for (int64_t s = first[c]; s < first[c] + count[c]; ++s) {
            double vx = near_image(ux[s], cref[0]);
            double vy = near_image(uy[s], cref[1]);
            double vz = near_image(uz[s], cref[2]);
            sm += m[s]; sx += m[s] * vx; sy += m[s] * vy; sz += m[s] * vz;
        }
        M[c] = sm; X[c] = sx / sm; Y[c] = sy / sm; Z[c] = sz / sm;
    }
}

/* ================================================================== */
/* Groups (Barnes' modified algorithm: one list per particle group)    */
/* ================================================================== */

/* A candidate is a cell at level >= 1 with at most n_g particles whose
 * parent is the root or holds more than n_g.  Under a parent of level >= 1
 * consecutive candidate children (octant order) are merged while the
 * running total stays <= n_g; a non-candidate child or an overflow closes
 * the run.  Under the root every candidate child is its own group.  A
 * level-21 cell with more than n_g particles is cut into chunks of n_g. */
typedef struct {
    const int32_t* level; const int64_t* first; const int64_t* count; const int64_t* child;
    int64_t n_g;
    int64_t ng;
    int64_t* gfirst; int64_t* gcount;
} group_ctx;

static void emit_group(group_ctx* c, int64_t first, int64_t count) {
    c->gfirst[c->ng] = first; c->gcount[c->ng] = count; c->ng++;
}

static void group_rec(group_ctx* c, int64_t node) {
    if (c->level[node] == MAX_LEVEL) {
        for (int64_t s = 0; s < c->count[node]; s += c->n_g) {
            int64_t k = c->count[node] - s < c->n_g ? c->count[node] - s : c->n_g;
            emit_group(c, c->first[node] + s, k);
        }
        return;
    }
    int merge = c->level[node] >= 1;
    int64_t run_first = -1, run_count = 0;
    for (int o = 0; o < 8; ++o) {
        int64_t ch = c->child[node * 8 + o];
        if (ch < 0) continue;
        if (c->count[ch] <= c->n_g) {
            if (merge && run_first >= 0 && run_count + c->count[ch] <= c->n_g) {
                run_count += c->count[ch];
            } else {
                if (run_first >= 0) emit_group(c, run_first, run_count);
                run_first = c->first[ch]; run_count = c->count[ch];
            }
        } else {
            if (run_first >= 0) emit_group(c, run_first, run_count);
            run_first = -1; run_count = 0;
            group_rec(c, ch);
        }
    }
    if (run_first >= 0) emit_group(c, run_first, run_count);
}

/* Groups in order of first; gfirst/gcount need capacity n.  Returns the count. */
int64_t or_groups(const int32_t* level, const int64_t* first, const int64_t* count, const int64_t* child,
                  int64_t n_g, int64_t* gfirst, int64_t* gcount) {
    group_ctx c;
    c.level = level; c.first = first; c.count = count; c.child = child; c.n_g = n_g;
    c.ng = 0; c.gfirst = gfirst; c.gcount = gcount;
    group_rec(&c, 0);
    return c.ng;
}

/* Tight bounding box of each group's wrapped positions. */
void or_group_bbox(int64_t ng, const int64_t* gfirst, const int64_t* gcount,
                   const double* ux, const double* uy, const double* uz, double* lo, double* hi) {
    const double* u[3] = {ux, uy, uz};
    for (int64_t g = 0; g < ng; ++g)
        for (int a = 0; a < 3; ++a) {
            double l = u[a][gfirst[g]], h = l;
            for (int64_t s = gfirst[g]; s < gfirst[g] + gcount[g]; ++s) {
                if (u[a][s] < l) l = u[a][s];
                if (u[a][s] > h) h = u[a][s];
            }
            lo[3 * g + a] = l; hi[3 * g + a] = h;
        }
}

/* ================================================================== */
/* Interaction lists                                                    */
/* ================================================================== */

/* Integer coordinates of a cell from its prefix (de-interleave). */
static void cell_ints(int level, uint64_t prefix, int64_t* ix, int64_t* iy, int64_t* iz) {
    int64_t a = 0, b = 0, c = 0;
    for (int l = 0; l < level; ++l) {
        uint64_t t = (prefix >> (3 * l)) & 7u;
        a |= (int64_t)((t >> 2) & 1u) << l;
        b |= (int64_t)((t >> 1) & 1u) << l;
        c |= (int64_t)(t & 1u) << l;
    }
    *ix = a; *iy = b; *iz = c;
}

/* Geometric centre and side of a cell: exact dyadic numbers. */
static void cell_geom(int level, uint64_t prefix, double cen[3], double* side) {
    int64_t i[3];
    cell_ints(level, prefix, &i[0], &i[1], &i[2]);
    for (int a = 0; a < 3; ++a) cen[a] = ldexp((double)i[a] + 0.5, -level);
    *side = ldexp(1.0, -level);
}

/* Per-axis periodic gap between the cell centre and the group box, less
 * `half`; squared distance with the association ((x + y) + z). */
static double gap2(const double cen[3], const double cg[3], const double hg[3], double half_c) {
    double e[3];
    for (int a = 0; a < 3; ++a) {
        double t = fabs(cen[a] - cg[a]);
        double t2 = 1.0 - t;
        if (t2 < t) t = t2;
        double r = t - (half_c + hg[a]);
        e[a] = r > 0.0 ? r : 0.0;
    }
    return (e[0] * e[0] + e[1] * e[1]) + e[2] * e[2];
}

/* Cutoff pruning (Fig. 2: only sources within r_cut interact): the exact
 * periodic box-box distance between cell and group box is >= r_cut. */
static int prune_cell(const double cen[3], double side, const double cg[3], const double hg[3], double rc) {
    return gap2(cen, cg, hg, side * 0.5) >= rc * rc;
}

/* Opening criterion: accept the cell as one monopole iff side^2 <
 * theta^2 d^2, d = distance from the group box to `cen`: the cell's
 * geometric centre, or (centre-of-mass variant) its centre of mass. */
static int accept_cell(const double cen[3], double side, const double cg[3], const double hg[3], double theta) {
    double d2 = gap2(cen, cg, hg, 0.0);
    return side * side < (theta * theta) * d2;
}

/* Refitted tree (tree reuse across the substeps of a step). */

/* Box of every cell of a refitted tree: its particles' positions, each
 * moved by the whole number of box lengths that brings it nearest the
 * cell's dyadic centre, then min and max per axis; an inner cell takes the
 * union of its children's boxes, each moved the same way as a whole (by the
 * image of its centre).  Cells in preorder, so children follow parents. */
void or_refit_cell_boxes(int64_t nn, const int32_t* level, const uint64_t* prefix, const int64_t* first,
                         const int64_t* count, const int64_t* child, const uint8_t* leaf,
                         const double* ux, const double* uy, const double* uz, double* lo, double* hi) {
    const double* u[3] = {ux, uy, uz};
    for (int64_t c = nn - 1; c >= 0; --c) {
        double cref[3], side, l[3] = {INFINITY, INFINITY, INFINITY}, h[3] = {-INFINITY, -INFINITY, -INFINITY};
        cell_geom(level[c], prefix[c], cref, &side);
        if (leaf[c]) {
            for (int64_t s = first[c]; s < first[c] + count[c]; ++s)
                for (int a = 0; a < 3; ++a) {
                    double v = u[a][s] - rint(u[a][s] - cref[a]);
                    if (v < l[a]) l[a] = v;
                    if (v > h[a]) h[a] = v;
                }
        } else {
            for (int o = 0; o < 8; ++o) {
                int64_t ch = child[c * 8 + o];
                if (ch < 0) continue;
                for (int a = 0; a < 3; ++a) {
                    double sh = rint((lo[3 * ch + a] + hi[3 * ch + a]) * 0.5 - cref[a]);
                    double vl = lo[3 * ch + a] - sh, vh = hi[3 * ch + a] - sh;
                    if (vl < l[a]) l[a] = vl;
                    if (vh > h[a]) h[a] = vh;
                }
            }
        }
        for (int a = 0; a < 3; ++a) { lo[3 * c + a] = l[a]; hi[3 * c + a] = h[a]; }
    }
}

/* Box of every group of a refitted tree: positions moved to the image
 * nearest the group's first particle, then min and max per axis. */
void or_refit_group_bbox(int64_t ng, const int64_t* gfirst, const int64_t* gcount,
                         const double* ux, const double* uy, const double* uz, double* lo, double* hi) {
    const double* u[3] = {ux, uy, uz};
    for (int64_t g = 0; g < ng; ++g)
        for (int a = 0; a < 3; ++a) {
            double ref = u[a][gfirst[g]], l = ref, h = ref;
            for (int64_t s = gfirst[g]; s < gfirst[g] + gcount[g]; ++s) {
                double v = u[a][s] - rint(u[a][s] - ref);
                if (v < l) l = v;
                if (v > h) h = v;
            }
            lo[3 * g + a] = l; hi[3 * g + a] = h;
        }
}

/* A refitted tree (reused after its particles moved) measures each cell by
 * the box [lo, hi] of its particles (rounded outward, refit_qbox) instead of
 * its dyadic box: per
 * axis t = |cen_c - cg| taken to the nearest image (t -= rint(t), since the
 * boxes of a refitted tree may reach past the unit box), gap r = t - (half
 * + h_g), e = max(0, r), d^2 = (e_x e_x + e_y e_y) + e_z e_z; prune iff
 * d^2(half = the box's half sides) >= r_cut^2; accept iff s^2 < theta^2
 * d^2(half = 0), s the larger of the cell's dyadic side and the box's
 * longest side, cen_c the box's centre (or the centre of mass with that
 * criterion).  Since the box holds the cell's particles, a cell holding a
 * member of the group is then never accepted (d <= s sqrt(3)/2 for the
 * geometric criterion), also where the box has shrunk to a point. */
static double refit_gap2(const double cen[3], const double half[3], const double cg[3], const double hg[3]) {
    double e[3];
    for (int a = 0; a < 3; ++a) {
        double t = cen[a] - cg[a];
        t = fabs(t - rint(t));
        double r = t - (half[a] + hg[a]);
        e[a] = r > 0.0 ? r : 0.0;
    }
    return (e[0] * e[0] + e[1] * e[1]) + e[2] * e[2];
}

/* The box a refitted cell is measured by in the list decisions: its
 * particles' box [lo, hi] with every bound rounded outward to a multiple of
 * q = 2^-(level + 10) (1/1024 of the cell's side), so that the bounds are
 * stored exactly as 16-bit multiples of q from the cell's dyadic centre.  A
 * bound more than 32767 q from the centre cannot be stored: the cell is then
 * unbounded -- never pruned, never accepted -- and the function returns 0. */
static int refit_qbox(int level, uint64_t prefix, const double lo[3], const double hi[3], double ql[3],
                      double qh[3]) {
    int64_t ic[3];
    cell_ints(level, prefix, &ic[0], &ic[1], &ic[2]);
    int e = level + 10;
    for (int a = 0; a < 3; ++a) {
        int64_t kc = ic[a] * 1024 + 512;                 /* the centre in units of q */
        double kl = floor(ldexp(lo[a], e)), kh = ceil(ldexp(hi[a], e));
        if (kl - (double)kc < -32767.0 || kh - (double)kc > 32767.0) return 0;
        ql[a] = ldexp(kl, -e);
        qh[a] = ldexp(kh, -e);
    }
    return 1;
}

/* refit_qbox for every cell (for the tests): bounded[c] = 0 marks an
 * unbounded cell, whose qlo/qhi are then left at its box. */
void or_refit_qboxes(int64_t nn, const int32_t* level, const uint64_t* prefix, const double* lo, const double* hi,
                     double* qlo, double* qhi, uint8_t* bounded) {
    for (int64_t c = 0; c < nn; ++c) {
        bounded[c] = (uint8_t)refit_qbox(level[c], prefix[c], lo + 3 * c, hi + 3 * c, qlo + 3 * c, qhi + 3 * c);
        if (!bounded[c])
            for (int a = 0; a < 3; ++a) { qlo[3 * c + a] = lo[3 * c + a]; qhi[3 * c + a] = hi[3 * c + a]; }
    }
}

typedef struct {
    const int32_t* level; const uint64_t* prefix; const int64_t* first; const int64_t* count;
    const int64_t* child; const uint8_t* leaf;
    double rc, theta;
    const double *X, *Y, *Z;          /* centres of mass for the MAC, or NULL (geometric centre) */
    const double *clo, *chi;          /* refitted cell boxes [nn*3], or NULL (dyadic cells) */
    double cg[3], hg[3];
    int64_t np, nn;
    int64_t* pidx; int64_t* nidx;     /* NULL in the counting pass */
} list_ctx;

static void list_rec(list_ctx* c, int64_t node) {
    double cen[3], side;
    int accept;
    if (c->clo) {
        double half[3], zero[3] = {0.0, 0.0, 0.0}, hmax = 0.0, ql[3], qh[3];
        if (refit_qbox(c->level[node], c->prefix[node], c->clo + 3 * node, c->chi + 3 * node, ql, qh)) {
            for (int a = 0; a < 3; ++a) {
                cen[a] = (ql[a] + qh[a]) * 0.5;
                half[a] = (qh[a] - ql[a]) * 0.5;
                if (half[a] > hmax) hmax = half[a];
            }
            side = hmax + hmax;
            double dyadic = ldexp(1.0, -c->level[node]);
            if (dyadic > side) side = dyadic;
            if (refit_gap2(cen, half, c->cg, c->hg) >= c->rc * c->rc) return;
            double mac_cen[3] = {cen[0], cen[1], cen[2]};
            if (c->X) { mac_cen[0] = c->X[node]; mac_cen[1] = c->Y[node]; mac_cen[2] = c->Z[node]; }
            accept = side * side < (c->theta * c->theta) * refit_gap2(mac_cen, zero, c->cg, c->hg);
        } else {
            accept = 0;
        }
    } else {
        cell_geom(c->level[node], c->prefix[node], cen, &side);
        if (prune_cell(cen, side, c->cg, c->hg, c->rc)) return;
        double mac_cen[3] = {cen[0], cen[1], cen[2]};
        if (c->X) { mac_cen[0] = c->X[node]; mac_cen[1] = c->Y[node]; mac_cen[2] = c->Z[node]; }
        accept = accept_cell(mac_cen, side, c->cg, c->hg, c->theta);
    }
    if (accept) {
        if (c->nidx) c->nidx[c->nn] = node;
        c->nn++;
        return;
    }
    if (c->leaf[node]) {
        for (int64_t s = c->first[node]; s < c->first[node] + c->count[node]; ++s) {
            if (c->pidx) c->pidx[c->np] = s;
            c->np++;
        }
        return;
    }
    for (int o = 0; o < 8; ++o) {
        int64_t ch = c->child[node * 8 + o];
        if (ch >= 0) list_rec(c, ch);
    }
}

static void group_frame(const double* lo, const double* hi, int64_t g, double cg[3], double hg[3]) {
    for (int a = 0; a < 3; ++a) {
        cg[a] = (lo[3 * g + a] + hi[3 * g + a]) * 0.5;
        hg[a] = (hi[3 * g + a] - lo[3 * g + a]) * 0.5;
    }
}

/* Pass 1: particle and node entry counts per group (clo/chi: the boxes of
 * a refitted tree, or NULL). */
void or_lists_count(int64_t ng, const double* lo, const double* hi,
                    const int32_t* level, const uint64_t* prefix, const int64_t* first, const int64_t* count,
                    const int64_t* child, const uint8_t* leaf, double rc, double theta,
                    const double* X, const double* Y, const double* Z, const double* clo, const double* chi,
                    int64_t* np, int64_t* nn) {
    #pragma omp parallel for schedule(dynamic, 8)
    for (int64_t g = 0; g < ng; ++g) {
        list_ctx c;
        memset(&c, 0, sizeof c);
        c.level = level; c.prefix = prefix; c.first = first; c.count = count; c.child = child; c.leaf = leaf;
        c.rc = rc; c.theta = theta; c.X = X; c.Y = Y; c.Z = Z; c.clo = clo; c.chi = chi;
        group_frame(lo, hi, g, c.cg, c.hg);
        list_rec(&c, 0);
        np[g] = c.np; nn[g] = c.nn;
    }
}

/* Pass 2: entries at the given offsets.  DFS order gives the canonical
 * form directly: particle indices ascending, nodes in preorder. */
void or_lists_fill(int64_t ng, const double* lo, const double* hi,
                   const int32_t* level, const uint64_t* prefix, const int64_t* first, const int64_t* count,
                   const int64_t* child, const uint8_t* leaf, double rc, double theta,
                   const double* X, const double* Y, const double* Z, const double* clo, const double* chi,
                   const int64_t* poff, const int64_t* noff, int64_t* pidx, int64_t* nidx) {
    #pragma omp parallel for schedule(dynamic, 8)
    for (int64_t g = 0; g < ng; ++g) {
        list_ctx c;
        memset(&c, 0, sizeof c);
        c.level = level; c.prefix = prefix; c.first = first; c.count = count; c.child = child; c.leaf = leaf;
        c.rc = rc; c.theta = theta; c.X = X; c.Y = Y; c.Z = Z; c.clo = clo; c.chi = chi;
        group_frame(lo, hi, g, c.cg, c.hg);
        c.pidx = pidx + poff[g]; c.nidx = nidx + noff[g];
        list_rec(&c, 0);
    }
}

/* ================================================================== */
/* Same-list force and its adjoint                                     */
/* ================================================================== */

/* For every group g and member i: a_i = G [ sum_{j in P_g} m_j F(x_j - x_i)
 *                                         + sum_{c in M_g} M_c F(X_c - x_i) ].
 * All arrays are in sorted order; `sel`/`nsel` optionally restrict the
 * groups evaluated (nsel < 0: all groups). */
void or_tree_force(int64_t ng, const int64_t* gfirst, const int64_t* gcount,
                   const int64_t* poff, const int64_t* pidx, const int64_t* noff, const int64_t* nidx,
                   const double* ux, const double* uy, const double* uz, const double* m,
                   const double* NM, const double* NX, const double* NY, const double* NZ,
                   double G, double rc, double eps, const int64_t* sel, int64_t nsel,
                   double* ax, double* ay, double* az) {
    int64_t todo = nsel < 0 ? ng : nsel;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < todo; ++q) {
        int64_t g = nsel < 0 ? q : sel[q];
        for (int64_t i = gfirst[g]; i < gfirst[g] + gcount[g]; ++i) {
            double a[3] = {0, 0, 0};
            for (int64_t e = poff[g]; e < poff[g + 1]; ++e) {
                int64_t j = pidx[e];
                double d[3] = {mimage(ux[j] - ux[i]), mimage(uy[j] - uy[i]), mimage(uz[j] - uz[i])};
                double p = phi_of(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], rc, eps);
                a[0] += m[j] * d[0] * p; a[1] += m[j] * d[1] * p; a[2] += m[j] * d[2] * p;
            }
            for (int64_t e = noff[g]; e < noff[g + 1]; ++e) {
                int64_t c = nidx[e];
                double d[3] = {mimage(NX[c] - ux[i]), mimage(NY[c] - uy[i]), mimage(NZ[c] - uz[i])};
                double p = phi_of(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], rc, eps);
                a[0] += NM[c] * d[0] * p; a[1] += NM[c] * d[1] * p; a[2] += NM[c] * d[2] * p;
            }
            ax[i] = G * a[0]; ay[i] = G * a[1]; az[i] = G * a[2];
        }
    }
}

/* Same-list short-range potential (sorted order): particle and cell sources
 * of each group's list, the target itself left out. */
void or_tree_potential(int64_t ng, const int64_t* gfirst, const int64_t* gcount,
                       const int64_t* poff, const int64_t* pidx, const int64_t* noff, const int64_t* nidx,
                       const double* ux, const double* uy, const double* uz, const double* m,
                       const double* NM, const double* NX, const double* NY, const double* NZ,
                       double G, double rc, double eps, double* phi) {
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t g = 0; g < ng; ++g) {
        for (int64_t i = gfirst[g]; i < gfirst[g] + gcount[g]; ++i) {
            double a = 0.0;
            for (int64_t e = poff[g]; e < poff[g + 1]; ++e) {
                int64_t j = pidx[e];
                if (j == i) continue;
                double d[3] = {mimage(ux[j] - ux[i]), mimage(uy[j] - uy[i]), mimage(uz[j] - uz[i])};
                a += m[j] * pot_of(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], rc, eps);
            }
            for (int64_t e = noff[g]; e < noff[g + 1]; ++e) {
                int64_t c = nidx[e];
                double d[3] = {mimage(NX[c] - ux[i]), mimage(NY[c] - uy[i]), mimage(NZ[c] - uz[i])};
                a += NM[c] * pot_of(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], rc, eps);
            }
            phi[i] = -G * a;
        }
    }
}

/* ================================================================== */
/* Quadrupole term of a cell (accuracy variant)                        */
/* ================================================================== */

/* The multipole expansion of a cell (Sec. 1) taken one order past the
 * monopole.  With phi(r) = g(k r) / s^3 (k = 2 / r_cut, s^2 = r^2 + eps^2),
 * psi = phi'(r) / r and chi = psi'(r) / r, the pair force F(D) = D phi(|D|)
 * has the second derivatives
 *   d_a d_b F_c = psi (delta_bc D_a + delta_ab D_c + delta_ac D_b) + chi D_a D_b D_c,
 * so a cell of mass M, centre of mass X and second moments
 * S_ab = sum_k m_k (x_k - X)_a (x_k - X)_b pulls a target at offset D = X - x by
 *   M F(D) + 1/2 S_ab d_a d_b F(D)
 *   = M F(D) + psi S D + (psi tr(S) / 2 + chi (D . S D) / 2) D      (first-order term: 0 at the COM).
 * psi and chi follow from g, g' and g'' by the chain rule:
 *   psi = k g' / (r s^3) - 3 g / s^5,
 *   chi = k^2 g'' / (r^2 s^3) - k g' / (r^3 s^3) - 6 k g' / (r s^5) + 15 g / s^7. */
static void quad_coefs(double r2, double rc, double eps, double* psi, double* chi) {
    *psi = *chi = 0.0;
    if (!(r2 < rc * rc) || !(r2 > 0.0)) return;
    double r = sqrt(r2), k = 2.0 / rc, xi = k * r;
    double s2 = r2 + eps * eps, s = sqrt(s2), s3 = s2 * s, s5 = s3 * s2, s7 = s5 * s2;
    double g = or_gcut(xi), g1 = or_gcut_deriv(xi), g2 = or_gcut_deriv2(xi);
    *psi = k * g1 / (r * s3) - 3.0 * g / s5;
    *chi = k * k * g2 / (r2 * s3) - k * g1 / (r2 * r * s3) - 6.0 * k * g1 / (r * s5) + 15.0 * g / s7;
}

/* 1/2 S_ab d_a d_b F(D) for S = (xx, yy, zz, xy, xz, yz); 0 at and beyond r_cut. */
void or_quad_term(double dx, double dy, double dz, const double* S, double rc, double eps, double* out) {
    double psi, chi;
    quad_coefs(dx * dx + dy * dy + dz * dz, rc, eps, &psi, &chi);
    double sd[3] = {S[0] * dx + S[3] * dy + S[4] * dz,
                    S[3] * dx + S[1] * dy + S[5] * dz,
                    S[4] * dx + S[5] * dy + S[2] * dz};
    double dsd = dx * sd[0] + dy * sd[1] + dz * sd[2];
    double c = 0.5 * psi * (S[0] + S[1] + S[2]) + 0.5 * chi * dsd;
    out[0] = psi * sd[0] + c * dx;
    out[1] = psi * sd[1] + c * dy;
    out[2] = psi * sd[2] + c * dz;
}

/* Second moments about the centre of mass, directly from the definition:
 * S_c = sum_{k in c} m_k (x_k - X_c)(x_k - X_c)^T as (xx, yy, zz, xy, xz, yz)
 * with x_k at its image nearest the cell's dyadic centre, as in the centre of
 * mass. */
void or_second_moments(int64_t nn, const int32_t* level, const uint64_t* prefix, const int64_t* first,
                       const int64_t* count, const double* ux, const double* uy, const double* uz, const double* m,
                       const double* X, const double* Y, const double* Z, double* S) {
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t c = 0; c < nn; ++c) {
        double cref[3], side, a[6] = {0, 0, 0, 0, 0, 0};
        cell_geom(level[c], prefix[c], cref, &side);
        for (int64_t k = first[c]; k < first[c] + count[c]; ++k) {
            double dx = near_image(ux[k], cref[0]) - X[c], dy = near_image(uy[k], cref[1]) - Y[c];
            double dz = near_image(uz[k], cref[2]) - Z[c];
            a[0] += m[k] * dx * dx; a[1] += m[k] * dy * dy; a[2] += m[k] * dz * dz;
            a[3] += m[k] * dx * dy; a[4] += m[k] * dx * dz; a[5] += m[k] * dy * dz;
        }
        for (int q = 0; q < 6; ++q) S[c * 6 + q] = a[q];
    }
}

/* Quadrupole correction of the same-list force (sorted order): for every
 * group g, member i and cell c of its list, G * 1/2 S_c : dd F(X_c - x_i)
 * (minimum image).  Written, not added; `sel`/`nsel` as in or_tree_force. */
void or_tree_quad(int64_t ng, const int64_t* gfirst, const int64_t* gcount, const int64_t* noff,
                  const int64_t* nidx, const double* ux, const double* uy, const double* uz,
                  const double* NX, const double* NY, const double* NZ, const double* S,
                  double G, double rc, double eps, const int64_t* sel, int64_t nsel,
                  double* ax, double* ay, double* az) {
    int64_t todo = nsel < 0 ? ng : nsel;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < todo; ++q) {
        int64_t g = nsel < 0 ? q : sel[q];
        for (int64_t i = gfirst[g]; i < gfirst[g] + gcount[g]; ++i) {
            double a[3] = {0, 0, 0}, t[3];
            for (int64_t e = noff[g]; e < noff[g + 1]; ++e) {
                int64_t c = nidx[e];
                or_quad_term(mimage(NX[c] - ux[i]), mimage(NY[c] - uy[i]), mimage(NZ[c] - uz[i]), S + 6 * c, rc,
                             eps, t);
                a[0] += t[0]; a[1] += t[1]; a[2] += t[2];
            }
            ax[i] = G * a[0]; ay[i] = G * a[1]; az[i] = G * a[2];
        }
    }
}

/* Gradient of L = sum_i w_i . a_i with perm, tree, groups and lists held
 * fixed.  For each pair (i, source s of mass mu at y):
 *     dL/dx_i -= G mu J w_i,  dL/dy_s += G mu J w_i,  dL/dmu_s += G w_i . F(d).
 * Node sources then pass their gradients to member particles through
 * M_c = sum m_k and X_c = sum m_k x_k / M_c (x_k at its image nearest the
 * cell's dyadic centre, as in the moments):
 *     dL/dx_k += (m_k / M_c) dL/dX_c,
 *     dL/dm_k += dL/dM_c + (x_k - X_c) . dL/dX_c / M_c.
 * Scatter contributions are accumulated per thread and summed afterwards. */
void or_tree_adjoint(int64_t n, int64_t ng, const int64_t* gfirst, const int64_t* gcount,
                     const int64_t* poff, const int64_t* pidx, const int64_t* noff, const int64_t* nidx,
                     int64_t nnodes, const int64_t* nfirst, const int64_t* ncount, const int32_t* nlevel,
                     const uint64_t* nprefix,
                     const double* ux, const double* uy, const double* uz, const double* m,
                     const double* NM, const double* NX, const double* NY, const double* NZ,
                     const double* wx, const double* wy, const double* wz,
                     double G, double rc, double eps,
                     double* gx, double* gy, double* gz, double* gm) {
    int nt = or_num_threads();
    /* per-thread scatter buffers: particles (4 per particle) and nodes (4 per node) */
    double* pbuf = (double*)calloc((size_t)nt * (size_t)n * 4, sizeof(double));
    double* nbuf = (double*)calloc((size_t)nt * (size_t)nnodes * 4, sizeof(double));
    #pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* pb = pbuf + (size_t)tid * (size_t)n * 4;
        double* nb = nbuf + (size_t)tid * (size_t)nnodes * 4;
        #pragma omp for schedule(dynamic, 4)
        for (int64_t g = 0; g < ng; ++g) {
            for (int64_t i = gfirst[g]; i < gfirst[g] + gcount[g]; ++i) {
                double w[3] = {wx[i], wy[i], wz[i]};
                for (int64_t e = poff[g]; e < poff[g + 1]; ++e) {
                    int64_t j = pidx[e];
                    if (j == i) continue;   /* the force sum runs over j != i */
                    double d[3] = {mimage(ux[j] - ux[i]), mimage(uy[j] - uy[i]), mimage(uz[j] - uz[i])};
                    double jw[3];
                    jac_times(d[0], d[1], d[2], rc, eps, w, jw);
                    double p = phi_of(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], rc, eps);
                    for (int a = 0; a < 3; ++a) {
                        pb[4 * i + a] -= m[j] * jw[a];
                        pb[4 * j + a] += m[j] * jw[a];
                    }
                    pb[4 * j + 3] += (w[0] * d[0] + w[1] * d[1] + w[2] * d[2]) * p;
                }
                for (int64_t e = noff[g]; e < noff[g + 1]; ++e) {
                    int64_t c = nidx[e];
                    double d[3] = {mimage(NX[c] - ux[i]), mimage(NY[c] - uy[i]), mimage(NZ[c] - uz[i])};
                    double jw[3];
                    jac_times(d[0], d[1], d[2], rc, eps, w, jw);
                    double p = phi_of(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], rc, eps);
                    for (int a = 0; a < 3; ++a) {
                        pb[4 * i + a] -= NM[c] * jw[a];
                        nb[4 * c + a] += NM[c] * jw[a];
                    }
                    nb[4 * c + 3] += (w[0] * d[0] + w[1] * d[1] + w[2] * d[2]) * p;
                }
            }
        }
    }
    /* sum the per-thread buffers */
    double* P = (double*)calloc((size_t)n * 4, sizeof(double));
    double* Q = (double*)calloc((size_t)nnodes * 4, sizeof(double));
    #pragma omp parallel for
    for (int64_t k = 0; k < n * 4; ++k)
        for (int t = 0; t < nt; ++t) P[k] += pbuf[(size_t)t * (size_t)n * 4 + k];
    #pragma omp parallel for
    for (int64_t k = 0; k < nnodes * 4; ++k)
        for (int t = 0; t < nt; ++t) Q[k] += nbuf[(size_t)t * (size_t)nnodes * 4 + k];
    free(pbuf); free(nbuf);
    /* node sources -> member particles, node by node over its range */
    for (int64_t c = 0; c < nnodes; ++c) {
        double gX[3] = {Q[4 * c], Q[4 * c + 1], Q[4 * c + 2]}, gM = Q[4 * c + 3];
        if (gX[0] == 0.0 && gX[1] == 0.0 && gX[2] == 0.0 && gM == 0.0) continue;
        double cref[3], side;
        cell_geom(nlevel[c], nprefix[c], cref, &side);
        for (int64_t k = nfirst[c]; k < nfirst[c] + ncount[c]; ++k) {
            double f = m[k] / NM[c];
            double o[3] = {near_image(ux[k], cref[0]) - NX[c], near_image(uy[k], cref[1]) - NY[c],
                           near_image(uz[k], cref[2]) - NZ[c]};
            P[4 * k] += f * gX[0]; P[4 * k + 1] += f * gX[1]; P[4 * k + 2] += f * gX[2];
            P[4 * k + 3] += gM + (o[0] * gX[0] + o[1] * gX[1] + o[2] * gX[2]) / NM[c];
        }
    }
    for (int64_t k = 0; k < n; ++k) {
        gx[k] = G * P[4 * k]; gy[k] = G * P[4 * k + 1]; gz[k] = G * P[4 * k + 2]; gm[k] = G * P[4 * k + 3];
    }
    free(P); free(Q);
}

/* ================================================================== */
/* First-order error magnitudes of the same-list force and gradient    */
/* ================================================================== */

/* The parity tests compare a kernel that evaluates each pair on offsets from
 * its group's centre, rounded to a working precision with unit roundoff
 * u_k, against the FP64 results above.  These functions return, for every
 * particle, a magnitude E such that a result whose every pair term carries
 * errors of the sizes below differs from the exact one by at most a small
 * multiple of E (the multiple, set by how many terms are summed in working
 * precision, is the test's constant):
 *   - each position enters the pair through d = o_s - o_i, o_i = x_i - c_g,
 *     o_s = image of x_s - c_g (c_g the centre of the group's box); rounding
 *     o_i, o_s and d perturbs d by at most u_k (|d| + |o_i| + |o_s|);
 *   - e_abs: a further absolute perturbation of every d (a test moves every
 *     particle by at most e_abs / 2);
 *   - a cell's centre of mass and mass are sums of its n_c particles, exact
 *     up to u_c (2 n_c + 2) in position (|x| <= 1) and relative in mass.
 * With J = dF/dd = phi I + psi d d^T (psi = phi'/r, chi = psi'/r):
 *   ||J|| <= nJ = |phi| + |psi| r^2,
 *   ||dJ/dd|| (as a map of two vectors) <= nH = 3 |psi| r + |chi| r^3,
 * so a perturbation e of d changes F by at most nJ e and J w by at most
 * nH e |w|; a relative rounding u_k of the pair arithmetic changes F by at
 * most u_k nJ |d| and J w by u_k nJ |w|.  Self pairs (d = 0 from the same
 * particle) contribute nothing and are skipped, as in the sums. */
static void bound_coefs(double r2, double rc, double eps, double* nJ, double* nH) {
    *nJ = *nH = 0.0;
    if (!(r2 < rc * rc)) return;
    double p = phi_of(r2, rc, eps);
    if (!(r2 > 0.0)) { *nJ = fabs(p); return; }
    double psi, chi, r = sqrt(r2);
    quad_coefs(r2, rc, eps, &psi, &chi);
    *nJ = fabs(p) + fabs(psi) * r2;
    *nH = 3.0 * fabs(psi) * r + fabs(chi) * r * r2;
}

static double norm3(double a, double b, double c) { return sqrt(a * a + b * b + c * c); }

/* Position uncertainty of one pair (see above); `nc` < 0 for a particle source. */
static double pair_unc(const double d[3], const double oi[3], const double os[3], double u_k, double u_c,
                       double e_abs, int64_t nc) {
    double e = u_k * (norm3(d[0], d[1], d[2]) + norm3(oi[0], oi[1], oi[2]) + norm3(os[0], os[1], os[2])) + e_abs;
    if (nc >= 0) e += u_c * (2.0 * (double)nc + 2.0);
    return e;
}

/* Force: E_i = |G| sum over the list of mu nJ e_pair (sorted order; sel/nsel
 * as in or_tree_force). */
void or_tree_force_bound(int64_t ng, const int64_t* gfirst, const int64_t* gcount,
                         const int64_t* poff, const int64_t* pidx, const int64_t* noff, const int64_t* nidx,
                         const double* ux, const double* uy, const double* uz, const double* m,
                         const double* NM, const double* NX, const double* NY, const double* NZ,
                         const int64_t* ncount, const double* lo, const double* hi,
                         double G, double rc, double eps, double u_k, double u_c, double e_abs,
                         const int64_t* sel, int64_t nsel, double* E) {
    int64_t todo = nsel < 0 ? ng : nsel;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < todo; ++q) {
        int64_t g = nsel < 0 ? q : sel[q];
        double cg[3], hg[3];
        group_frame(lo, hi, g, cg, hg);
        for (int64_t i = gfirst[g]; i < gfirst[g] + gcount[g]; ++i) {
            double oi[3] = {mimage(ux[i] - cg[0]), mimage(uy[i] - cg[1]), mimage(uz[i] - cg[2])};
            double acc = 0.0, nJ, nH;
            for (int64_t e = poff[g]; e < poff[g + 1]; ++e) {
                int64_t j = pidx[e];
                if (j == i) continue;
                double d[3] = {mimage(ux[j] - ux[i]), mimage(uy[j] - uy[i]), mimage(uz[j] - uz[i])};
                double os[3] = {mimage(ux[j] - cg[0]), mimage(uy[j] - cg[1]), mimage(uz[j] - cg[2])};
                bound_coefs(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], rc, eps, &nJ, &nH);
                acc += m[j] * nJ * pair_unc(d, oi, os, u_k, u_c, e_abs, -1);
            }
            for (int64_t e = noff[g]; e < noff[g + 1]; ++e) {
                int64_t c = nidx[e];
                double d[3] = {mimage(NX[c] - ux[i]), mimage(NY[c] - uy[i]), mimage(NZ[c] - uz[i])};
                double os[3] = {mimage(NX[c] - cg[0]), mimage(NY[c] - cg[1]), mimage(NZ[c] - cg[2])};
                bound_coefs(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], rc, eps, &nJ, &nH);
                acc += NM[c] * nJ * pair_unc(d, oi, os, u_k, u_c, e_abs, ncount[c]);
            }
            E[i] = fabs(G) * acc;
        }
    }
}

/* Gradient: per pair (target i with weight w, source of mass mu), with e the
 * pair's position uncertainty,
 *   error of J w:      |w| (u_k nJ + nH e)  -> to dL/dx of the target (x mu) and of the source,
 *   error of w . F:    |w| nJ e             -> to dL/dm of the source;
 * a cell source collects them (EX with its mass, EM) together with
 * GX >= |dL/dX_c| and passes them to its particles k as the chain rule does:
 *   Ex_k += (m_k / M_c) (EX + GX u_c (2 n_c + 2)),
 *   Em_k += EM + |x_k - X_c| EX / M_c + (GX / M_c) (e_abs + u_c (2 n_c + 2)).
 * Outputs in sorted order, times |G|. */
void or_tree_adjoint_bound(int64_t n, int64_t ng, const int64_t* gfirst, const int64_t* gcount,
                           const int64_t* poff, const int64_t* pidx, const int64_t* noff, const int64_t* nidx,
                           int64_t nnodes, const int64_t* nfirst, const int64_t* ncount, const int32_t* nlevel,
                     const uint64_t* nprefix,
                           const double* ux, const double* uy, const double* uz, const double* m,
                           const double* NM, const double* NX, const double* NY, const double* NZ,
                           const double* wx, const double* wy, const double* wz, const double* lo, const double* hi,
                           double G, double rc, double eps, double u_k, double u_c, double e_abs,
                           double* Ex, double* Em) {
    int nt = or_num_threads();
    /* per-thread accumulators: particles (Ex, Em) and cells (EX, EM, GX) */
    double* pbuf = (double*)calloc((size_t)nt * (size_t)n * 2, sizeof(double));
    double* nbuf = (double*)calloc((size_t)nt * (size_t)nnodes * 3, sizeof(double));
    #pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* pb = pbuf + (size_t)tid * (size_t)n * 2;
        double* nb = nbuf + (size_t)tid * (size_t)nnodes * 3;
        #pragma omp for schedule(dynamic, 4)
        for (int64_t g = 0; g < ng; ++g) {
            double cg[3], hg[3];
            group_frame(lo, hi, g, cg, hg);
            for (int64_t i = gfirst[g]; i < gfirst[g] + gcount[g]; ++i) {
                double oi[3] = {mimage(ux[i] - cg[0]), mimage(uy[i] - cg[1]), mimage(uz[i] - cg[2])};
                double wn = norm3(wx[i], wy[i], wz[i]), nJ, nH;
                for (int64_t e = poff[g]; e < poff[g + 1]; ++e) {
                    int64_t j = pidx[e];
                    if (j == i) continue;
                    double d[3] = {mimage(ux[j] - ux[i]), mimage(uy[j] - uy[i]), mimage(uz[j] - uz[i])};
                    double os[3] = {mimage(ux[j] - cg[0]), mimage(uy[j] - cg[1]), mimage(uz[j] - cg[2])};
                    bound_coefs(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], rc, eps, &nJ, &nH);
                    double un = pair_unc(d, oi, os, u_k, u_c, e_abs, -1);
                    double tV = wn * (u_k * nJ + nH * un);
                    pb[2 * i] += m[j] * tV;
                    pb[2 * j] += m[j] * tV;
                    pb[2 * j + 1] += wn * nJ * un;
                }
                for (int64_t e = noff[g]; e < noff[g + 1]; ++e) {
                    int64_t c = nidx[e];
                    double d[3] = {mimage(NX[c] - ux[i]), mimage(NY[c] - uy[i]), mimage(NZ[c] - uz[i])};
                    double os[3] = {mimage(NX[c] - cg[0]), mimage(NY[c] - cg[1]), mimage(NZ[c] - cg[2])};
                    bound_coefs(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], rc, eps, &nJ, &nH);
                    double un = pair_unc(d, oi, os, u_k, u_c, e_abs, ncount[c]);
                    double tV = wn * (u_k * nJ + nH * un);
                    pb[2 * i] += NM[c] * tV;
                    nb[3 * c] += NM[c] * tV;
                    nb[3 * c + 1] += wn * nJ * un;
                    nb[3 * c + 2] += NM[c] * wn * nJ;
                }
            }
        }
    }
    double* P = (double*)calloc((size_t)n * 2, sizeof(double));
    double* Q = (double*)calloc((size_t)nnodes * 3, sizeof(double));
    #pragma omp parallel for
    for (int64_t k = 0; k < n * 2; ++k)
        for (int t = 0; t < nt; ++t) P[k] += pbuf[(size_t)t * (size_t)n * 2 + k];
    #pragma omp parallel for
    for (int64_t k = 0; k < nnodes * 3; ++k)
        for (int t = 0; t < nt; ++t) Q[k] += nbuf[(size_t)t * (size_t)nnodes * 3 + k];
    free(pbuf); free(nbuf);
    for (int64_t c = 0; c < nnodes; ++c) {
        double EXc = Q[3 * c], EMc = Q[3 * c + 1], GXc = Q[3 * c + 2];
        if (EXc == 0.0 && EMc == 0.0 && GXc == 0.0) continue;
        double uc = u_c * (2.0 * (double)ncount[c] + 2.0), cref[3], side;
        cell_geom(nlevel[c], nprefix[c], cref, &side);
        for (int64_t k = nfirst[c]; k < nfirst[c] + ncount[c]; ++k) {
            double o[3] = {near_image(ux[k], cref[0]) - NX[c], near_image(uy[k], cref[1]) - NY[c],
                           near_image(uz[k], cref[2]) - NZ[c]};
            P[2 * k] += (m[k] / NM[c]) * (EXc + GXc * uc);
            P[2 * k + 1] += EMc + norm3(o[0], o[1], o[2]) * EXc / NM[c]
                          + (GXc / NM[c]) * (e_abs + uc);
        }
    }
    for (int64_t k = 0; k < n; ++k) {
        Ex[k] = fabs(G) * P[2 * k];
        Em[k] = fabs(G) * P[2 * k + 1];
    }
    free(P); free(Q);
}
