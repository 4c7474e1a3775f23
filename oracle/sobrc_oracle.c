/* sobrc_oracle.c -- plain FP64 reference for the per-iteration hot path of
 * particle-based Region Competition with particle-approximated Sobolev
 * gradients (Sbalzarini, Schneider, Cardinale, arXiv:1403.0240).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  Written to be
 * read against the paper, not to be fast: every step is a direct loop in FP64,
 * single pass, no blocking or fusion.  OpenMP (optional, ora_params.threads)
 * only splits independent per-particle loops; results do not depend on it.
 *
 * Readings of points the paper leaves open (all follow the paper's text where
 * it speaks):
 *  - particles sit on both sides of the contour, one per pixel and per
 *    distinct neighbouring label in the full 8/26 neighbourhood (Fig. 1 and the
 *    two-sided storage described with Eq. (6));
 *  - Q_p / Q'_p match the ordered label pair (a, b) / swapped pair (b, a), which
 *    is the paper's set definition when there are two labels; p is in Q_p;
 *  - the support test is strict, d < E/2, with Euclidean distance between pixel
 *    centres standing in for geodesic distance (as the paper does);
 *  - an empty Q'_p contributes nothing (the paper leaves 0/0 undefined);
 *  - the smoothing is a Jacobi update: all sums read the un-smoothed values;
 *  - piecewise-constant data term: exact change of sum (I - mu)^2 when one pixel
 *    moves, with both region means re-estimated (theta_i = region mean);
 *  - piecewise-smooth data term: local means over a closed ball of radius R;
 *  - Poisson noise (ORA_POISSON): pixel energy J - I log J; a move changes it
 *    with both expected intensities held at their current values (region
 *    means for PC, local means for PS), means below 1e-6 raised to 1e-6;
 *  - deconvolving model (psf_sigma > 0): separable Gaussian PSF truncated at
 *    3 sigma, zero outside the image; theta by least squares over the image
 *    for the labels at the start of the iteration, held fixed for every move;
 *  - length prior: number of face-adjacent pixel pairs with different labels;
 *  - acceptance: every particle with gradient < 0 is a candidate, per pixel the
 *    smallest gradient wins (ties: smaller target label), all chosen moves are
 *    applied together (no topology control);
 *  - topological control (ORA_TOPO_SIMPLE): candidates ranked by (gradient,
 *    pixel, target label) and executed in that order; a move runs only if
 *    its pixel is a simple point (26/6 connectivity, 8/4 in 2D) of both
 *    foreground regions it touches; background (label 0) is not controlled;
 *  - oscillation (AUTO mode): an iteration oscillates when at least half of
 *    its flips revert pixels that changed in the iteration before; after two
 *    oscillating iterations in a row, L2-type gradients are used from the
 *    next iteration on (ora_reversals, ora_run); with a flip tolerance, two
 *    L2 iterations in a row in which every flip is a reversal (a settled
 *    period-2 cycle) also end the run: the contour sits in a minimum at
 *    pixel resolution.
 *
 * parity unpinned: whole-run segmentations against the paper's figures (the
 * paper's images are not available).
 */
#include "sobrc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static int64_t lin_of(const ora_params* P, int x, int y, int z)
{
    return (int64_t)x + (int64_t)P->nx * ((int64_t)y + (int64_t)P->ny * z);
}

static void coords_of(const ora_params* P, int64_t i, int* x, int* y, int* z)
{
    *x = (int)(i % P->nx);
    *y = (int)((i / P->nx) % P->ny);
    *z = (int)(i / ((int64_t)P->nx * P->ny));
}

static int in_bounds(const ora_params* P, int x, int y, int z)
{
    return x >= 0 && x < P->nx && y >= 0 && y < P->ny && z >= 0 && z < P->nz;
}

static int zrange(const ora_params* P)
{
    return P->ndim == 3 ? 1 : 0;
}

static int nthreads(const ora_params* P)
{
    return P->threads > 1 ? P->threads : 1;
}

/* Eq. (5): K(r) = (1/E) (1 + ((|r|/E)^2 - |r|/E + 1/6) / (2 eps)) for
 * r in [-E/2, E/2]; outside that interval the kernel has no support. */
double ora_kernel(double r, double E, double eps)
{
    double u = fabs(r) / E;
    if (u > 0.5)
        return 0.0;
    return (1.0 + (u * u - u + 1.0 / 6.0) / (2.0 * eps)) / E;
}

/* Particles at contour pixels on both sides of the contour (Fig. 1 caption;
 * particles store L2 gradients on both sides, text before Eq. (6)). */
int64_t ora_particles(const ora_params* P, const int32_t* L, int64_t cap,
                      int64_t* lin, int32_t* a, int32_t* b)
{
    int64_t count = 0;
    int zr = zrange(P);
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                int64_t i = lin_of(P, x, y, z);
                int32_t own = L[i];
                /* distinct neighbouring labels, emitted in ascending order */
                int32_t prev = -1;
                for (;;) {
                    int32_t next = -1;
                    for (int dz = -zr; dz <= zr; ++dz)
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dx = -1; dx <= 1; ++dx) {
                                if (!dx && !dy && !dz)
                                    continue;
                                int xx = x + dx, yy = y + dy, zz = z + dz;
                                if (!in_bounds(P, xx, yy, zz))
                                    continue;
                                int32_t l = L[lin_of(P, xx, yy, zz)];
                                if (l == own || l <= prev)
                                    continue;
                                if (next < 0 || l < next)
                                    next = l;
                            }
                    if (next < 0)
                        break;
                    if (count < cap) {
                        lin[count] = i;
                        a[count] = own;
                        b[count] = next;
                    }
                    ++count;
                    prev = next;
                }
            }
    return count;
}

/* Photometric estimate: region intensity = mean intensity of the region
 * (Bayesian image models, Methods). */
void ora_region_stats(const ora_params* P, const double* I, const int32_t* L,
                      int64_t* n, double* s1, double* s2)
{
    int64_t nvox = (int64_t)P->nx * P->ny * P->nz;
    for (int l = 0; l < P->max_labels; ++l) {
        n[l] = 0;
        s1[l] = 0.0;
        s2[l] = 0.0;
    }
    for (int64_t i = 0; i < nvox; ++i) {
        int32_t l = L[i];
        n[l] += 1;
        s1[l] += I[i];
        s2[l] += I[i] * I[i];
    }
}

/* Number of face neighbours (4 in 2D, 6 in 3D) of pixel (x,y,z) carrying label l. */
static int face_count(const ora_params* P, const int32_t* L, int x, int y, int z, int32_t l)
{
    static const int off[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
    int c = 0;
    int nf = P->ndim == 3 ? 6 : 4;
    for (int k = 0; k < nf; ++k) {
        int xx = x + off[k][0], yy = y + off[k][1], zz = z + off[k][2];
        if (in_bounds(P, xx, yy, zz) && L[lin_of(P, xx, yy, zz)] == l)
            ++c;
    }
    return c;
}

/* L2-type gradient of a single particle move: energy difference between the
 * perturbed and the original contour (Eq. (11)), with the energy
 * E_ext + lambda E_int of Eq. (10), i.i.d. Gaussian pixel noise (squared
 * residuals) and a contour-length prior. */
/* Poisson pixel energy J - v log J (Methods: negative log-likelihood of
 * independent Poisson noise, constant log v! dropped) of a move from an
 * expected intensity m_a to m_b, both held at their current values. */
static double poisson_move(double v, double m_a, double m_b)
{
    double ja = m_a > ORA_POISSON_MIN_MEAN ? m_a : ORA_POISSON_MIN_MEAN;
    double jb = m_b > ORA_POISSON_MIN_MEAN ? m_b : ORA_POISSON_MIN_MEAN;
    return (jb - v * log(jb)) - (ja - v * log(ja));
}

/* --- deconvolving model (Eq. (8)) ---------------------------------------- */

int32_t ora_psf_radius(double sigma)
{
    return (int32_t)ceil(3.0 * sigma);
}

void ora_psf_taps(double sigma, double* taps)
{
    int r = ora_psf_radius(sigma);
    double sum = 0.0;
    for (int t = -r; t <= r; ++t) {
        taps[t + r] = exp(-(double)(t * t) / (2.0 * sigma * sigma));
        sum += taps[t + r];
    }
    for (int t = -r; t <= r; ++t)
        taps[t + r] /= sum;
}

/* out(y) = sum over image pixels x with |y - x| <= r per axis of
 * K(y - x) f(x), written out directly (no separable passes). */
static void psf_apply(const ora_params* P, const double* f, double* out)
{
    int r = ora_psf_radius(P->psf_sigma);
    double* k = (double*)malloc(sizeof(double) * (size_t)(2 * r + 1));
    ora_psf_taps(P->psf_sigma, k);
    int rz = P->ndim == 3 ? r : 0;
    int64_t nvox = (int64_t)P->nx * P->ny * P->nz;
#pragma omp parallel for schedule(static) num_threads(nthreads(P)) if (nthreads(P) > 1)
    for (int64_t i = 0; i < nvox; ++i) {
        int x, y, z;
        coords_of(P, i, &x, &y, &z);
        double acc = 0.0;
        for (int dz = -rz; dz <= rz; ++dz)
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    if (!in_bounds(P, x + dx, y + dy, z + dz))
                        continue;
                    double kk = k[dx + r] * k[dy + r] * (P->ndim == 3 ? k[dz + r] : 1.0);
                    acc += kk * f[lin_of(P, x + dx, y + dy, z + dz)];
                }
        out[i] = acc;
    }
    free(k);
}

/* Solve the n x n system A t = c in place (Gaussian elimination with partial
 * pivoting).  Returns 0 if a pivot vanishes. */
static int solve_dense(int n, double* A, double* c, double* t)
{
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(A[r * n + col]) > fabs(A[piv * n + col]))
                piv = r;
        if (A[piv * n + col] == 0.0)
            return 0;
        if (piv != col) {
            for (int j = 0; j < n; ++j) {
                double tmp = A[col * n + j];
                A[col * n + j] = A[piv * n + j];
                A[piv * n + j] = tmp;
            }
            double tmp = c[col];
            c[col] = c[piv];
            c[piv] = tmp;
        }
        for (int r = col + 1; r < n; ++r) {
            double f = A[r * n + col] / A[col * n + col];
            for (int j = col; j < n; ++j)
                A[r * n + j] -= f * A[col * n + j];
            c[r] -= f * c[col];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double acc = c[r];
        for (int j = r + 1; j < n; ++j)
            acc -= A[r * n + j] * t[j];
        t[r] = acc / A[r * n + r];
    }
    return 1;
}

void ora_deconv_theta(const ora_params* P, const double* I, const int32_t* L, double* theta)
{
    int M = P->max_labels;
    int64_t nvox = (int64_t)P->nx * P->ny * P->nz;
    /* u_l = K * chi_l for the labels present */
    int* idx = (int*)malloc(sizeof(int) * (size_t)M);
    int n = 0;
    for (int l = 0; l < M; ++l) {
        idx[l] = -1;
        theta[l] = 0.0;
        for (int64_t i = 0; i < nvox; ++i)
            if (L[i] == l) {
                idx[l] = n++;
                break;
            }
    }
    double* u = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)nvox);
    double* chi = (double*)malloc(sizeof(double) * (size_t)nvox);
    for (int l = 0; l < M; ++l) {
        if (idx[l] < 0)
            continue;
        for (int64_t i = 0; i < nvox; ++i)
            chi[i] = L[i] == l ? 1.0 : 0.0;
        psf_apply(P, chi, u + (size_t)idx[l] * (size_t)nvox);
    }
    /* normal equations of min sum (I - sum_l theta_l u_l)^2 */
    double* A = (double*)calloc((size_t)(n * n > 0 ? n * n : 1), sizeof(double));
    double* c = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double* t = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (int p = 0; p < n; ++p) {
        const double* up = u + (size_t)p * (size_t)nvox;
        for (int q = 0; q < n; ++q) {
            const double* uq = u + (size_t)q * (size_t)nvox;
            double acc = 0.0;
            for (int64_t i = 0; i < nvox; ++i)
                acc += up[i] * uq[i];
            A[p * n + q] = acc;
        }
        double acc = 0.0;
        for (int64_t i = 0; i < nvox; ++i)
            acc += up[i] * I[i];
        c[p] = acc;
    }
    if (n > 0 && solve_dense(n, A, c, t))
        for (int l = 0; l < M; ++l)
            if (idx[l] >= 0)
                theta[l] = t[idx[l]];
    free(idx);
    free(u);
    free(chi);
    free(A);
    free(c);
    free(t);
}

void ora_deconv_model(const ora_params* P, const int32_t* L, const double* theta, double* J)
{
    int64_t nvox = (int64_t)P->nx * P->ny * P->nz;
    double* s = (double*)malloc(sizeof(double) * (size_t)nvox);
    for (int64_t i = 0; i < nvox; ++i)
        s[i] = theta[L[i]];
    psf_apply(P, s, J);
    free(s);
}

/* Data term of moving pixel i by delta under the deconvolving model: the
 * change of sum_y (R(y) - delta K(y - x))^2 over the image, R = I - J. */
static double deconv_move(const ora_params* P, const double* R, const double* k, int r, int64_t i, double delta)
{
    int x, y, z;
    coords_of(P, i, &x, &y, &z);
    int rz = P->ndim == 3 ? r : 0;
    double d = 0.0;
    for (int dz = -rz; dz <= rz; ++dz)
        for (int dy = -r; dy <= r; ++dy)
            for (int dx = -r; dx <= r; ++dx) {
                if (!in_bounds(P, x + dx, y + dy, z + dz))
                    continue;
                double kk = k[dx + r] * k[dy + r] * (P->ndim == 3 ? k[dz + r] : 1.0);
                double rv = R[lin_of(P, x + dx, y + dy, z + dz)];
                d += (rv - delta * kk) * (rv - delta * kk) - rv * rv;
            }
    return d;
}

void ora_l2diff(const ora_params* P, const double* I, const int32_t* L,
                int64_t np, const int64_t* lin, const int32_t* a, const int32_t* b,
                double* dE)
{
    if (P->psf_sigma > 0.0) {
        int M = P->max_labels;
        int64_t nvox = (int64_t)P->nx * P->ny * P->nz;
        int r = ora_psf_radius(P->psf_sigma);
        double* theta = (double*)malloc(sizeof(double) * (size_t)M);
        double* R = (double*)malloc(sizeof(double) * (size_t)nvox);
        double* k = (double*)malloc(sizeof(double) * (size_t)(2 * r + 1));
        ora_psf_taps(P->psf_sigma, k);
        ora_deconv_theta(P, I, L, theta);
        ora_deconv_model(P, L, theta, R);
        for (int64_t i = 0; i < nvox; ++i)
            R[i] = I[i] - R[i];
#pragma omp parallel for schedule(dynamic, 256) num_threads(nthreads(P)) if (nthreads(P) > 1)
        for (int64_t q = 0; q < np; ++q) {
            int x, y, z;
            coords_of(P, lin[q], &x, &y, &z);
            double d_ext = deconv_move(P, R, k, r, lin[q], theta[b[q]] - theta[a[q]]);
            double d_int = (double)(face_count(P, L, x, y, z, a[q]) - face_count(P, L, x, y, z, b[q]));
            dE[q] = d_ext + P->lambda * d_int;
        }
        free(theta);
        free(R);
        free(k);
        return;
    }
    int M = P->max_labels;
    int64_t* n = (int64_t*)calloc((size_t)M, sizeof(int64_t));
    double* s1 = (double*)calloc((size_t)M, sizeof(double));
    double* s2 = (double*)calloc((size_t)M, sizeof(double));
    ora_region_stats(P, I, L, n, s1, s2);
    int zr = zrange(P);
    int R = P->ps_radius;

#pragma omp parallel for schedule(dynamic, 256) num_threads(nthreads(P)) if (nthreads(P) > 1)
    for (int64_t k = 0; k < np; ++k) {
        int x, y, z;
        coords_of(P, lin[k], &x, &y, &z);
        double v = I[lin[k]];
        int32_t la = a[k], lb = b[k];
        double d_ext;
        if (P->model == ORA_PC) {
            /* exact change of sum_x (I(x) - mu_{L(x)})^2 when v leaves region a
             * (n_a pixels) and joins region b (n_b pixels), means re-estimated */
            double mu_a = s1[la] / (double)n[la];
            double mu_b = s1[lb] / (double)n[lb];
            if (P->noise == ORA_POISSON) {
                d_ext = poisson_move(v, mu_a, mu_b);
            } else {
                double gain_b = (double)n[lb] / ((double)n[lb] + 1.0) * (v - mu_b) * (v - mu_b);
                double loss_a = 0.0;
                if (n[la] > 1)
                    loss_a = (double)n[la] / ((double)n[la] - 1.0) * (v - mu_a) * (v - mu_a);
                d_ext = gain_b - loss_a;
            }
        } else {
            /* local means over the closed ball |y - x|^2 <= R^2, per label */
            double sa = 0.0, sb = 0.0;
            int64_t ca = 0, cb = 0;
            int rz = zr ? R : 0;
            for (int dz = -rz; dz <= rz; ++dz)
                for (int dy = -R; dy <= R; ++dy)
                    for (int dx = -R; dx <= R; ++dx) {
                        if (dx * dx + dy * dy + dz * dz > R * R)
                            continue;
                        int xx = x + dx, yy = y + dy, zz = z + dz;
                        if (!in_bounds(P, xx, yy, zz))
                            continue;
                        int64_t j = lin_of(P, xx, yy, zz);
                        if (L[j] == la) {
                            sa += I[j];
                            ++ca;
                        } else if (L[j] == lb) {
                            sb += I[j];
                            ++cb;
                        }
                    }
            double m_a = sa / (double)ca;
            double m_b = sb / (double)cb;
            if (P->noise == ORA_POISSON)
                d_ext = poisson_move(v, m_a, m_b);
            else
                d_ext = (v - m_b) * (v - m_b) - (v - m_a) * (v - m_a);
        }
        /* contour length: unlike face pairs at x change by c_a - c_b */
        double d_int = (double)(face_count(P, L, x, y, z, la) - face_count(P, L, x, y, z, lb));
        dE[k] = d_ext + P->lambda * d_int;
    }
    free(n);
    free(s1);
    free(s2);
}

/* --- Eq. (6): sums over Q_p and Q'_p ------------------------------------ */

static void pair_sums(const ora_params* P, int64_t p, int64_t q, const int* X, const int* Y,
                      const int* Z, const int32_t* a, const int32_t* b, const double* dE,
                      double* s_same, int64_t* c_same, double* s_other, int64_t* c_other)
{
    double dx = X[q] - X[p], dy = Y[q] - Y[p], dz = Z[q] - Z[p];
    double d = sqrt(dx * dx + dy * dy + dz * dz);
    if (!(d < P->E / 2.0))
        return;
    double w = ora_kernel(d, P->E, P->eps);
    if (a[q] == a[p] && b[q] == b[p]) {
        *s_same += w * dE[q];
        ++*c_same;
    } else if (a[q] == b[p] && b[q] == a[p]) {
        *s_other += w * dE[q];
        ++*c_other;
    }
}

static double sobolev_value(double s_same, int64_t c_same, double s_other, int64_t c_other)
{
    double v = s_same / (double)c_same;  /* c_same >= 1: p is in Q_p */
    if (c_other > 0)
        v -= s_other / (double)c_other;
    return v;
}

void ora_sobolev(const ora_params* P, int64_t np, const int64_t* lin,
                 const int32_t* a, const int32_t* b, const double* dE_in,
                 double* out, int32_t neigh, int64_t nsel, const int64_t* sel)
{
    int* X = (int*)malloc(sizeof(int) * (size_t)(np > 0 ? np : 1));
    int* Y = (int*)malloc(sizeof(int) * (size_t)(np > 0 ? np : 1));
    int* Z = (int*)malloc(sizeof(int) * (size_t)(np > 0 ? np : 1));
    for (int64_t k = 0; k < np; ++k)
        coords_of(P, lin[k], &X[k], &Y[k], &Z[k]);
    int64_t nout = sel ? nsel : np;

    if (neigh == ORA_NEIGH_BRUTE) {
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads(P)) if (nthreads(P) > 1)
        for (int64_t k = 0; k < nout; ++k) {
            int64_t p = sel ? sel[k] : k;
            double s1 = 0.0, s2 = 0.0;
            int64_t c1 = 0, c2 = 0;
            for (int64_t q = 0; q < np; ++q)
                pair_sums(P, p, q, X, Y, Z, a, b, dE_in, &s1, &c1, &s2, &c2);
            out[k] = sobolev_value(s1, c1, s2, c2);
        }
    } else {
        /* cell lists with edge E/2, the interaction cutoff (text after Eq. (6)) */
        double h = P->E / 2.0;
        int ncx = (int)floor((P->nx - 1) / h) + 1;
        int ncy = (int)floor((P->ny - 1) / h) + 1;
        int ncz = (int)floor((P->nz - 1) / h) + 1;
        int64_t ncell = (int64_t)ncx * ncy * ncz;
        int64_t* start = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
        int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
        int64_t* cell = (int64_t*)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
        for (int64_t k = 0; k < np; ++k) {
            int cx = (int)floor(X[k] / h), cy = (int)floor(Y[k] / h), cz = (int)floor(Z[k] / h);
            cell[k] = cx + (int64_t)ncx * (cy + (int64_t)ncy * cz);
            start[cell[k] + 1] += 1;
        }
        for (int64_t c = 0; c < ncell; ++c)
            start[c + 1] += start[c];
        int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncell);
        memcpy(fill, start, sizeof(int64_t) * (size_t)ncell);
        for (int64_t k = 0; k < np; ++k)
            order[fill[cell[k]]++] = k;
        free(fill);

#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads(P)) if (nthreads(P) > 1)
        for (int64_t k = 0; k < nout; ++k) {
            int64_t p = sel ? sel[k] : k;
            int cx = (int)floor(X[p] / h), cy = (int)floor(Y[p] / h), cz = (int)floor(Z[p] / h);
            double s1 = 0.0, s2 = 0.0;
            int64_t c1 = 0, c2 = 0;
            for (int jz = cz - 1; jz <= cz + 1; ++jz)
                for (int jy = cy - 1; jy <= cy + 1; ++jy)
                    for (int jx = cx - 1; jx <= cx + 1; ++jx) {
                        if (jx < 0 || jy < 0 || jz < 0 || jx >= ncx || jy >= ncy || jz >= ncz)
                            continue;
                        int64_t c = jx + (int64_t)ncx * (jy + (int64_t)ncy * jz);
                        for (int64_t t = start[c]; t < start[c + 1]; ++t)
                            pair_sums(P, p, order[t], X, Y, Z, a, b, dE_in, &s1, &c1, &s2, &c2);
                    }
            out[k] = sobolev_value(s1, c1, s2, c2);
        }
        free(start);
        free(order);
        free(cell);
    }
    free(X);
    free(Y);
    free(Z);
}

/* --- topological control ------------------------------------------------- */

/* Membership of the 3x3(x3) neighbourhood of pixel i in {L == l}; index
 * (dx+1) + 3(dy+1) + 9(dz+1), centre left out (0).  Outside the image: 0. */
static void neighbourhood(const ora_params* P, const int32_t* L, int64_t i, int32_t l, int in[27])
{
    int x, y, z;
    coords_of(P, i, &x, &y, &z);
    int dz0 = P->ndim == 3 ? -1 : 0, dz1 = P->ndim == 3 ? 1 : 0;
    for (int k = 0; k < 27; ++k)
        in[k] = 0;
    for (int dz = dz0; dz <= dz1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0 && dz == 0)
                    continue;
                int k = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
                in[k] = in_bounds(P, x + dx, y + dy, z + dz) && L[lin_of(P, x + dx, y + dy, z + dz)] == l;
            }
}

/* Number of connected components among the cells k with sel[k] set, where
 * two cells are adjacent when their offsets differ by at most 1 in every
 * axis (full = 1) or by 1 in exactly one axis (full = 0).  Only components
 * holding a cell with need[k] set are counted (need = NULL: all). */
static int components(const int sel[27], int full, const int* need)
{
    int comp[27], stack[27], count = 0;
    for (int k = 0; k < 27; ++k)
        comp[k] = -1;
    for (int s0 = 0; s0 < 27; ++s0) {
        if (!sel[s0] || comp[s0] >= 0)
            continue;
        int top = 0, hit = 0;
        stack[top++] = s0;
        comp[s0] = s0;
        while (top > 0) {
            int k = stack[--top];
            if (!need || need[k])
                hit = 1;
            int kx = k % 3, ky = (k / 3) % 3, kz = k / 9;
            for (int j = 0; j < 27; ++j) {
                if (!sel[j] || comp[j] >= 0)
                    continue;
                int ax = abs(j % 3 - kx), ay = abs((j / 3) % 3 - ky), az = abs(j / 9 - kz);
                int adj = full ? (ax <= 1 && ay <= 1 && az <= 1) : (ax + ay + az == 1);
                if (adj) {
                    comp[j] = s0;
                    stack[top++] = j;
                }
            }
        }
        count += hit;
    }
    return count;
}

int32_t ora_simple(const ora_params* P, const int32_t* L, int64_t i, int32_t l)
{
    int in[27], fg[27], bg[27], face[27];
    neighbourhood(P, L, i, l, in);
    const int three = P->ndim == 3;
    for (int k = 0; k < 27; ++k) {
        int ax = abs(k % 3 - 1), ay = abs((k / 3) % 3 - 1), az = abs(k / 9 - 1);
        int cells = ax + ay + az;       /* 0 centre, 1 face, 2 edge, 3 corner */
        int present = three || az == 0; /* 2D: the middle plane only */
        fg[k] = present && cells > 0 && in[k];
        /* complement: 18-neighbourhood in 3D (no corners), 8 in 2D */
        bg[k] = present && cells > 0 && (three ? cells < 3 : 1) && !in[k];
        face[k] = cells == 1;
    }
    int t_fg = components(fg, 1, NULL);
    int t_bg = components(bg, 0, face);
    return t_fg == 1 && t_bg == 1;
}

typedef struct {
    double g;
    int64_t i;
    int32_t b;
    int64_t k; /* particle index */
} ora_cand;

static int cand_cmp(const void* u, const void* v)
{
    const ora_cand* p = (const ora_cand*)u;
    const ora_cand* q = (const ora_cand*)v;
    if (p->g != q->g)
        return p->g < q->g ? -1 : 1;
    if (p->i != q->i)
        return p->i < q->i ? -1 : 1;
    return (p->b > q->b) - (p->b < q->b);
}

int64_t ora_accept_ranked(const ora_params* P, int32_t* L, int64_t np, const int64_t* lin,
                          const int32_t* a, const int32_t* b, const double* g, int32_t topo,
                          uint8_t* done)
{
    ora_cand* c = (ora_cand*)malloc(sizeof(ora_cand) * (size_t)(np > 0 ? np : 1));
    int64_t nc = 0;
    for (int64_t k = 0; k < np; ++k) {
        if (done)
            done[k] = 0;
        if (g[k] < 0.0) {
            c[nc].g = g[k];
            c[nc].i = lin[k];
            c[nc].b = b[k];
            c[nc].k = k;
            ++nc;
        }
    }
    qsort(c, (size_t)nc, sizeof(ora_cand), cand_cmp);
    int64_t moves = 0;
    for (int64_t r = 0; r < nc; ++r) {
        int64_t k = c[r].k, i = lin[k];
        if (L[i] != a[k])
            continue; /* the pixel already moved */
        if (topo == ORA_TOPO_SIMPLE) {
            if (a[k] >= 1 && !ora_simple(P, L, i, a[k]))
                continue;
            if (b[k] >= 1 && !ora_simple(P, L, i, b[k]))
                continue;
        }
        L[i] = b[k];
        if (done)
            done[k] = 1;
        ++moves;
    }
    free(c);
    return moves;
}

/* --- one Region Competition iteration ------------------------------------ */

int64_t ora_step(const ora_params* P, const double* I, int32_t* L, int32_t mode,
                 int64_t cap, int64_t* lin_o, int32_t* a_o, int32_t* b_o,
                 double* dE_l2_o, double* dE_h1_o, int64_t* nflips)
{
    int64_t np = ora_particles(P, L, 0, NULL, NULL, NULL);
    int64_t* lin = (int64_t*)malloc(sizeof(int64_t) * (size_t)(np > 0 ? np : 1));
    int32_t* a = (int32_t*)malloc(sizeof(int32_t) * (size_t)(np > 0 ? np : 1));
    int32_t* b = (int32_t*)malloc(sizeof(int32_t) * (size_t)(np > 0 ? np : 1));
    double* g2 = (double*)malloc(sizeof(double) * (size_t)(np > 0 ? np : 1));
    double* g1 = (double*)malloc(sizeof(double) * (size_t)(np > 0 ? np : 1));
    ora_particles(P, L, np, lin, a, b);
    ora_l2diff(P, I, L, np, lin, a, b, g2);
    if (mode == ORA_MODE_SOBOLEV)
        ora_sobolev(P, np, lin, a, b, g2, g1, ORA_NEIGH_CELLS, 0, NULL);
    else
        memcpy(g1, g2, sizeof(double) * (size_t)np);

    int64_t flips = 0;
    int64_t nvox = (int64_t)P->nx * P->ny * P->nz;
    if (P->topo == ORA_TOPO_SIMPLE) {
        flips = ora_accept_ranked(P, L, np, lin, a, b, g1, ORA_TOPO_SIMPLE, NULL);
        goto out;
    }
    /* moves are decided from L_t only, then applied together */
    int32_t* Lnew = (int32_t*)malloc(sizeof(int32_t) * (size_t)nvox);
    memcpy(Lnew, L, sizeof(int32_t) * (size_t)nvox);
    for (int64_t k = 0; k < np;) {
        int64_t e = k;
        int64_t best = -1;
        while (e < np && lin[e] == lin[k]) {
            if (g1[e] < 0.0 && (best < 0 || g1[e] < g1[best]))
                best = e;
            ++e;
        }
        if (best >= 0) {
            Lnew[lin[best]] = b[best];
            ++flips;
        }
        k = e;
    }
    memcpy(L, Lnew, sizeof(int32_t) * (size_t)nvox);
    free(Lnew);

out:;
    int64_t ret = np;
    if (lin_o || a_o || b_o || dE_l2_o || dE_h1_o) {
        if (np > cap) {
            ret = -1;
        } else {
            if (lin_o) memcpy(lin_o, lin, sizeof(int64_t) * (size_t)np);
            if (a_o) memcpy(a_o, a, sizeof(int32_t) * (size_t)np);
            if (b_o) memcpy(b_o, b, sizeof(int32_t) * (size_t)np);
            if (dE_l2_o) memcpy(dE_l2_o, g2, sizeof(double) * (size_t)np);
            if (dE_h1_o) memcpy(dE_h1_o, g1, sizeof(double) * (size_t)np);
        }
    }
    if (nflips)
        *nflips = flips;
    free(lin);
    free(a);
    free(b);
    free(g2);
    free(g1);
    return ret;
}

int64_t ora_reversals(int64_t nvox, const int32_t* L_prev, const int32_t* L_next,
                      uint32_t* stamp, int64_t t)
{
    int64_t back = 0;
    for (int64_t x = 0; x < nvox; ++x) {
        if (L_prev[x] == L_next[x])
            continue;
        if (stamp[x] != 0 && stamp[x] == (uint32_t)t) /* changed in iteration t - 1 */
            ++back;
        stamp[x] = (uint32_t)(t + 1);
    }
    return back;
}

void ora_auto_init(ora_auto* s, int32_t mode)
{
    s->t = 0;
    s->grad = mode == ORA_MODE_L2 ? ORA_MODE_L2 : ORA_MODE_SOBOLEV;
    s->osc_prev = 0;
    s->cycle_prev = 0;
    s->switch_iter = -1;
}

int32_t ora_auto_update(ora_auto* s, int32_t mode, double tol, int64_t n, int64_t flips,
                        int64_t reversals)
{
    const int32_t t = s->t;
    const int osc = flips > 0 && 2 * reversals >= flips;
    const int cycle = flips > 0 && reversals == flips; /* every flip undoes the previous iteration's */
    /* iterations t - 1 and t both ran with L2 gradients after the switch */
    const int l2_both = s->switch_iter >= 0 && t - 1 >= s->switch_iter;
    const int stop_cycle = mode == ORA_MODE_AUTO && tol > 0.0 && l2_both && cycle && s->cycle_prev;
    if (mode == ORA_MODE_AUTO && s->grad == ORA_MODE_SOBOLEV && osc && s->osc_prev) {
        s->grad = ORA_MODE_L2;
        s->switch_iter = t + 1;
    }
    s->osc_prev = osc;
    s->cycle_prev = cycle;
    s->t = t + 1;
    return (double)flips < tol * (double)n || stop_cycle;
}

int32_t ora_run(const ora_params* P, const double* I, int32_t* L, int32_t mode,
                int32_t max_iters, double tol, int64_t* hist_n, int64_t* hist_f,
                int64_t* hist_b, int32_t* switch_iter)
{
    int64_t nvox = (int64_t)P->nx * P->ny * P->nz;
    int32_t* prev = (int32_t*)malloc(sizeof(int32_t) * (size_t)nvox);
    uint32_t* stamp = (uint32_t*)calloc((size_t)nvox, sizeof(uint32_t));
    ora_auto st;
    ora_auto_init(&st, mode);
    while (st.t < max_iters) {
        const int32_t t = st.t;
        int64_t flips = 0;
        memcpy(prev, L, sizeof(int32_t) * (size_t)nvox);
        int64_t np = ora_step(P, I, L, st.grad, 0, NULL, NULL, NULL, NULL, NULL, &flips);
        int64_t back = ora_reversals(nvox, prev, L, stamp, t);
        if (hist_n) hist_n[t] = np;
        if (hist_f) hist_f[t] = flips;
        if (hist_b) hist_b[t] = back;
        if (ora_auto_update(&st, mode, tol, np, flips, back))
            break;
    }
    if (switch_iter)
        *switch_iter = st.switch_iter;
    free(prev);
    free(stamp);
    return st.t;
}

double ora_energy_pc(const ora_params* P, const double* I, const int32_t* L)
{
    int M = P->max_labels;
    int64_t* n = (int64_t*)calloc((size_t)M, sizeof(int64_t));
    double* s1 = (double*)calloc((size_t)M, sizeof(double));
    double* s2 = (double*)calloc((size_t)M, sizeof(double));
    ora_region_stats(P, I, L, n, s1, s2);
    double e = 0.0;
    int64_t nvox = (int64_t)P->nx * P->ny * P->nz;
    for (int64_t i = 0; i < nvox; ++i) {
        double mu = s1[L[i]] / (double)n[L[i]];
        e += (I[i] - mu) * (I[i] - mu);
    }
    int64_t unlike = 0;
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                int32_t l = L[lin_of(P, x, y, z)];
                if (x + 1 < P->nx && L[lin_of(P, x + 1, y, z)] != l) ++unlike;
                if (y + 1 < P->ny && L[lin_of(P, x, y + 1, z)] != l) ++unlike;
                if (z + 1 < P->nz && L[lin_of(P, x, y, z + 1)] != l) ++unlike;
            }
    free(n);
    free(s1);
    free(s2);
    return e + P->lambda * (double)unlike;
}

/* Eq. (4) evaluated with true geodesic (arc-length) distances on a closed
 * curve: a midpoint-rule quadrature over n equispaced samples. */
void ora_conv_closed_curve(int64_t n, double Lc, double E, double eps,
                           const double* g, double* out)
{
    double ds = Lc / (double)n;
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            int64_t d = i > j ? i - j : j - i;
            if (n - d < d)
                d = n - d;
            acc += ora_kernel((double)d * ds, E, eps) * g[j] * ds;
        }
        out[i] = acc;
    }
}
