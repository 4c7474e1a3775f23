/* sobrc_oracle.h -- FP64 CPU oracle for particle-based Region Competition with
 * particle-approximated Sobolev gradients (Sbalzarini, Schneider, Cardinale,
 * arXiv:1403.0240).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP implementation; the two agree only
 * because both follow the paper.
 *
 * Layout: images and label fields are [nz][ny][nx], x fastest; 2D means nz = 1.
 * Linear index i = x + nx*(y + ny*z).  Labels: 0 = background, 1..M-1 foreground.
 */
#ifndef SOBRC_ORACLE_H
#define SOBRC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_PC = 0, ORA_PS = 1 };
/* AUTO: Sobolev gradients until oscillation is detected, L2-type gradients
 * from the next iteration on (Section "Particle approximation", the remark
 * after Eq. (6), and the Fig. 3 experiment); see ora_reversals. */
enum { ORA_MODE_SOBOLEV = 0, ORA_MODE_L2 = 1, ORA_MODE_AUTO = 2 };
enum { ORA_NEIGH_BRUTE = 0, ORA_NEIGH_CELLS = 1 };

typedef struct {
    int32_t ndim, nx, ny, nz;  /* nz = 1 when ndim = 2 */
    int32_t model;             /* ORA_PC or ORA_PS */
    int32_t ps_radius;         /* PS local-mean ball: |y-x|^2 <= R^2 */
    double E, eps, lambda;     /* Sobolev length scale, smoothness, prior weight */
    int32_t max_labels;
    int32_t threads;           /* OpenMP threads for per-particle loops (<=1: serial) */
    int32_t noise;             /* ORA_GAUSS or ORA_POISSON pixel noise */
    int32_t topo;              /* ORA_TOPO_OFF or ORA_TOPO_SIMPLE acceptance */
    double psf_sigma;          /* > 0: deconvolving model with a Gaussian PSF (PC, Gaussian noise) */
} ora_params;

/* Deconvolving image model (Methods, Eq. (8): J = s_theta(Gamma) * K).  K is
 * a separable Gaussian point-spread function: per axis the taps
 * exp(-t^2 / (2 sigma^2)) for |t| <= ceil(3 sigma), normalised to sum 1, and
 * K(d) their product over the axes; s is zero outside the image.  The region
 * intensities theta (photometric estimate) minimise sum_y (I(y) - J(y))^2
 * over the image for the current labels (least squares; a label with no
 * pixel gets theta 0).  A move of pixel x from a to b changes s(x) by
 * delta = theta_b - theta_a with theta held fixed, so its data term is
 * sum_y [(I(y) - J(y) - delta K(y - x))^2 - (I(y) - J(y))^2] over the image. */
int32_t ora_psf_radius(double sigma);
void ora_psf_taps(double sigma, double* taps); /* 2 ora_psf_radius(sigma) + 1 taps */
void ora_deconv_theta(const ora_params* P, const double* I, const int32_t* L, double* theta);
void ora_deconv_model(const ora_params* P, const int32_t* L, const double* theta, double* J);

/* Acceptance of the moves.  OFF: simultaneous, per pixel the smallest
 * gradient.  SIMPLE: the moves are ranked by gradient (most negative first)
 * and executed one after the other; a move runs only if its pixel still has
 * the label it started from and is a simple point of the region it leaves and
 * of the region it joins (labels >= 1; the background label 0 is not
 * controlled), so no foreground region splits, merges, vanishes, or gains or
 * loses a hole or tunnel (the topological control of Region Competition,
 * Introduction, "The Region Competition (RC) algorithm"). */
enum { ORA_TOPO_OFF = 0, ORA_TOPO_SIMPLE = 1 };

/* Pixel noise of the likelihood (Methods, Eq. (11) with independent noise):
 * Gaussian -- energy (I - J)^2 per pixel; Poisson -- energy J - I log J (the
 * negative log-likelihood without the constant log I!). */
enum { ORA_GAUSS = 0, ORA_POISSON = 1 };
#define ORA_POISSON_MIN_MEAN 1e-6 /* expected intensities below are raised to it */

/* Sobolev kernel of Eq. (5); zero outside its support |r| <= E/2. */
double ora_kernel(double r, double E, double eps);

/* Contour particle set (Fig. 1 and the particle-representation section): one
 * particle (i, a = L(i), b) per pixel i and per distinct label b != a found in
 * its full neighbourhood (8 in 2D, 26 in 3D).  Canonical order: i, then b.
 * Writes at most cap entries; returns the total count. */
int64_t ora_particles(const ora_params* P, const int32_t* L, int64_t cap,
                      int64_t* lin, int32_t* a, int32_t* b);

/* Region statistics over the label field: n_l, sum I, sum I^2. */
void ora_region_stats(const ora_params* P, const double* I, const int32_t* L,
                      int64_t* n, double* s1, double* s2);

/* L2-type gradient: per-particle energy difference of the single move
 * a -> b (Eqs. (10)-(11)), piecewise-constant or piecewise-smooth model (or
 * the deconvolving model when P->psf_sigma > 0) plus lambda times the change
 * in contour length. */
void ora_l2diff(const ora_params* P, const double* I, const int32_t* L,
                int64_t np, const int64_t* lin, const int32_t* a, const int32_t* b,
                double* dE);

/* Discrete Sobolev update, Eq. (6).  If sel != NULL only the nsel particles
 * listed there are evaluated and out[k] belongs to particle sel[k]; otherwise
 * out has np entries.  neigh selects brute force or cell lists. */
void ora_sobolev(const ora_params* P, int64_t np, const int64_t* lin,
                 const int32_t* a, const int32_t* b, const double* dE_in,
                 double* out, int32_t neigh, int64_t nsel, const int64_t* sel);

/* One Region Competition iteration on L (in place): particles, stats, L2
 * gradient, Sobolev smoothing (mode), acceptance (simultaneous, or ranked
 * with topological control when P->topo is ORA_TOPO_SIMPLE).  Optional
 * outputs (may be NULL, each needs cap entries): particle list and both
 * gradients.  Returns the particle count N_t (or -1 if N_t > cap while an
 * output array was requested); *nflips receives the number of changed pixels. */
int64_t ora_step(const ora_params* P, const double* I, int32_t* L, int32_t mode,
                 int64_t cap, int64_t* lin, int32_t* a, int32_t* b,
                 double* dE_l2, double* dE_h1, int64_t* nflips);

/* Digital topology (26/6 connectivity in 3D, 8/4 in 2D; pixels outside the
 * image belong to no region).  Returns 1 if pixel i is a simple point of the
 * set X = {L == l}: adding i to X (or removing it) leaves X's topology
 * unchanged.  The label of i itself is ignored.  Test: the number of
 * 26-components (8 in 2D) of X in the 26-neighbourhood of i is 1, and the
 * number of 6-components (4 in 2D) of the complement within the
 * 18-neighbourhood (8 in 2D) that touch a face neighbour of i is 1. */
int32_t ora_simple(const ora_params* P, const int32_t* L, int64_t i, int32_t l);

/* Ranked acceptance (Introduction, "The Region Competition (RC) algorithm":
 * particles are ranked by energy difference before any move is executed, so
 * the result does not depend on particle order; topological control keeps
 * contours intact).  Candidates are the particles with g < 0, executed in
 * order of (g, i, b) ascending on L in place; with topo = ORA_TOPO_SIMPLE a
 * move of pixel i from a to b runs only if i still has label a, is simple
 * for a (if a >= 1) and simple for b (if b >= 1).  Without topology control
 * only the label check applies, which gives the simultaneous per-pixel rule.
 * done (may be NULL, np entries) receives 1 for executed moves.  Returns the
 * number of executed moves. */
int64_t ora_accept_ranked(const ora_params* P, int32_t* L, int64_t np, const int64_t* lin,
                          const int32_t* a, const int32_t* b, const double* g, int32_t topo,
                          uint8_t* done);

/* Oscillation test of one iteration.  A reversal is a pixel that changes
 * label in iteration t (L_prev -> L_next differ) and also changed in
 * iteration t - 1; stamp[x] holds 1 + the last iteration in which pixel x
 * changed (0: never) and is updated here.  Returns the number of reversals.
 * Reading (the paper only says oscillations are easily detected): the
 * contour oscillates when at least half of an iteration's flips are
 * reversals, in two iterations in a row (ora_run). */
int64_t ora_reversals(int64_t nvox, const int32_t* L_prev, const int32_t* L_next,
                      uint32_t* stamp, int64_t t);

/* The AUTO gradient-mode rule, one iteration at a time (reading: the paper
 * only says that the oscillation near an energy extremum is easily detected
 * and that the optimizer then returns to L2-type gradients).  An iteration
 * oscillates when flips > 0 and 2 * reversals >= flips; it cycles when
 * flips > 0 and reversals == flips.  In ORA_MODE_AUTO, the first iteration t
 * that oscillates right after an oscillating iteration t - 1 makes every
 * later iteration use L2-type gradients (switch_iter = t + 1).  A run stops
 * after iteration t when flips < tol * N_t, or (AUTO, tol > 0) when t - 1 and
 * t both ran with L2 gradients and both cycled.
 * ora_auto_init starts a run; ora_auto_update takes iteration s->t's
 * particle count, flips and reversals, advances s->t and returns 1 when the
 * run stops after that iteration.  s->grad is the gradient mode
 * (ORA_MODE_SOBOLEV or ORA_MODE_L2) of the next iteration. */
typedef struct {
    int32_t t;           /* iterations done */
    int32_t grad;        /* gradient of iteration t */
    int32_t osc_prev;    /* iteration t - 1 oscillated */
    int32_t cycle_prev;  /* iteration t - 1 cycled */
    int32_t switch_iter; /* first iteration with L2 gradients in AUTO mode, -1: none */
} ora_auto;
void ora_auto_init(ora_auto* s, int32_t mode);
int32_t ora_auto_update(ora_auto* s, int32_t mode, double tol, int64_t n, int64_t flips,
                        int64_t reversals);

/* Repeat ora_step until max_iters or nflips < tol * N_t.  Per-iteration N_t,
 * flips and reversals go to hist_n / hist_f / hist_b (max_iters entries
 * each, may be NULL).  An iteration oscillates when flips > 0 and
 * 2 * reversals >= flips.  In ORA_MODE_AUTO the first iteration t that
 * oscillates right after an oscillating iteration t - 1 switches every later
 * iteration to L2-type gradients; *switch_iter receives t + 1 (or -1: no
 * switch; may be NULL).  The switch and the stops follow ora_auto_update.
 * Returns iterations done. */
int32_t ora_run(const ora_params* P, const double* I, int32_t* L, int32_t mode,
                int32_t max_iters, double tol, int64_t* hist_n, int64_t* hist_f,
                int64_t* hist_b, int32_t* switch_iter);

/* Total piecewise-constant energy: sum_x (I(x) - mu_{L(x)})^2 with region means
 * mu_l, plus lambda times the number of face-adjacent pixel pairs with
 * different labels (discrete contour length). */
double ora_energy_pc(const ora_params* P, const double* I, const int32_t* L);

/* Continuous form of Eq. (4) on a closed curve of arc length Lc sampled at n
 * equispaced points: out_i = sum_j K(geodesic(s_i, s_j)) g_j (Lc/n). */
void ora_conv_closed_curve(int64_t n, double Lc, double E, double eps,
                           const double* g, double* out);

#ifdef __cplusplus
}
#endif
#endif
