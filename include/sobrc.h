/* sobrc.h -- C ABI of the MI355X (gfx950) implementation of the per-iteration
 * hot path of particle-based Region Competition with particle-approximated
 * Sobolev gradients (Sbalzarini, Schneider, Cardinale, arXiv:1403.0240).
 *
 * One iteration on the contour particles:
 *   compute_l2_diff : L2-type gradient of every particle, i.e. the energy change
 *                     of its single move (Eqs. (10)-(11), region models from the
 *                     Methods section);
 *   sobolev_smooth  : the discrete Sobolev update of Eq. (6), kernel of Eq. (5),
 *                     neighbours found with cell lists (text after Eq. (6));
 *   step / run      : acceptance of moves, label update and contour-particle
 *                     bookkeeping, repeated until a flip-rate tolerance.
 *
 * Conventions shared by every entry point
 *  - Every function is extern "C", returns an int32 status (SOBRC_OK = 0 or a
 *    negative SOBRC_E* code) and never throws.  last_error() returns a
 *    thread-local message describing the last failure of this thread.
 *  - "d_" pointers are device (HIP) pointers, "h_" pointers host pointers.
 *    All device memory is owned by the caller; the library never allocates
 *    device memory.  A context lives in a caller-provided device workspace of
 *    workspace_size() bytes and borrows the image until ctx_destroy.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are asynchronous on that stream unless stated otherwise.  One
 *    context must not be used from two streams at once.
 *  - Grids: images and label fields are [nz][ny][nx], x fastest, nz = 1 for 2D;
 *    pixel centres sit at integer coordinates; linear index i = x + nx*(y + ny*z).
 *    Labels are in [0, max_labels); 0 is the single background region (an open
 *    set), 1.. are foreground regions (closed sets), as in the Methods.
 *  - Contour particles: one particle (i, a = L(i), b) for every pixel i and
 *    every distinct label b != a among its in-bounds full neighbours (8 in 2D,
 *    26 in 3D), i.e. particles on both sides of the contour (Fig. 1).  The
 *    library's particle order is tile-major (tiles of 16x16 pixels in 2D,
 *    8x8x8 voxels in 3D, tiles in x-fastest order), then the pixel's position
 *    inside the tile (x fastest), then b ascending.  All per-particle arrays of
 *    a context use that order.
 */
#ifndef SOBRC_H
#define SOBRC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SOBRC_OK = 0,
    SOBRC_EINVAL = -1,     /* bad parameter, null pointer, label out of range */
    SOBRC_ECAPACITY = -2,  /* particle count would exceed max_particles */
    SOBRC_EDEVICE = -3,    /* HIP runtime error, or a ranked acceptance that did not finish
                              within its pass limit (message kept in last_error) */
    SOBRC_ESTATE = -4      /* call order (e.g. step before init_labels) */
};
enum { SOBRC_F32 = 0, SOBRC_U16 = 1 };            /* image element type */
enum { SOBRC_PC = 0, SOBRC_PS = 1 };              /* piecewise constant / smooth */
/* Pixel noise of the likelihood (Methods, Eq. (11), noise independent per
 * pixel).  GAUSS: energy (I - J)^2 per pixel, the PC move re-estimates both
 * region means exactly.  POISSON: energy J - I log J (negative log-likelihood
 * without log I!), a move evaluated with both expected intensities J held at
 * their current values (region means for PC, local means for PS), J raised
 * to at least 1e-6; intended for photon-count images (I >= 0). */
enum { SOBRC_NOISE_GAUSS = 0, SOBRC_NOISE_POISSON = 1 };
/* Gradient mode of step/run.  AUTO: Sobolev gradients until the contour
 * oscillates, L2-type gradients from then on (the paper's remark after
 * Eq. (6) and its Fig. 3 experiment; the detection rule is this library's,
 * see get_gradient_mode). */
enum { SOBRC_MODE_SOBOLEV = 0, SOBRC_MODE_L2 = 1, SOBRC_MODE_AUTO = 2 };
/* Acceptance of the moves (Introduction, "The Region Competition (RC)
 * algorithm": moves are ranked by energy difference before they are executed,
 * so the result does not depend on particle order, and topological control
 * keeps contours intact).  OFF: every particle with gradient < 0 is a
 * candidate, per pixel the smallest gradient wins (ties: smaller b), all
 * chosen moves are applied together.  SIMPLE: the candidates run one after
 * the other in order of (gradient, pixel linear index, b); a move runs only
 * if its pixel still has the label it started from and is a simple point
 * (26/6 connectivity in 3D, 8/4 in 2D; pixels outside the image belong to no
 * region) of the region it leaves and of the region it joins, for labels >= 1
 * (the background label 0 is not controlled).  No foreground region then
 * splits, merges with another piece of itself, vanishes, or gains or loses a
 * hole or tunnel.  The device reproduces the sequential order exactly.
 * Contexts with SIMPLE take 8 bytes per pixel and 1 per particle more
 * workspace and are not batched. */
enum { SOBRC_TOPO_OFF = 0, SOBRC_TOPO_SIMPLE = 1 };
/* Cell lists ("Discrete particle approximation", text after Eq. (6):
 * particles binned in cells so that the Eq. (6) sums visit only neighbouring
 * cells; the paper's cells have edge E/2).  Here a cell is a tile of the
 * image, and the results do not depend on its shape (every sum tests the
 * integer distance), only the speed: DEFAULT = 8x8x8 voxels in 3D, 16x16
 * pixels in 2D; WIDE = twice as long along one axis (16x8x8 in 3D, 16x32 in
 * 2D); TALL (2D only) = 16x64 pixels.  Longer tiles are fewer and fuller, with
 * less halo per particle.  tile_autotune times the shapes on a given image.
 * Only DEFAULT is available with topological control. */
enum { SOBRC_TILE_DEFAULT = 0, SOBRC_TILE_WIDE = 1, SOBRC_TILE_TALL = 2 };
/* Deconvolving image model (Methods, Eq. (8): J = s_theta(Gamma) * K), used
 * when params.psf_sigma > 0.  K is a separable Gaussian point-spread function:
 * per axis the taps exp(-t^2 / (2 sigma^2)) for |t| <= ceil(3 sigma),
 * normalised to sum 1; s is zero outside the image.  At the start of every
 * gradient evaluation the region intensities theta are the least-squares fit
 * of sum_l theta_l (K * chi_l) to the image (labels without pixels get 0);
 * a move of pixel x from a to b then has the data term
 * sum_y [(I - J - delta K(y - x))^2 - (I - J)^2] over the image, delta =
 * theta_b - theta_a, theta held fixed.  Needs SOBRC_PC, SOBRC_NOISE_GAUSS and
 * max_labels <= 4; takes (max_labels + 4) x 4 bytes per pixel more workspace;
 * not batched. */

typedef struct {
    int32_t ndim;          /* 2 or 3 */
    int32_t nx, ny, nz;    /* 3D: each in [1, 1024]; 2D: nx, ny in [1, 32768], nz = 1 */
    int32_t image_dtype;   /* SOBRC_F32 or SOBRC_U16 */
    int32_t model;         /* SOBRC_PC or SOBRC_PS */
    int32_t ps_radius;     /* PS local-mean ball |y-x|^2 <= R^2, R in [2, 32]; ignored for PC */
    double E;              /* Sobolev length scale, 0 < E <= 64; interaction radius E/2 */
    double eps;            /* smoothness hyper-parameter of Eq. (1), > 0 (paper: 1/24) */
    double lambda;         /* prior weight of Eq. (10), >= 0 */
    int32_t max_labels;    /* labels lie in [0, max_labels), 2 <= max_labels <= 65535 */
    int64_t max_particles; /* particle capacity, 1 <= max_particles < 2^31 */
    int32_t noise;         /* SOBRC_NOISE_GAUSS or SOBRC_NOISE_POISSON */
    int32_t topo;          /* SOBRC_TOPO_OFF or SOBRC_TOPO_SIMPLE (acceptance, see below) */
    double psf_sigma;      /* 0, or the width (pixels, <= 16) of a Gaussian PSF: deconvolving model */
    int32_t tile;          /* SOBRC_TILE_*: shape of the cells (see below) */
} sobrc_params;

typedef struct sobrc_ctx sobrc_ctx;

/* Bytes of device workspace a context with these parameters needs: the
 * label field, two particle-record buffers of max_particles entries (the
 * contour particles of Fig. 1 at iterations t and t + 1), both gradients,
 * the per-tile cell lists (text after Eq. (6)), the region statistics of the
 * photometric estimate (Methods) and the model's extra fields.  Host only,
 * no device call.  EINVAL on bad parameters. */
int32_t workspace_size(const sobrc_params* params, size_t* bytes);

/* Create a context -- one segmentation job of the energy of Eq. (10) on one
 * image -- inside a caller-owned device workspace (d_workspace, 256-byte
 * aligned, at least workspace_size bytes).  Host only: no device call is made
 * until init_labels.  *out receives a library-owned host handle. */
int32_t ctx_create(const sobrc_params* params, void* d_workspace, size_t bytes,
                   sobrc_ctx** out);

/* Release the host handle (the workspace stays the caller's).  Synchronises
 * with nothing; the caller must not destroy a context with work in flight. */
int32_t ctx_destroy(sobrc_ctx* ctx);

/* Start a segmentation job: copy the initial label field (int32, nvox entries)
 * into the workspace, compute region statistics (photometric estimate: region
 * mean intensities, Methods) and build the contour particle set.  The context
 * borrows d_image (nvox elements of image_dtype) until ctx_destroy.
 * Synchronises `stream` once.  EINVAL if a label is outside [0, max_labels),
 * ECAPACITY if the particle set exceeds max_particles (the context then stays
 * uninitialised).  Resuming from a checkpoint is init_labels with saved labels. */
int32_t init_labels(sobrc_ctx* ctx, const void* d_image, const int32_t* d_labels,
                    void* stream);

/* L2-type gradient (energy difference of each particle's single move a -> b,
 * Eq. (11) with E_ext + lambda E_int of Eq. (10)): piecewise-constant data
 * term with re-estimated region means, or piecewise-smooth local means over
 * the PS ball; plus lambda times the change of the number of face-adjacent
 * pixel pairs with different labels (contour-length prior).  Writes fp32
 * values for the current particles, in context order, to d_dE_l2 (room for
 * max_particles entries).  Asynchronous. */
int32_t compute_l2_diff(sobrc_ctx* ctx, float* d_dE_l2, void* stream);

/* Discrete Sobolev update of Eq. (6) on the current particles: for particle p,
 *   out_p = (1/|Q_p|) sum_{q in Q_p} K(d_pq) in_q - (1/|Q'_p|) sum_{q in Q'_p} K(d_pq) in_q
 * with Q_p the particles of the same label pair (a, b) (p included), Q'_p those
 * of the swapped pair (b, a), both within Euclidean distance d_pq < E/2, K the
 * kernel of Eq. (5), and the second term 0 when Q'_p is empty.  Reads
 * d_dE_l2, writes d_dE_h1 (distinct buffers, context order, fp32 with fp32
 * accumulation).  Asynchronous. */
int32_t sobolev_smooth(sobrc_ctx* ctx, const float* d_dE_l2, float* d_dE_h1, void* stream);

/* One iteration of the Region Competition optimizer with particle-approximated
 * Sobolev gradients (Introduction, "The Region Competition (RC) algorithm",
 * and the text after Eq. (6)): L2 gradient, Sobolev update (mode SOBOLEV;
 * mode AUTO until it has switched) or none (mode L2), acceptance of the
 * moves with negative gradient as params.topo says (see SOBRC_TOPO_*), then
 * region statistics and the particle set are brought up to date.
 * If d_nflips != NULL the number of changed pixels is written there (device
 * int32).  Asynchronous, no host synchronisation.  If the new particle set
 * would exceed max_particles the step is rolled back on the device and the
 * context reports ECAPACITY from its next synchronising call (ctx_sync, run,
 * get_particles); further steps do nothing until a new init_labels.  The
 * roll-back restores the labels, the particle set and the region statistics;
 * compute_l2_diff and sobolev_smooth do not run on the restored state: they
 * write NaN for every particle until init_labels, and return ECAPACITY once a
 * synchronising call has reported the overflow. */
int32_t step(sobrc_ctx* ctx, int32_t mode, int32_t* d_nflips, void* stream);

/* One iteration with a caller-supplied gradient instead of the computed one:
 * d_grad (fp32, device, one value per current particle in context order, as
 * get_particles lists them) drives the acceptance (params.topo), then region
 * statistics and the particle set are brought up to date as in step().  For
 * gradients from another source (e.g. another energy) and for checking the
 * acceptance on its own.  d_grad is read during the call's kernels only.
 * Asynchronous; errors as step(). */
int32_t step_with_gradient(sobrc_ctx* ctx, const float* d_grad, int32_t* d_nflips, void* stream);

/* Up to max_iters iterations of step(), the optimizer run to convergence
 * (the paper counts iterations until the contour stops moving, e.g. Fig. 3
 * and Fig. 8); stops after the first iteration t whose flip count is below
 * flip_tol * N_t (N_t = particles at the start of t; flip_tol = 0 runs all
 * iterations), or in mode AUTO at the settled cycle of get_gradient_mode.  The stop is decided on the device, so the result
 * does not depend on how often the host looks.  Synchronises at the end;
 * *h_iters_done (may be NULL) receives the iterations executed. */
int32_t run(sobrc_ctx* ctx, int32_t max_iters, double flip_tol, int32_t mode,
            int32_t* h_iters_done, void* stream);

/* Synchronise `stream` and report the context's device-side status
 * (SOBRC_OK, SOBRC_ECAPACITY after an overflowing step). */
int32_t ctx_sync(sobrc_ctx* ctx, void* stream);

/* Current particle count (synchronises) and, for non-NULL arrays (each with
 * room for *h_n entries), the particles in context order: linear pixel index,
 * own label a and target label b (int32). */
int32_t get_particles(sobrc_ctx* ctx, int64_t* h_n, int32_t* d_lin, int32_t* d_a,
                      int32_t* d_b, void* stream);

/* Copy the current label field to d_labels (int32, nvox).  Asynchronous. */
int32_t get_labels(sobrc_ctx* ctx, int32_t* d_labels, void* stream);

/* Copy the current label field as the context holds it (uint16, nvox,
 * x fastest) to `labels`: device memory or page-locked host memory
 * (hipHostMalloc; pageable host memory makes the copy synchronous).  One
 * asynchronous copy on `stream`, half the bytes of get_labels: the result
 * path of a serving loop.  EINVAL for NULL arguments, ESTATE before
 * init_labels. */
int32_t get_labels_u16(sobrc_ctx* ctx, uint16_t* labels, void* stream);

/* Region statistics per label (synchronises): pixel count and intensity sum
 * (h_sum may be NULL).  Sums are kept exactly: integers for uint16 images,
 * 2^-s fixed point for fp32 images (s chosen at init_labels from max |I|). */
int32_t get_region_stats(sobrc_ctx* ctx, int64_t* h_count, double* h_sum, void* stream);

/* Per-iteration telemetry of the last iterations (synchronises): for up to
 * `cap` most recent iterations, particle count N_t, flips_t and (h_reversals
 * may be NULL) reversals_t -- flips of pixels that also changed in iteration
 * t - 1 -- oldest first.  *h_len receives the number written. */
int32_t get_history(sobrc_ctx* ctx, int32_t cap, int32_t* h_n, int32_t* h_flips,
                    int32_t* h_reversals, int32_t* h_len, void* stream);

/* Oscillation fallback of mode AUTO (synchronises).  Iteration t oscillates
 * when flips_t > 0 and 2 * reversals_t >= flips_t.  An AUTO iteration t that
 * oscillates right after an oscillating iteration t - 1 makes every later
 * AUTO iteration use L2-type gradients; *h_switch_iter receives that first
 * L2 iteration (counted from init_labels), or -1 while there is none.  The
 * switch lasts until the next init_labels; iterations count from
 * init_labels across step and run calls.  A run (or batch run) in mode AUTO
 * with flip_tol > 0 also stops after two iterations in a row that both used
 * L2 gradients and in which every flip was a reversal (a settled period-2
 * cycle: the contour sits in a minimum at pixel resolution). */
int32_t get_gradient_mode(sobrc_ctx* ctx, int32_t* h_switch_iter, void* stream);

/* Cell-shape autotuner (the cells of the neighbour search, text after
 * Eq. (6); shapes as SOBRC_TILE_*).  For each shape that params admits
 * (params->tile is ignored), builds a context inside d_workspace, runs
 * `iters` iterations (1..1000) of `mode` without a tolerance stop from
 * d_labels on d_image (int32 labels and the image as for init_labels),
 * after two warm-up iterations from the same start, and times them with HIP
 * events on `stream`, in two rounds with the shapes alternating.  h_ms[3]
 * receives the milliseconds per iteration (the faster round) of
 * SOBRC_TILE_DEFAULT, SOBRC_TILE_WIDE and SOBRC_TILE_TALL (-1 for a shape not
 * admitted); *h_tile is the fastest other shape if that is at least 1.5 %
 * faster than the default (the trials' timing noise reaches about 1 %), else
 * the default.  Results do not depend on the shape, so a caller then creates its
 * context with that tile.  d_workspace: device memory of at
 * least tile_autotune_workspace_size bytes, 256-byte aligned, owned by the
 * caller; its contents are scratch.  Synchronous.  EINVAL for NULL arguments
 * or iters out of range; errors of the trial runs (e.g. ECAPACITY) are
 * returned as they are. */
int32_t tile_autotune_workspace_size(const sobrc_params* params, size_t* bytes);
int32_t tile_autotune(const sobrc_params* params, const void* d_image, const int32_t* d_labels, int32_t iters,
                      int32_t mode, void* d_workspace, size_t bytes, int32_t* h_tile, double* h_ms,
                      void* stream);

/* ---- batches: many contexts advanced by one set of launches per iteration ----
 *
 * A batch is a table of n_slots slots, each empty or holding one initialised
 * context.  batch_step / batch_run advance every live slot by whole
 * iterations with seven launches per iteration for the whole batch (a
 * persistent grid per step kernel walks all slots' work); each context's
 * results are bit-identical to stepping it on its own.  The contexts of one
 * batch must share ndim, E and eps (the Sobolev kernel geometry); image
 * sizes, models, lambda, labels and capacities may differ.  While in a batch
 * a context accepts only read calls (get_*, compute_l2_diff, sobolev_smooth);
 * step, run, init_labels and ctx_destroy return ESTATE.  The workspace is
 * caller-owned device memory (256-byte aligned) that the batch borrows until
 * batch_destroy; contexts stay owned by the caller. */
typedef struct sobrc_batch sobrc_batch;

int32_t batch_workspace_size(int32_t n_slots, size_t* bytes);
int32_t batch_create(int32_t n_slots, void* d_workspace, size_t bytes, sobrc_batch** out);
/* Releases the host object and frees every slot (contexts are not destroyed). */
int32_t batch_destroy(sobrc_batch* batch);

/* Put an initialised context into `slot` (ctx != NULL) or empty the slot
 * (ctx == NULL); a context already in the slot leaves it.  Synchronises
 * `stream`.  EINVAL: slot out of range, or a context whose ndim / E / eps
 * differ from the batch's; ESTATE: context not initialised or in another
 * slot. */
int32_t batch_set(sobrc_batch* batch, int32_t slot, sobrc_ctx* ctx, void* stream);

/* One iteration of every live slot (as step() on each).  Asynchronous. */
int32_t batch_step(sobrc_batch* batch, int32_t mode, void* stream);

/* Up to max_iters iterations of every live slot; each slot stops on its own
 * tolerance (as run() on each) while the others go on.  Synchronises at the
 * end; h_iters_done (n_slots entries, may be NULL) receives each slot's
 * iterations (0 for empty slots).  Returns the first error status of a
 * slot, else SOBRC_OK. */
int32_t batch_run(sobrc_batch* batch, int32_t max_iters, double flip_tol, int32_t mode,
                  int32_t* h_iters_done, void* stream);

/* The two halves of batch_run, for callers that keep several batches busy at
 * once (one stream each): batch_launch_iters enqueues `iters` iterations of
 * every live slot (each stops on its own tolerance) without synchronising;
 * batch_collect synchronises `stream`, writes per slot (n_slots entries each,
 * may be NULL) the iterations committed since its init_labels and its state
 * (h_stopped: 0 running, 1 stopped at its tolerance, or the slot's negative
 * SOBRC_E* status, e.g. SOBRC_ECAPACITY after a rolled-back step), clears the
 * tolerance stops, and returns the first error status of a slot.  A failed
 * slot does nothing more until its context leaves the batch and is
 * re-initialised; the other slots are unaffected. */
int32_t batch_launch_iters(sobrc_batch* batch, int32_t iters, double flip_tol, int32_t mode,
                           void* stream);
int32_t batch_collect(sobrc_batch* batch, int32_t* h_iters, int32_t* h_stopped, void* stream);

/* Launch shape of the batch's slots: particles per block-item of the
 * particle kernels (part_chunk), log2 of the tiles per emission range
 * (lg_range, <= 8) and tiles per Sobolev block-item of the generic Sobolev
 * kernel (sob_tiles; the brick kernel takes the batch's non-empty tiles as
 * they come); 0 keeps each context's own stand-alone value.  Shapes only
 * regroup the work -- integer
 * partial sums, the tile-major particle order and every tile's Sobolev sums
 * are unchanged -- so results do not depend on them.  Synchronises. */
int32_t batch_set_shape(sobrc_batch* batch, int32_t part_chunk, int32_t lg_range,
                        int32_t sob_tiles, void* stream);

/* Autotuner: runs every live slot through a fixed list of launch shapes,
 * iters_per_trial + 1 iterations each (the real iterations of the run, which
 * the shape does not affect), times each trial with HIP events and keeps the
 * fastest shape.  h_shape (3 entries, may be NULL) receives it,
 * *h_iters_done (may be NULL) the iterations run.  Synchronises. */
int32_t batch_autotune(sobrc_batch* batch, int32_t mode, int32_t iters_per_trial,
                       int32_t* h_shape, int32_t* h_iters_done, void* stream);

/* Stateless Eq. (6) on caller-given particles (any order, n >= 0): positions
 * as linear indices d_lin, labels d_a != d_b in [0, max_labels), values d_in;
 * writes d_out in the input order.  Needs a device workspace of
 * sobolev_particles_workspace_size bytes.  Synchronises once to validate the
 * particles (EINVAL on bad input).  fp32 sums are summed in an order that
 * depends on the binning, so repeated calls may differ in the last bits. */
int32_t sobolev_particles_workspace_size(const sobrc_params* params, int64_t n,
                                         size_t* bytes);
int32_t sobolev_smooth_particles(const sobrc_params* params, int64_t n,
                                 const int32_t* d_lin, const int32_t* d_a,
                                 const int32_t* d_b, const float* d_in, float* d_out,
                                 void* d_workspace, size_t ws_bytes, void* stream);

/* sobolev_smooth_particles for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation with its scratch memory in a static
 * device array of SOBRC_STATIC_SCRATCH_BYTES (one per GPU, held until the
 * process ends); the caller passes only inputs and outputs.  Allocates
 * nothing.  EINVAL when sobolev_particles_workspace_size(params, n) exceeds
 * the static size.  Every call on one GPU uses that GPU's one array: calls
 * that overlap on one GPU (other streams or threads) race and must be
 * serialised by the caller.  Synchronises once, as sobolev_smooth_particles. */
#define SOBRC_STATIC_SCRATCH_BYTES (32u << 20)
int32_t sobolev_smooth_particles_static(const sobrc_params* params, int64_t n,
                                        const int32_t* d_lin, const int32_t* d_a,
                                        const int32_t* d_b, const float* d_in, float* d_out,
                                        void* stream);

/* Kernel timing with HIP events on the launch stream.  profile_enable(ctx, 1)
 * records an event pair around every kernel the context launches;
 * profile_read synchronises and returns, per kernel kind k (see
 * SOBRC_K_* below), the summed milliseconds and launch count since the last
 * reset.  Kinds: */
enum { SOBRC_K_L2DIFF = 0, SOBRC_K_SOBOLEV = 1, SOBRC_K_FLIP = 2, SOBRC_K_COUNT = 3,
       SOBRC_K_SCAN = 4, SOBRC_K_WRITE = 5, SOBRC_K_TOPO = 6, SOBRC_K_DECONV = 7, SOBRC_K_NKINDS = 8 };
int32_t profile_enable(sobrc_ctx* ctx, int32_t on);
int32_t profile_read(sobrc_ctx* ctx, double* h_ms, int64_t* h_launches, int32_t reset);

const char* last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SOBRC_H */
