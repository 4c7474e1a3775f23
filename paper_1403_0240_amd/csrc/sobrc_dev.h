// sobrc_dev.h -- internal types shared by the HIP kernels and the C ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sobrc {

constexpr int kBlock = 256;        // threads per block of the particle/tile kernels
constexpr int kSobBlock = 256;     // threads per block of the Sobolev kernels
constexpr int kScanThreads = 1024; // single-block scan of per-block partials
constexpr int kHist = 4096;        // telemetry ring (iterations)
constexpr int kStageCap = 2048;    // staged neighbour particles per round (generic Sobolev path)
constexpr int kMaxT = 1024;        // support table entries: d^2 < T <= (E/2)^2 rounded up
constexpr int kMaxLim = 81;        // (h+1)^2 for the largest brick halo (2D, h = 8)
constexpr int kSmallM = 16;        // label counts up to this use per-block statistics partials
constexpr int kMaxGrid = 2048;     // blocks of the particle and emission kernels
constexpr int kPsLdsMax = 64 * 1024;  // LDS bound of the tile-staged PS L2 gradient

// Tile shapes (cells of the particle lists): the default 8x8x8 voxels in 3D
// and 16x16 pixels in 2D (wide = 0); the wide shape, twice as long along one
// axis (16x8x8 in 3D, along x; 16x32 in 2D, along y; wide = 1); in 2D also
// the tall shape 16x64 (wide = 2).  Every shape keeps at most 16 pixels per
// tile row and at most 64 rows, the emission slot's format.
__host__ __device__ constexpr int tile_ex(int nd, int wide) { return nd == 3 ? (wide ? 16 : 8) : 16; }
__host__ __device__ constexpr int tile_ey(int nd, int wide) { return nd == 3 ? 8 : (16 << wide); }
__host__ __device__ constexpr int tile_ez(int nd) { return nd == 3 ? 8 : 1; }

// Largest axis offset h with h*h < T: the halo a Sobolev brick needs.
// Bricks exist for 3D halos 1..4 and 2D halos 1..8, for both tile shapes.
// Emission slot of a tile (written by the particle count when the tile is
// dirty, valid until it is dirty again): word 0 = lo | hi << 16 of a
// two-label box (0xFFFF: several labels); words 1..64: per tile row
// (ly + TY*lz), particle bits | bits of pixels labelled lo << 16 (zero for a
// tile whose box holds one label); words 65..128: particles in the rows
// before (the row's offset in the tile).
constexpr int kSlotRows = 64;
constexpr int kSlotWords = 1 + 2 * kSlotRows;
constexpr int kBrickMaxH3 = 4;
constexpr int kBrickMaxH2 = 8;

// LDS bytes of a brick kernel: the dense brick (two fp32 values per cell) and
// two side bitmasks per box row or, if larger, the generic path's staging of
// 256 particles with its weight table.
__host__ __device__ constexpr int brick_rows(int nd, int h, int wide)
{
    return (tile_ey(nd, wide) + 2 * h) * (nd == 3 ? tile_ez(nd) + 2 * h : 1);
}
__host__ __device__ constexpr int brick_cells(int nd, int h, int wide)
{
    // rows padded to an odd stride (see the brick kernels)
    return ((tile_ex(nd, wide) + 2 * h) | 1) * brick_rows(nd, h, wide);
}
__host__ __device__ constexpr int brick_lds_bytes(int nd, int h, int wide)
{
    return brick_cells(nd, h, wide) * 8 + brick_rows(nd, h, wide) * 8 > 256 * 12 + kMaxLim * 4 + 16
               ? brick_cells(nd, h, wide) * 8 + brick_rows(nd, h, wide) * 8
               : 256 * 12 + kMaxLim * 4 + 16;
}

// Kernel weights by integer squared distance: w[d2] = K(sqrt(d2)) inside the
// support (d2 < T), 0 outside.  Support rows: rw[(dy + h) + (2h + 1)(dz + hz)]
// is the largest dx >= 0 with dx^2 + dy^2 + dz^2 < T, or -1 if there is none
// (h = halo, hz = h in 3D and 0 in 2D).
struct SobW {
    float w[kMaxLim];
    int rw[kMaxLim];
};

// Deconvolving model: separable Gaussian PSF taps (per axis), passed by value.
constexpr int kPsfMaxR = 48;                 // sigma <= 16, truncated at 3 sigma
constexpr int kPsfTaps = 2 * kPsfMaxR + 1;
constexpr int kDeconvM = 4;                  // labels of a deconvolving context
constexpr int kDeconvSums = kDeconvM * (kDeconvM + 1) / 2 + kDeconvM;  // normal-equation sums
constexpr int kDeconvGrid = 512;             // blocks of the per-pixel deconvolution kernels
struct Psf {
    int r;                 // radius: taps t = -r .. r
    float k[kPsfTaps];     // K per axis, sum 1
    float k2[kPsfTaps];    // K^2 per axis (for the move's own term)
};

// error bits kept on the device (sticky until init_labels)
constexpr unsigned kErrCapacity = 1u;
constexpr unsigned kErrLabel = 2u;
constexpr unsigned kErrInput = 4u;
constexpr unsigned kErrTopo = 8u;  // ranked acceptance did not finish within kTopoMaxPasses

// Parallel rounds of the ranked acceptance before one block finishes the rest.
constexpr int kTopoRounds = 16;
constexpr int kTopoMaxPasses = 4096;  // passes of the finishing block over the tiles left

// Problem geometry and parameters, passed by value to every kernel.
struct Geom {
    int nx, ny, nz, ndim;
    int tsx, tsy, tsz;          // log2 of the tile edge per axis
    int wide;                   // tile shape: 0 default, 1 wide, 2 tall (2D; tile_ex/ey/ez)
    int ntx, nty, ntz, ntiles;  // tiles per axis, total
    int sy, sz;                 // particle position packing: x | y << sy | z << sz
    unsigned mx, my, mz;        // field masks after shifting
    int T;                      // Sobolev support: integer d^2 < T  <=>  d < E/2
    int h;                      // largest axis offset k with k*k < T
    int R, R2;                  // PS ball radius and radius^2
    int model;                  // 0 PC, 1 PS
    int noise;                  // 0 Gaussian, 1 Poisson pixel noise
    int img_u16;                // image element type
    float lambda;
    double fx_scale;            // fixed-point scale of intensity sums (2^s)
    double fx_inv;              // 1 / fx_scale
    int max_labels;
    int small_m;                // max_labels <= kSmallM
    int gp;                     // blocks of the particle kernels (l2diff, flip)
    int ge, Re, lgRe;           // emission ranges: count, tiles per range (2^lgRe)
    int brick;                  // Sobolev brick kernel for (ndim, h) exists
    int full;                   // T == (h+1)^2: every offset of the brick stencil is inside
    int stage_cap;              // generic-path staging capacity
    int sob_lds;                // dynamic LDS bytes of the generic Sobolev kernel
    int sob_grid;               // blocks of the generic Sobolev and tile-staged kernels (multiple of 8)
    int brick_grid;             // blocks of the stand-alone brick Sobolev kernel (multiple of 8)
    int ps_lds;                 // PS model: LDS bytes of the tile-staged L2 gradient (0: per particle)
    int dlistm;                 // dirty tiles go through a flat list balanced over all waves (ge <= kMaxGrid)
    int topo;                   // ranked acceptance with topological control
    int psf;                    // deconvolving model (Gaussian PSF)
};

// Device-resident control block of a context.
struct DevState {
    unsigned n[2];          // particle count of state buffer 0/1
    unsigned n_active[2];   // non-empty tiles of state buffer 0/1
    unsigned nflips;        // pixels changed by the running step
    unsigned epoch;         // iteration stamp of dirty tiles (bumped at each step start)
    unsigned err;           // sticky error bits
    unsigned undo;          // running step overflowed: roll back in k_write
    unsigned go;            // running step passed k_scan and commits in k_write
    unsigned need;          // particle count that did not fit
    unsigned converged;     // flip tolerance reached: further steps do nothing
    unsigned iters;         // steps committed
    unsigned maxbits;       // init: bit pattern of max |I| (fp32 images)
    unsigned lmode;         // bit 0: L2 gradients in force for the running step (auto mode, latched at its
                            // start); bit 1: the last committed step oscillated (reversals >= flips / 2);
                            // bit 2: every flip of the last committed step was a reversal
    unsigned switch_it;     // 1 + first iteration run with L2 gradients in auto mode, 0: none yet
    unsigned ndirty;        // dirty tiles of the running step (flat list, when listed)
    unsigned topo_cnt[kTopoRounds + 1];  // ranked acceptance: tiles listed for each round
};

// A block's place in the work of one context: its index and the block count
// of that context's launch.  Stand-alone launches use the hardware block
// index; batched launches map their blocks onto the contexts of the batch.
struct VB {
    unsigned id, n;
};

// Step-kernel flags: stop when the context has stopped (error or tolerance);
// auto gradient mode (Sobolev until oscillation, then L2).
constexpr int kGate = 1, kAuto = 2;


// Device pointers of one context (all carved from the caller's workspace).
struct Bufs {
    unsigned short* lab;     // label field, nvox
    unsigned short* labt;    // the same labels tile-major (ntiles x tile pixels), read by the particle count
    uint2* rec[2];           // particle records {pos, a | b << 16}, capacity each
    unsigned* tstart[2];     // tile_start, ntiles + 1 each
    unsigned* active[2];     // non-empty tiles, ntiles each
    unsigned* tcnt;          // per-tile particle count of the next state
    unsigned* dirty;         // epoch of the last flip within one pixel of the tile
    unsigned* fstamp;        // per pixel: 1 + the last iteration that changed its label (0: never)
    unsigned* dcnt;          // per emission block: dirty tiles it listed
    unsigned* dlist;         // per emission block: its dirty tiles (kBlock entries each)
    unsigned* dflat;         // dirty tiles of the step, flat: positions in dlist (ntiles entries)
    unsigned* tslot;         // per tile: emission bitmasks from k_count for k_write
    float* dE;               // L2 gradient, capacity
    float* gH1;              // Sobolev gradient, capacity
    float* dv;               // brick kernels: L2 gradient per pixel, tile-major (ntiles x tile pixels;
                             // meaningful at the particles of the current set only)
    long long* st_n;         // region pixel counts, max_labels
    long long* st_s1;        // region intensity sums (fixed point), max_labels
    float4* lstat;           // per label: mean, n/(n-1) (0 if n <= 1), n/(n+1)
    float* W;                // kernel table W[d^2], T entries
    unsigned* hist;          // 2 * kHist: N_t and flips_t
    unsigned* part_f;        // per k_flip block: flips [gp], then reversals [gp]
    long long* part_n;       // per label x k_flip block: pixel-count deltas (small M)
    long long* part_q;       // per label x k_flip block: intensity-sum deltas (small M)
    unsigned* part_cnt;      // particles per emission block (tiles [b*Re, (b+1)*Re))
    unsigned* part_act;      // non-empty tiles per emission block
    unsigned* part_off;      // exclusive prefix of part_cnt
    unsigned* part_aoff;     // exclusive prefix of part_act
    // ranked acceptance with topological control (topo only)
    unsigned char* tstate;   // per particle: 0 no candidate, 1 undecided, 2 executed, 3 refused
    unsigned* tmark;         // per tile: odd stamp of the iteration that listed it
    unsigned* tlist[2];      // tiles of the even / odd rounds
    unsigned long long* pmap;  // per pixel: smallest undecided key << 16 | label (~0: no candidate)
    // deconvolving model (psf only)
    float* du;               // K * chi_l for labels 1 .. M-1, nvox each
    float* dt[2];            // scratch images of the separable passes
    float* dC;               // K * (I - J): correlation of the residual with the PSF
    float* dN;               // sum over the image of K(y - x)^2, per pixel x
    float* dw;               // K * 1: PSF mass inside the image, per pixel
    double* dtheta;          // region intensities (least squares), M
    double* dpart;           // per block: normal-equation partial sums (kDeconvSums)
    DevState* ds;
    unsigned cap;
};

// One slot of a batch (device memory): the context's geometry, buffers and
// image; live = 0 marks an empty slot.
struct ImgDesc {
    Geom g;
    Bufs b;
    const void* img;
    unsigned live;
    unsigned pad;
};

// Item spaces of a batched step: per slot, the blocks the context would
// launch on its own -- particle kernels (gp), emission kernels (ge), the
// generic Sobolev kernel (sob_grid), one scan block -- and the blocks of the
// dirty-tile count (at most kBatchListItems).  Each slot's range starts at a
// multiple of 8 so that item & 7 names the XCD as in a stand-alone launch.
// The brick Sobolev kernel instead deals the batch's non-empty tiles
// (BatchTab::tpre).
enum { kPhPart = 0, kPhEmit = 1, kPhSob = 2, kPhScan = 3, kPhList = 4, kNumPh = 5 };
// blocks of the batched dirty-tile count per image (its waves take the
// image's dirty tiles round-robin; each block forms the prefix of the
// image's list lengths, so more blocks than the dirty tiles need only cost)
constexpr int kBatchListItems = 32;
constexpr int kPersist = 2048;  // blocks of a persistent batched launch
constexpr int kListGrid = 1024;  // blocks of the dirty-list count (all resident at once)

struct BatchTab {
    const ImgDesc* d;     // nslot descriptors
    unsigned* par;        // per slot: parity of the current state buffer
    const unsigned* off;  // kNumPh rows of nslot + 1 item offsets
    unsigned* tpre;       // nslot + 1: prefix of the slots' non-empty tile counts (device-written)
    int nslot;
};


// Host wrappers around kernel launches (defined in sobrc_kernels.hip).
hipError_t launch_init_labels(const Geom& g, const Bufs& b, const int32_t* labels_in,
                              const void* img, hipStream_t s);
hipError_t launch_stats_init(const Geom& g, const Bufs& b, const void* img, hipStream_t s);
hipError_t launch_l2diff(const Geom& g, const Bufs& b, const void* img, int cur, float* out,
                         int gated, hipStream_t s);
// L2 gradients given in record order to the per-pixel field of the brick kernels.
hipError_t launch_dense_put(const Geom& g, const Bufs& b, int cur, const float* in, hipStream_t s);
hipError_t launch_sobolev(const Geom& g, const Bufs& b, const SobW& sw, int cur, const float* in,
                          float* out, int gated, int use_slots, hipStream_t s);
hipError_t launch_flip(const Geom& g, const Bufs& b, const void* img, int cur, const float* grad,
                       const float* grad_l2, int flags, hipStream_t s);
hipError_t launch_topo(const Geom& g, const Bufs& b, int cur, const float* grad, const float* grad_l2,
                       int flags, hipStream_t s);
hipError_t launch_count(const Geom& g, const Bufs& b, int cur, int gated, int all_dirty, hipStream_t s);
hipError_t launch_deconv_init(const Geom& g, const Bufs& b, const Psf& k, hipStream_t s);
hipError_t launch_deconv(const Geom& g, const Bufs& b, const Psf& k, const void* img, hipStream_t s);
hipError_t launch_scan(const Geom& g, const Bufs& b, int cur, int nxt, int is_init, float tol,
                       int32_t* d_nflips, int gated, hipStream_t s);
hipError_t launch_write(const Geom& g, const Bufs& b, const void* img, int cur, int nxt,
                        const float* grad, const float* grad_l2, int flags, int all_dirty, hipStream_t s);
// One batched iteration: every live slot advances by one step (seven
// launches: gradient, Sobolev, acceptance, count, scan, write, parity).
// totals: item counts per phase (host copy of the offsets' last entries).
hipError_t launch_batch_step(const BatchTab& t, const unsigned* totals, const Geom& g0, const SobW& sw,
                             int l2, int flags, float tol, hipStream_t s);
hipError_t launch_batch_clear(const BatchTab& t, hipStream_t s);
hipError_t launch_batch_gather(const BatchTab& t, uint4* out, hipStream_t s);
hipError_t launch_unpack(const Geom& g, const Bufs& b, int cur, int32_t* lin, int32_t* a,
                         int32_t* bb, hipStream_t s);
hipError_t launch_labels_out(const Geom& g, const Bufs& b, int32_t* out, hipStream_t s);

hipError_t launch_fill_u32(unsigned* p, unsigned v, size_t n, hipStream_t s);

// Stateless binning for sobolev_smooth_particles.
hipError_t launch_bin_count(const Geom& g, const Bufs& b, long long n, const int32_t* lin,
                            const int32_t* a, const int32_t* bb, hipStream_t s);
hipError_t launch_bin_scan(const Geom& g, const Bufs& b, hipStream_t s);
hipError_t launch_bin_scatter(const Geom& g, const Bufs& b, long long n, const int32_t* lin,
                              const int32_t* a, const int32_t* bb, const float* in,
                              unsigned* fill, unsigned* origin, hipStream_t s);
hipError_t launch_unbin(const Bufs& b, long long n, const unsigned* origin, const float* binned,
                        float* out, hipStream_t s);

}  // namespace sobrc
