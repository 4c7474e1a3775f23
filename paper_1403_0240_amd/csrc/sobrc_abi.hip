// sobrc_abi.hip -- extern "C" entry points declared in include/sobrc.h.
//
// Host-side work only: parameter validation, workspace layout, the kernel
// table W[d^2] of Eq. (5) in FP64, launch sequencing and error reporting.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "sobrc.h"
#include "sobrc_dev.h"

using namespace sobrc;

namespace {

thread_local char g_err[512];

int32_t fail(int32_t code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int32_t dev_fail(hipError_t e, const char* where)
{
    return fail(SOBRC_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

#define SOBRC_HIP(call, where)                 \
    do {                                       \
        hipError_t e_ = (call);                \
        if (e_ != hipSuccess)                  \
            return dev_fail(e_, where);        \
    } while (0)

int32_t validate(const sobrc_params* p)
{
    if (!p)
        return fail(SOBRC_EINVAL, "params is NULL");
    if (p->ndim != 2 && p->ndim != 3)
        return fail(SOBRC_EINVAL, "ndim must be 2 or 3 (got %d)", p->ndim);
    int lim = p->ndim == 3 ? 1024 : 32768;
    if (p->nx < 1 || p->ny < 1 || p->nx > lim || p->ny > lim)
        return fail(SOBRC_EINVAL, "nx, ny must lie in [1, %d] (got %d, %d)", lim, p->nx, p->ny);
    if (p->ndim == 2 && p->nz != 1)
        return fail(SOBRC_EINVAL, "2D images need nz = 1 (got %d)", p->nz);
    if (p->ndim == 3 && (p->nz < 1 || p->nz > 1024))
        return fail(SOBRC_EINVAL, "nz must lie in [1, 1024] (got %d)", p->nz);
    if (p->image_dtype != SOBRC_F32 && p->image_dtype != SOBRC_U16)
        return fail(SOBRC_EINVAL, "image_dtype must be SOBRC_F32 or SOBRC_U16");
    if (p->model != SOBRC_PC && p->model != SOBRC_PS)
        return fail(SOBRC_EINVAL, "model must be SOBRC_PC or SOBRC_PS");
    if (p->noise != SOBRC_NOISE_GAUSS && p->noise != SOBRC_NOISE_POISSON)
        return fail(SOBRC_EINVAL, "noise must be SOBRC_NOISE_GAUSS or SOBRC_NOISE_POISSON");
    if (p->model == SOBRC_PS && (p->ps_radius < 2 || p->ps_radius > 32))
        return fail(SOBRC_EINVAL, "ps_radius must lie in [2, 32] (got %d)", p->ps_radius);
    if (!(p->E > 0.0 && p->E <= 64.0))
        return fail(SOBRC_EINVAL, "E must lie in (0, 64] (got %g)", p->E);
    if (!(p->eps > 0.0 && isfinite(p->eps)))
        return fail(SOBRC_EINVAL, "eps must be positive (got %g)", p->eps);
    if (!(p->lambda >= 0.0 && isfinite(p->lambda)))
        return fail(SOBRC_EINVAL, "lambda must be >= 0 (got %g)", p->lambda);
    if (p->max_labels < 2 || p->max_labels > 65535)
        return fail(SOBRC_EINVAL, "max_labels must lie in [2, 65535] (got %d)", p->max_labels);
    if (p->max_particles < 1 || p->max_particles > 0x7fffffffLL)
        return fail(SOBRC_EINVAL, "max_particles must lie in [1, 2^31-1]");
    if (p->topo != SOBRC_TOPO_OFF && p->topo != SOBRC_TOPO_SIMPLE)
        return fail(SOBRC_EINVAL, "topo must be SOBRC_TOPO_OFF or SOBRC_TOPO_SIMPLE");
    if (!(p->psf_sigma >= 0.0 && p->psf_sigma <= kPsfMaxR / 3.0))
        return fail(SOBRC_EINVAL, "psf_sigma must lie in [0, %d] (got %g)", kPsfMaxR / 3, p->psf_sigma);
    if (p->psf_sigma > 0.0 && (p->model != SOBRC_PC || p->noise != SOBRC_NOISE_GAUSS || p->max_labels > kDeconvM))
        return fail(SOBRC_EINVAL, "the deconvolving model needs SOBRC_PC, SOBRC_NOISE_GAUSS and max_labels <= %d",
                    kDeconvM);
    if (p->tile != SOBRC_TILE_DEFAULT && p->tile != SOBRC_TILE_WIDE && p->tile != SOBRC_TILE_TALL)
        return fail(SOBRC_EINVAL, "tile must be SOBRC_TILE_DEFAULT, SOBRC_TILE_WIDE or SOBRC_TILE_TALL (got %d)",
                    p->tile);
    if (p->tile == SOBRC_TILE_TALL && p->ndim != 2)
        return fail(SOBRC_EINVAL, "SOBRC_TILE_TALL is a 2D shape");
    if (p->tile != SOBRC_TILE_DEFAULT && p->topo != SOBRC_TOPO_OFF)
        return fail(SOBRC_EINVAL, "topological control runs on the default tile shape only");
    return SOBRC_OK;
}

// Support of the discrete kernel: d < E/2 with d^2 integer  <=>  d^2 < T.
int support_T(double E)
{
    double r2 = (E / 2.0) * (E / 2.0);
    int T = (int)ceil(r2);
    if (T < 1)
        T = 1;
    // guard against r2 landing a rounding step away from an integer
    while (T > 1 && !(sqrt((double)(T - 1)) < E / 2.0))
        --T;
    while (sqrt((double)T) < E / 2.0)
        ++T;
    return T;
}

Geom make_geom(const sobrc_params* p)
{
    Geom g{};
    g.nx = p->nx;
    g.ny = p->ny;
    g.nz = p->ndim == 3 ? p->nz : 1;
    g.ndim = p->ndim;
    g.wide = p->tile;
    if (p->ndim == 3) {
        g.tsx = g.wide ? 4 : 3;  // 8x8x8 or 16x8x8 voxel tiles
        g.tsy = g.tsz = 3;
        g.sy = 10;
        g.sz = 20;
        g.mx = g.my = g.mz = 1023u;
    } else {
        g.tsx = 4;                  // 16x16, 16x32 or 16x64 pixel tiles
        g.tsy = 4 + g.wide;
        g.tsz = 0;
        g.sy = 16;
        g.sz = 31;
        g.mx = g.my = 0xffffu;
        g.mz = 0u;
    }
    g.ntx = (g.nx + (1 << g.tsx) - 1) >> g.tsx;
    g.nty = (g.ny + (1 << g.tsy) - 1) >> g.tsy;
    g.ntz = (g.nz + (1 << g.tsz) - 1) >> g.tsz;
    g.ntiles = g.ntx * g.nty * g.ntz;
    g.T = support_T(p->E);
    int h = 0;
    while ((h + 1) * (h + 1) < g.T)
        ++h;
    g.h = h;
    g.R = p->model == SOBRC_PS ? p->ps_radius : 0;
    g.R2 = g.R * g.R;
    g.model = p->model;
    g.noise = p->noise;
    g.topo = p->topo;
    g.psf = p->psf_sigma > 0.0 ? 1 : 0;
    g.img_u16 = p->image_dtype == SOBRC_U16;
    g.lambda = (float)p->lambda;
    g.fx_scale = 1.0;
    g.fx_inv = 1.0;
    g.max_labels = p->max_labels;
    g.small_m = p->max_labels <= kSmallM;
    long long gp = (p->max_particles + kBlock - 1) / kBlock;
    gp = gp < 8 ? gp : (gp + 7) / 8 * 8;  // whole rounds over the 8 XCDs
    g.gp = (int)(gp < 1 ? 1 : (gp > kMaxGrid ? kMaxGrid : gp));
    // emission ranges of Re = 2^lgRe tiles, at most kMaxGrid / 2 ranges unless
    // a range would exceed kBlock tiles (the count and write kernels take one
    // block per range; 1024 of them are resident at once)
    g.lgRe = 0;
    while ((1LL << g.lgRe) * (kMaxGrid / 2) < g.ntiles && (1 << g.lgRe) < kBlock)
        ++g.lgRe;
    g.Re = 1 << g.lgRe;
    g.ge = (g.ntiles + g.Re - 1) >> g.lgRe;
    // a flat dirty list pays when an emission block holds many tiles
    g.dlistm = g.ge <= kMaxGrid && g.Re >= 8 ? 1 : 0;
    // Sobolev kernel: dense LDS brick for (ndim, h) when instantiated, else
    // the generic staged scan
    g.brick = g.h >= 1 && g.h <= (g.ndim == 3 ? kBrickMaxH3 : kBrickMaxH2);
    g.full = g.T == (g.h + 1) * (g.h + 1);
    int fixed = g.T * 4 + (kSobBlock / 64) * 4;
    // The brick kernel falls back to the staged scan inside its static LDS,
    // so the staging capacity must fit there; the generic kernel (also used
    // by the stateless entry point) takes the same capacity as dynamic LDS.
    g.stage_cap = kStageCap;
    if (g.brick) {
        int cap = (brick_lds_bytes(g.ndim, g.h, g.wide) - fixed) / 12 / kSobBlock * kSobBlock;
        g.stage_cap = cap > kStageCap ? kStageCap : cap;
    }
    g.sob_lds = g.stage_cap * 12 + fixed;
    int sg = g.ntiles < 2 * kMaxGrid ? g.ntiles : 2 * kMaxGrid;  // mostly one tile per block
    g.sob_grid = (sg + 7) / 8 * 8;
    // the brick kernel: up to twice as many blocks as the other tile
    // kernels (the surplus exits at once; measured faster on the 3D workload)
    const int bg = g.ntiles < 4 * kMaxGrid ? g.ntiles : 4 * kMaxGrid;
    g.brick_grid = (bg + 7) / 8 * 8;
    // PS model: tile-staged L2 gradient when the tile's box (tile and R pixels
    // on every side; fp32 intensity and label, 8 bytes per pixel) fits the LDS bound
    g.ps_lds = 0;
    if (g.model == SOBRC_PS && !g.psf) {
        const long long rz = g.ndim == 3 ? g.R : 0;
        const long long cells = ((1LL << g.tsx) + 2LL * g.R) * ((1LL << g.tsy) + 2LL * g.R) * ((1LL << g.tsz) + 2 * rz);
        const long long bytes = cells * 8 + (2LL * g.R + 1) * (2 * rz + 1) * 4;  // box, row half-widths
        if (bytes <= kPsLdsMax)
            g.ps_lds = (int)bytes;
    }
    return g;
}

// W[k] = K(sqrt(k)) of Eq. (5), k < T, computed in FP64 and rounded to fp32.
void kernel_table(double E, double eps, int T, float* W)
{
    for (int k = 0; k < T; ++k) {
        double u = sqrt((double)k) / E;
        double v = (1.0 + (u * u - u + 1.0 / 6.0) / (2.0 * eps)) / E;
        W[k] = (float)v;
    }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
    size_t lab, labt, fstamp, dcnt, dlist, dflat, rec0, rec1, ts0, ts1, act0, act1, tcnt, dirty, tslot, dE, gH1, dv, st_n, st_s1, lstat, W, hist,
        part_f, part_n, part_q, part_cnt, part_act, part_off, part_aoff, tstate, tmark, tlist0, tlist1, pmap, du, dt0, dt1, dC, dN, dw, dtheta, dpart, ds;
    size_t dv_bytes;
    size_t total;
};

Layout make_layout(const Geom& g, const sobrc_params* p, long long cap)
{
    Layout L{};
    size_t o = 0;
    long long nvox = (long long)g.nx * g.ny * g.nz;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = align256(o + bytes);
        return r;
    };
    L.lab = take((size_t)nvox * 2);
    L.labt = take((size_t)g.ntiles * ((size_t)1 << (g.tsx + g.tsy + g.tsz)) * 2);
    L.fstamp = take((size_t)nvox * 4);
    L.dcnt = take((size_t)kMaxGrid * 4);  // read as whole 16-byte groups
    L.dlist = take((size_t)g.ge * kBlock * 4);
    L.dflat = take((size_t)g.ntiles * 4);
    L.rec0 = take((size_t)cap * 8);
    L.rec1 = take((size_t)cap * 8);
    L.ts0 = take((size_t)(g.ntiles + 1) * 4);
    L.ts1 = take((size_t)(g.ntiles + 1) * 4);
    L.act0 = take((size_t)g.ntiles * 4);
    L.act1 = take((size_t)g.ntiles * 4);
    L.tcnt = take((size_t)g.ntiles * 4);
    L.dirty = take((size_t)g.ntiles * 4);
    L.tslot = take((size_t)g.ntiles * kSlotWords * 4);
    L.dE = take((size_t)cap * 4);
    L.gH1 = take((size_t)cap * 4);
    // brick kernels: the L2 gradient scattered to its pixel, whole tiles
    L.dv_bytes = g.brick ? (size_t)g.ntiles * ((size_t)1 << (g.tsx + g.tsy + g.tsz)) * 4 : 0;
    L.dv = take(L.dv_bytes);
    L.st_n = take((size_t)p->max_labels * 8);
    L.st_s1 = take((size_t)p->max_labels * 8);
    L.lstat = take((size_t)p->max_labels * 16);
    L.W = take((size_t)kMaxT * 4);
    L.hist = take((size_t)3 * kHist * 4);
    L.part_f = take((size_t)g.gp * 8);
    L.part_n = take((size_t)g.gp * kSmallM * 8);
    L.part_q = take((size_t)g.gp * kSmallM * 8);
    L.part_cnt = take((size_t)g.ge * 4);
    L.part_act = take((size_t)g.ge * 4);
    L.part_off = take((size_t)g.ge * 4);
    L.part_aoff = take((size_t)g.ge * 4);
    const bool topo = p->topo != SOBRC_TOPO_OFF;  // buffers of the ranked acceptance
    L.tstate = take(topo ? (size_t)cap : 0);
    L.tmark = take(topo ? (size_t)g.ntiles * 4 : 0);
    L.tlist0 = take(topo ? (size_t)g.ntiles * 4 : 0);
    L.tlist1 = take(topo ? (size_t)g.ntiles * 4 : 0);
    L.pmap = take(topo ? (size_t)nvox * 8 : 0);
    const bool psf = p->psf_sigma > 0.0;  // images of the deconvolving model
    L.du = take(psf ? (size_t)(p->max_labels - 1) * nvox * 4 : 0);
    L.dt0 = take(psf ? (size_t)nvox * 4 : 0);
    L.dt1 = take(psf ? (size_t)nvox * 4 : 0);
    L.dC = take(psf ? (size_t)nvox * 4 : 0);
    L.dN = take(psf ? (size_t)nvox * 4 : 0);
    L.dw = take(psf ? (size_t)nvox * 4 : 0);
    L.dtheta = take(psf ? (size_t)p->max_labels * 8 : 0);
    L.dpart = take(psf ? (size_t)kDeconvGrid * kDeconvSums * 8 : 0);
    L.ds = take(sizeof(DevState));
    L.total = o;
    return L;
}

Bufs carve(const Layout& L, char* base, long long cap)
{
    Bufs b{};
    b.lab = (unsigned short*)(base + L.lab);
    b.labt = (unsigned short*)(base + L.labt);
    b.fstamp = (unsigned*)(base + L.fstamp);
    b.dcnt = (unsigned*)(base + L.dcnt);
    b.dlist = (unsigned*)(base + L.dlist);
    b.dflat = (unsigned*)(base + L.dflat);
    b.rec[0] = (uint2*)(base + L.rec0);
    b.rec[1] = (uint2*)(base + L.rec1);
    b.tstart[0] = (unsigned*)(base + L.ts0);
    b.tstart[1] = (unsigned*)(base + L.ts1);
    b.active[0] = (unsigned*)(base + L.act0);
    b.active[1] = (unsigned*)(base + L.act1);
    b.tcnt = (unsigned*)(base + L.tcnt);
    b.dirty = (unsigned*)(base + L.dirty);
    b.tslot = (unsigned*)(base + L.tslot);
    b.dE = (float*)(base + L.dE);
    b.gH1 = (float*)(base + L.gH1);
    b.dv = L.dv_bytes ? (float*)(base + L.dv) : nullptr;
    b.st_n = (long long*)(base + L.st_n);
    b.st_s1 = (long long*)(base + L.st_s1);
    b.lstat = (float4*)(base + L.lstat);
    b.W = (float*)(base + L.W);
    b.hist = (unsigned*)(base + L.hist);
    b.part_f = (unsigned*)(base + L.part_f);
    b.part_n = (long long*)(base + L.part_n);
    b.part_q = (long long*)(base + L.part_q);
    b.part_cnt = (unsigned*)(base + L.part_cnt);
    b.part_act = (unsigned*)(base + L.part_act);
    b.part_off = (unsigned*)(base + L.part_off);
    b.part_aoff = (unsigned*)(base + L.part_aoff);
    b.tstate = (unsigned char*)(base + L.tstate);
    b.tmark = (unsigned*)(base + L.tmark);
    b.tlist[0] = (unsigned*)(base + L.tlist0);
    b.tlist[1] = (unsigned*)(base + L.tlist1);
    b.pmap = (unsigned long long*)(base + L.pmap);
    b.du = (float*)(base + L.du);
    b.dt[0] = (float*)(base + L.dt0);
    b.dt[1] = (float*)(base + L.dt1);
    b.dC = (float*)(base + L.dC);
    b.dN = (float*)(base + L.dN);
    b.dw = (float*)(base + L.dw);
    b.dtheta = (double*)(base + L.dtheta);
    b.dpart = (double*)(base + L.dpart);
    b.ds = (DevState*)(base + L.ds);
    b.cap = (unsigned)cap;
    return b;
}

// Upload the kernel table W[d^2] (generic path) and fill the by-value weights
// of the brick kernels.
int32_t upload_tables(const Geom& g, double E, double eps, float* d_W, SobW* sw, hipStream_t s)
{
    static thread_local float W[kMaxT];
    memset(W, 0, sizeof W);
    kernel_table(E, eps, g.T, W);
    for (int k = 0; k < kMaxLim; ++k) {
        sw->w[k] = k < g.T ? W[k] : 0.f;
        sw->rw[k] = -1;
    }
    const int hz = g.ndim == 3 ? g.h : 0;
    for (int dz = -hz; dz <= hz; ++dz)
        for (int dy = -g.h; dy <= g.h; ++dy) {
            int w = -1;
            while (w + 1 <= g.h && (w + 1) * (w + 1) + dy * dy + dz * dz < g.T)
                ++w;
            const int k = (dy + g.h) + (2 * g.h + 1) * (dz + hz);
            if (k < kMaxLim)
                sw->rw[k] = w;
        }
    SOBRC_HIP(hipMemcpyAsync(d_W, W, sizeof W, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    // the host array is reused by the next call: wait for the copy
    SOBRC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    return SOBRC_OK;
}

}  // namespace

// Per-axis taps of the Gaussian point-spread function (deconvolving model):
// exp(-t^2 / (2 sigma^2)) for |t| <= ceil(3 sigma), normalised to sum 1.
Psf make_psf(double sigma)
{
    Psf k{};
    if (!(sigma > 0.0))
        return k;
    k.r = (int)ceil(3.0 * sigma);
    double t[kPsfTaps], sum = 0.0;
    for (int i = -k.r; i <= k.r; ++i) {
        t[i + k.r] = exp(-(double)(i * i) / (2.0 * sigma * sigma));
        sum += t[i + k.r];
    }
    for (int i = 0; i <= 2 * k.r; ++i) {
        k.k[i] = (float)(t[i] / sum);
        k.k2[i] = (float)((t[i] / sum) * (t[i] / sum));
    }
    return k;
}

struct sobrc_ctx {
    sobrc_params p;
    Geom g;
    SobW sw{};
    Psf psf{};
    Layout L;
    Bufs b;
    const void* image = nullptr;
    int cur = 0;
    bool initialized = false;
    unsigned seen_err = 0;  // device error bits a synchronising call has read (cleared by init_labels)
    // hipGraph of two consecutive steps, per start parity and mode
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec[2][3] = {};  // [start parity][gradient mode]
    float gtol[2][3] = {};
    // profiling
    bool prof = false;
    std::vector<hipEvent_t> ev;   // pool, pairs
    std::vector<int> ev_kind;     // kind of each pair
    size_t ev_used = 0;           // pairs in use
    double prof_ms[SOBRC_K_NKINDS] = {};
    long long prof_n[SOBRC_K_NKINDS] = {};
    // batch membership: while in a batch the batch owns the parity
    sobrc_batch* batch = nullptr;
};

struct sobrc_batch {
    int nslot = 0;
    char* ws = nullptr;          // device tables: descriptors, parities, item offsets
    ImgDesc* d_desc = nullptr;
    unsigned* d_par = nullptr;
    unsigned* d_off = nullptr;
    uint4* d_state = nullptr;    // gathered per-slot state words
    unsigned* d_tpre = nullptr;  // prefix of the slots' non-empty tile counts
    std::vector<sobrc_ctx*> slot;
    std::vector<unsigned> off;   // host copy, kNumPh rows of nslot + 1
    unsigned totals[kNumPh] = {};
    bool has_class = false;      // kernel geometry shared by every slot
    Geom g0{};
    SobW sw{};
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec[3] = {};  // per gradient mode: two batched steps
    float gtol[3] = {};
    // launch shape of the slots (0: each context's own): particles per item
    // of the particle kernels, log2 tiles per emission range, tiles per
    // Sobolev item.  None of them changes any result.
    int part_chunk = 0, lg_range = 0, sob_tiles = 0;
};

namespace {

constexpr size_t kEventPairs = 8192;

// Launch with optional event pair around it (profiling).
template <typename F>
int32_t timed(sobrc_ctx* c, int kind, hipStream_t s, const char* where, F&& launch)
{
    bool t = c->prof && c->ev_used < kEventPairs;
    if (t)
        SOBRC_HIP(hipEventRecord(c->ev[2 * c->ev_used], s), "hipEventRecord");
    SOBRC_HIP(launch(), where);
    if (t) {
        SOBRC_HIP(hipEventRecord(c->ev[2 * c->ev_used + 1], s), "hipEventRecord");
        c->ev_kind[c->ev_used] = kind;
        ++c->ev_used;
    }
    return SOBRC_OK;
}

#define SOBRC_TRY(expr)            \
    do {                           \
        int32_t r_ = (expr);       \
        if (r_ != SOBRC_OK)        \
            return r_;             \
    } while (0)

int32_t read_state(sobrc_ctx* c, DevState* h, hipStream_t s)
{
    SOBRC_HIP(hipMemcpyAsync(h, c->b.ds, sizeof(DevState), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    SOBRC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    c->seen_err |= h->err;
    return SOBRC_OK;
}

int32_t status_of(const DevState& h)
{
    if (h.err & kErrCapacity)
        return fail(SOBRC_ECAPACITY, "particle set needs %u entries, capacity exceeded", h.need);
    if (h.err & kErrLabel)
        return fail(SOBRC_EINVAL, "label outside [0, max_labels)");
    if (h.err & kErrTopo)
        return fail(SOBRC_EDEVICE, "ranked acceptance did not finish within %d passes", kTopoMaxPasses);
    return SOBRC_OK;
}

// Launch one iteration on stream s, reading state buffer `cur` and writing
// the other; the host parity c->cur flips.
int32_t launch_step(sobrc_ctx* c, int mode, int32_t* d_nflips, float tol, hipStream_t s)
{
    int cur = c->cur, nxt = 1 - cur;
    const Geom& g = c->g;
    const Bufs& b = c->b;
    // auto mode: the Sobolev kernel skips itself and the acceptance reads the
    // L2 gradients once the device has switched (latched per step)
    const int flags = kGate | (mode == SOBRC_MODE_AUTO ? kAuto : 0);
    if (g.psf)
        SOBRC_TRY(timed(c, SOBRC_K_DECONV, s, "k_deconv",
                        [&] { return launch_deconv(g, b, c->psf, c->image, s); }));
    SOBRC_TRY(timed(c, SOBRC_K_L2DIFF, s, "k_l2diff",
                    [&] { return launch_l2diff(g, b, c->image, cur, b.dE, 1, s); }));
    const float* grad = b.dE;
    if (mode != SOBRC_MODE_L2) {
        SOBRC_TRY(timed(c, SOBRC_K_SOBOLEV, s, "k_sobolev",
                        [&] { return launch_sobolev(g, b, c->sw, cur, b.dE, b.gH1, flags, 1, s); }));
        grad = b.gH1;
    }
    if (g.topo)
        SOBRC_TRY(timed(c, SOBRC_K_TOPO, s, "k_topo",
                        [&] { return launch_topo(g, b, cur, grad, b.dE, flags, s); }));
    SOBRC_TRY(timed(c, SOBRC_K_FLIP, s, "k_flip",
                    [&] { return launch_flip(g, b, c->image, cur, grad, b.dE, flags, s); }));
    SOBRC_TRY(timed(c, SOBRC_K_COUNT, s, "k_count", [&] { return launch_count(g, b, cur, 1, 0, s); }));
    SOBRC_TRY(timed(c, SOBRC_K_SCAN, s, "k_scan",
                    [&] { return launch_scan(g, b, cur, nxt, 0, tol, d_nflips, flags, s); }));
    SOBRC_TRY(timed(c, SOBRC_K_WRITE, s, "k_write",
                    [&] { return launch_write(g, b, c->image, cur, nxt, grad, b.dE, flags, 0, s); }));
    c->cur = nxt;
    return SOBRC_OK;
}

void drop_graphs(sobrc_ctx* c)
{
    for (auto& row : c->gexec)
        for (auto& e : row)
            if (e) {
                (void)hipGraphExecDestroy(e);
                e = nullptr;
            }
}

// Instantiate (once per start parity, mode and tolerance) a graph holding two
// consecutive iterations; run() replays it.  Captured on a private stream.
int32_t pair_graph(sobrc_ctx* c, int mode, float tol, hipGraphExec_t* out)
{
    int par = c->cur;
    hipGraphExec_t& e = c->gexec[par][mode];
    if (e && c->gtol[par][mode] == tol) {
        *out = e;
        return SOBRC_OK;
    }
    if (e) {
        (void)hipGraphExecDestroy(e);
        e = nullptr;
    }
    if (!c->cap_stream)
        SOBRC_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    bool prof = c->prof;
    c->prof = false;
    hipGraph_t graph = nullptr;
    SOBRC_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    int32_t r1 = launch_step(c, mode, nullptr, tol, c->cap_stream);
    int32_t r2 = r1 == SOBRC_OK ? launch_step(c, mode, nullptr, tol, c->cap_stream) : r1;
    hipError_t ec = hipStreamEndCapture(c->cap_stream, &graph);
    c->prof = prof;
    c->cur = par;  // capture only recorded the launches
    if (r2 != SOBRC_OK) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return r2;
    }
    if (ec != hipSuccess)
        return dev_fail(ec, "hipStreamEndCapture");
    hipError_t ei = hipGraphInstantiate(&e, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        e = nullptr;
        return dev_fail(ei, "hipGraphInstantiate");
    }
    c->gtol[par][mode] = tol;
    *out = e;
    return SOBRC_OK;
}

}  // namespace

extern "C" {

const char* last_error(void) { return g_err; }

int32_t workspace_size(const sobrc_params* params, size_t* bytes)
{
    SOBRC_TRY(validate(params));
    if (!bytes)
        return fail(SOBRC_EINVAL, "bytes is NULL");
    Geom g = make_geom(params);
    *bytes = make_layout(g, params, params->max_particles).total;
    return SOBRC_OK;
}

int32_t ctx_create(const sobrc_params* params, void* d_workspace, size_t bytes, sobrc_ctx** out)
{
    SOBRC_TRY(validate(params));
    if (!out)
        return fail(SOBRC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d_workspace)
        return fail(SOBRC_EINVAL, "workspace is NULL");
    if (((uintptr_t)d_workspace & 255u) != 0)
        return fail(SOBRC_EINVAL, "workspace must be 256-byte aligned");
    Geom g = make_geom(params);
    if (g.T > kMaxT)
        return fail(SOBRC_EINVAL, "kernel support too large");
    Layout L = make_layout(g, params, params->max_particles);
    if (bytes < L.total)
        return fail(SOBRC_EINVAL, "workspace too small: %zu < %zu bytes", bytes, L.total);
    sobrc_ctx* c = new (std::nothrow) sobrc_ctx;
    if (!c)
        return fail(SOBRC_EINVAL, "out of host memory");
    c->p = *params;
    c->g = g;
    c->L = L;
    c->b = carve(L, (char*)d_workspace, params->max_particles);
    c->psf = make_psf(params->psf_sigma);
    *out = c;
    return SOBRC_OK;
}

int32_t ctx_destroy(sobrc_ctx* ctx)
{
    if (!ctx)
        return fail(SOBRC_EINVAL, "ctx is NULL");
    if (ctx->batch)
        return fail(SOBRC_ESTATE, "context is in a batch: remove it (batch_set) first");
    for (hipEvent_t e : ctx->ev)
        (void)hipEventDestroy(e);
    drop_graphs(ctx);
    if (ctx->cap_stream)
        (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    return SOBRC_OK;
}

int32_t init_labels(sobrc_ctx* c, const void* d_image, const int32_t* d_labels, void* stream)
{
    if (!c)
        return fail(SOBRC_EINVAL, "ctx is NULL");
    if (c->batch)
        return fail(SOBRC_ESTATE, "context is in a batch: remove it (batch_set) first");
    if (!d_image || !d_labels)
        return fail(SOBRC_EINVAL, "image and labels must be device pointers");
    hipStream_t s = (hipStream_t)stream;
    c->initialized = false;
    c->seen_err = 0;
    drop_graphs(c);  // graphs hold the image pointer and the intensity scale
    c->image = d_image;
    Geom& g = c->g;
    const Bufs& b = c->b;
    // state block and statistics start cleared; every tile is scanned once
    SOBRC_HIP(hipMemsetAsync(b.ds, 0, sizeof(DevState), s), "hipMemsetAsync");
    SOBRC_HIP(hipMemsetAsync(b.st_n, 0, (size_t)c->p.max_labels * 8, s), "hipMemsetAsync");
    SOBRC_HIP(hipMemsetAsync(b.st_s1, 0, (size_t)c->p.max_labels * 8, s), "hipMemsetAsync");
    SOBRC_HIP(hipMemsetAsync(b.dirty, 0, (size_t)g.ntiles * 4, s), "hipMemsetAsync");
    SOBRC_HIP(hipMemsetAsync(b.fstamp, 0, (size_t)g.nx * g.ny * g.nz * 4, s), "hipMemsetAsync");
    SOBRC_HIP(hipMemsetAsync(b.part_cnt, 0, (size_t)g.ge * 4, s), "hipMemsetAsync");
    SOBRC_HIP(hipMemsetAsync(b.part_act, 0, (size_t)g.ge * 4, s), "hipMemsetAsync");
    if (g.topo) {
        const size_t nvox = (size_t)g.nx * g.ny * g.nz;
        SOBRC_HIP(hipMemsetAsync(b.pmap, 0xFF, nvox * 8, s), "hipMemsetAsync");
        SOBRC_HIP(hipMemsetAsync(b.tmark, 0, (size_t)g.ntiles * 4, s), "hipMemsetAsync");
    }
    SOBRC_TRY(upload_tables(g, c->p.E, c->p.eps, b.W, &c->sw, s));
    SOBRC_HIP(launch_init_labels(g, b, d_labels, d_image, s), "k_init_labels");
    DevState h;
    SOBRC_TRY(read_state(c, &h, s));
    if (h.err & kErrLabel)
        return fail(SOBRC_EINVAL, "label outside [0, %d)", c->p.max_labels);
    // fixed-point scale of fp32 intensity sums: |sum| < 2^62 over the whole image
    if (!g.img_u16) {
        float mx;
        memcpy(&mx, &h.maxbits, 4);
        if (!isfinite(mx))
            return fail(SOBRC_EINVAL, "image contains non-finite values");
        long long nvox = (long long)g.nx * g.ny * g.nz;
        double lim = ldexp(1.0, 62) / ((double)nvox * (mx > 0 ? (double)mx : 1.0));
        int s2 = (int)floor(log2(lim));
        if (s2 > 60)
            s2 = 60;
        if (s2 < -60)
            s2 = -60;
        g.fx_scale = ldexp(1.0, s2);
        g.fx_inv = ldexp(1.0, -s2);
    }
    SOBRC_HIP(launch_stats_init(g, b, d_image, s), "k_stats_init");
    if (g.psf)
        SOBRC_HIP(launch_deconv_init(g, b, c->psf, s), "k_psf_pass");
    SOBRC_HIP(launch_count(g, b, 0, 0, 1, s), "k_count");
    SOBRC_HIP(launch_scan(g, b, 0, 0, 1, 0.f, nullptr, 0, s), "k_scan");
    SOBRC_HIP(launch_write(g, b, d_image, 0, 0, nullptr, nullptr, 0, 1, s), "k_write");
    SOBRC_TRY(read_state(c, &h, s));
    if (h.err & kErrCapacity)
        return fail(SOBRC_ECAPACITY, "initial particle set needs %u entries > max_particles %lld", h.need,
                    (long long)c->p.max_particles);
    c->cur = 0;
    c->initialized = true;
    return SOBRC_OK;
}

int32_t compute_l2_diff(sobrc_ctx* c, float* d_dE_l2, void* stream)
{
    if (!c)
        return fail(SOBRC_EINVAL, "ctx is NULL");
    if (!c->initialized)
        return fail(SOBRC_ESTATE, "compute_l2_diff before init_labels");
    if (!d_dE_l2)
        return fail(SOBRC_EINVAL, "output is NULL");
    if (c->seen_err & kErrCapacity)
        return fail(SOBRC_ECAPACITY, "a step overflowed the particle capacity: init_labels first");
    hipStream_t s = (hipStream_t)stream;
    if (c->g.psf)
        SOBRC_TRY(timed(c, SOBRC_K_DECONV, s, "k_deconv",
                        [&] { return launch_deconv(c->g, c->b, c->psf, c->image, s); }));
    return timed(c, SOBRC_K_L2DIFF, s, "k_l2diff",
                 [&] { return launch_l2diff(c->g, c->b, c->image, c->cur, d_dE_l2, 0, s); });
}

int32_t sobolev_smooth(sobrc_ctx* c, const float* d_in, float* d_out, void* stream)
{
    if (!c)
        return fail(SOBRC_EINVAL, "ctx is NULL");
    if (!c->initialized)
        return fail(SOBRC_ESTATE, "sobolev_smooth before init_labels");
    if (!d_in || !d_out)
        return fail(SOBRC_EINVAL, "input and output must be device pointers");
    if (d_in == d_out)
        return fail(SOBRC_EINVAL, "input and output must be distinct buffers (Jacobi update)");
    if (c->seen_err & kErrCapacity)
        return fail(SOBRC_ECAPACITY, "a step overflowed the particle capacity: init_labels first");
    hipStream_t s = (hipStream_t)stream;
    // the brick kernels read the L2 gradients by pixel
    SOBRC_HIP(launch_dense_put(c->g, c->b, c->cur, d_in, s), "k_dense_put");
    return timed(c, SOBRC_K_SOBOLEV, s, "k_sobolev",
                 [&] { return launch_sobolev(c->g, c->b, c->sw, c->cur, d_in, d_out, 0, 1, s); });
}

int32_t step(sobrc_ctx* c, int32_t mode, int32_t* d_nflips, void* stream)
{
    if (!c)
        return fail(SOBRC_EINVAL, "ctx is NULL");
    if (!c->initialized)
        return fail(SOBRC_ESTATE, "step before init_labels");
    if (c->batch)
        return fail(SOBRC_ESTATE, "context is in a batch: step the batch");
    if (mode != SOBRC_MODE_SOBOLEV && mode != SOBRC_MODE_L2 && mode != SOBRC_MODE_AUTO)
        return fail(SOBRC_EINVAL, "mode must be SOBRC_MODE_SOBOLEV, SOBRC_MODE_L2 or SOBRC_MODE_AUTO");
    return launch_step(c, mode, d_nflips, 0.f, (hipStream_t)stream);
}

int32_t step_with_gradient(sobrc_ctx* c, const float* d_grad, int32_t* d_nflips, void* stream)
{
    if (!c)
        return fail(SOBRC_EINVAL, "ctx is NULL");
    if (!c->initialized)
        return fail(SOBRC_ESTATE, "step_with_gradient before init_labels");
    if (c->batch)
        return fail(SOBRC_ESTATE, "context is in a batch: step the batch");
    if (!d_grad)
        return fail(SOBRC_EINVAL, "gradient must be a device pointer");
    hipStream_t s = (hipStream_t)stream;
    const int cur = c->cur, nxt = 1 - cur;
    const Geom& g = c->g;
    const Bufs& b = c->b;
    if (g.topo)
        SOBRC_TRY(timed(c, SOBRC_K_TOPO, s, "k_topo",
                        [&] { return launch_topo(g, b, cur, d_grad, d_grad, kGate, s); }));
    SOBRC_TRY(timed(c, SOBRC_K_FLIP, s, "k_flip",
                    [&] { return launch_flip(g, b, c->image, cur, d_grad, d_grad, kGate, s); }));
    SOBRC_TRY(timed(c, SOBRC_K_COUNT, s, "k_count", [&] { return launch_count(g, b, cur, 1, 0, s); }));
    SOBRC_TRY(timed(c, SOBRC_K_SCAN, s, "k_scan",
                    [&] { return launch_scan(g, b, cur, nxt, 0, 0.f, d_nflips, kGate, s); }));
    SOBRC_TRY(timed(c, SOBRC_K_WRITE, s, "k_write",
                    [&] { return launch_write(g, b, c->image, cur, nxt, d_grad, d_grad, kGate, 0, s); }));
    c->cur = nxt;
    return SOBRC_OK;
}

int32_t run(sobrc_ctx* c, int32_t max_iters, double flip_tol, int32_t mode, int32_t* h_iters_done, void* stream)
{
    if (!c)
        return fail(SOBRC_EINVAL, "ctx is NULL");
    if (!c->initialized)
        return fail(SOBRC_ESTATE, "run before init_labels");
    if (c->batch)
        return fail(SOBRC_ESTATE, "context is in a batch: run the batch");
    if (mode != SOBRC_MODE_SOBOLEV && mode != SOBRC_MODE_L2 && mode != SOBRC_MODE_AUTO)
        return fail(SOBRC_EINVAL, "mode must be SOBRC_MODE_SOBOLEV, SOBRC_MODE_L2 or SOBRC_MODE_AUTO");
    if (max_iters < 0 || !(flip_tol >= 0.0))
        return fail(SOBRC_EINVAL, "max_iters must be >= 0 and flip_tol >= 0");
    hipStream_t s = (hipStream_t)stream;
    DevState h;
    SOBRC_TRY(read_state(c, &h, s));
    SOBRC_TRY(status_of(h));
    unsigned it0 = h.iters;
    // a previous run may have stopped on its tolerance: start afresh
    SOBRC_HIP(hipMemsetAsync(&c->b.ds->converged, 0, sizeof(unsigned), s), "hipMemsetAsync");
    int t = 0;
    if (!c->prof && max_iters >= 2) {
        hipGraphExec_t e = nullptr;
        SOBRC_TRY(pair_graph(c, mode, (float)flip_tol, &e));
        for (; t + 2 <= max_iters; t += 2)
            SOBRC_HIP(hipGraphLaunch(e, s), "hipGraphLaunch");
    }
    for (; t < max_iters; ++t)
        SOBRC_TRY(launch_step(c, mode, nullptr, (float)flip_tol, s));
    SOBRC_TRY(read_state(c, &h, s));
    // Steps after a tolerance stop were no-ops: the state sits at the parity
    // of the completed iterations (after a capacity roll-back both buffers
    // hold it).  Clear the stop so that later step() calls proceed.
    c->cur = (int)(h.iters & 1u);
    SOBRC_HIP(hipMemsetAsync(&c->b.ds->converged, 0, sizeof(unsigned), s), "hipMemsetAsync");
    if (h_iters_done)
        *h_iters_done = (int32_t)(h.iters - it0);
    return status_of(h);
}

int32_t ctx_sync(sobrc_ctx* c, void* stream)
{
    if (!c)
        return fail(SOBRC_EINVAL, "ctx is NULL");
    if (!c->initialized)
        return fail(SOBRC_ESTATE, "ctx_sync before init_labels");
    DevState h;
    SOBRC_TRY(read_state(c, &h, (hipStream_t)stream));
    c->cur = (int)(h.iters & 1u);
    return status_of(h);
}

int32_t get_particles(sobrc_ctx* c, int64_t* h_n, int32_t* d_lin, int32_t* d_a, int32_t* d_b, void* stream)
{
    if (!c || !h_n)
        return fail(SOBRC_EINVAL, "ctx and h_n must be non-NULL");
    if (!c->initialized)
        return fail(SOBRC_ESTATE, "get_particles before init_labels");
    hipStream_t s = (hipStream_t)stream;
    DevState h;
    SOBRC_TRY(read_state(c, &h, s));
    *h_n = h.n[c->cur];
    if (d_lin || d_a || d_b)
        SOBRC_HIP(launch_unpack(c->g, c->b, c->cur, d_lin, d_a, d_b, s), "k_unpack");
    return status_of(h);
}

int32_t get_labels(sobrc_ctx* c, int32_t* d_labels, void* stream)
{
    if (!c || !d_labels)
        return fail(SOBRC_EINVAL, "ctx and labels must be non-NULL");
    if (!c->initialized)
        return fail(SOBRC_ESTATE, "get_labels before init_labels");
    SOBRC_HIP(launch_labels_out(c->g, c->b, d_labels, (hipStream_t)stream), "k_labels_out");
    return SOBRC_OK;
}

int32_t get_labels_u16(sobrc_ctx* c, uint16_t* labels, void* stream)
{
    if (!c || !labels)
        return fail(SOBRC_EINVAL, "ctx and labels must be non-NULL");
    if (!c->initialized)
        return fail(SOBRC_ESTATE, "get_labels_u16 before init_labels");
    const size_t nvox = (size_t)c->g.nx * c->g.ny * c->g.nz;
    SOBRC_HIP(hipMemcpyAsync(labels, c->b.lab, nvox * 2, hipMemcpyDefault, (hipStream_t)stream), "hipMemcpyAsync");
    return SOBRC_OK;
}

int32_t get_region_stats(sobrc_ctx* c, int64_t* h_count, double* h_sum, void* stream)
{
    if (!c || !h_count)
        return fail(SOBRC_EINVAL, "ctx and h_count must be non-NULL");
    if (!c->initialized)
        return fail(SOBRC_ESTATE, "get_region_stats before init_labels");
    hipStream_t s = (hipStream_t)stream;
    int M = c->p.max_labels;
    std::vector<long long> n(M), s1(M);
    SOBRC_HIP(hipMemcpyAsync(n.data(), c->b.st_n, 8 * (size_t)M, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    SOBRC_HIP(hipMemcpyAsync(s1.data(), c->b.st_s1, 8 * (size_t)M, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    SOBRC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    for (int l = 0; l < M; ++l) {
        h_count[l] = n[l];
        if (h_sum)
            h_sum[l] = (double)s1[l] * c->g.fx_inv;
    }
    return SOBRC_OK;
}

int32_t get_history(sobrc_ctx* c, int32_t cap, int32_t* h_n, int32_t* h_flips, int32_t* h_reversals,
                    int32_t* h_len, void* stream)
{
    if (!c || !h_len || cap < 0 || (cap > 0 && (!h_n || !h_flips)))
        return fail(SOBRC_EINVAL, "bad arguments to get_history");
    if (!c->initialized)
        return fail(SOBRC_ESTATE, "get_history before init_labels");
    hipStream_t s = (hipStream_t)stream;
    DevState h;
    SOBRC_TRY(read_state(c, &h, s));
    std::vector<unsigned> hist(3 * kHist);
    SOBRC_HIP(hipMemcpyAsync(hist.data(), c->b.hist, 12 * (size_t)kHist, hipMemcpyDeviceToHost, s),
              "hipMemcpyAsync");
    SOBRC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    unsigned avail = h.iters < (unsigned)kHist ? h.iters : (unsigned)kHist;
    unsigned take = (unsigned)cap < avail ? (unsigned)cap : avail;
    for (unsigned k = 0; k < take; ++k) {
        unsigned it = h.iters - take + k;
        h_n[k] = (int32_t)hist[it % kHist];
        h_flips[k] = (int32_t)hist[kHist + it % kHist];
        if (h_reversals)
            h_reversals[k] = (int32_t)hist[2 * kHist + it % kHist];
    }
    *h_len = (int32_t)take;
    return SOBRC_OK;
}

int32_t get_gradient_mode(sobrc_ctx* c, int32_t* h_switch_iter, void* stream)
{
    if (!c || !h_switch_iter)
        return fail(SOBRC_EINVAL, "ctx and h_switch_iter must be non-NULL");
    if (!c->initialized)
        return fail(SOBRC_ESTATE, "get_gradient_mode before init_labels");
    DevState h;
    SOBRC_TRY(read_state(c, &h, (hipStream_t)stream));
    *h_switch_iter = h.switch_it == 0 ? -1 : (int32_t)(h.switch_it - 1);
    return SOBRC_OK;
}

}  // extern "C"

namespace {
// Tile shapes that parameters admit (the others are not tried by the autotuner).
bool tile_admitted(const sobrc_params& q, int k)
{
    return k == SOBRC_TILE_DEFAULT || (q.topo == SOBRC_TOPO_OFF && (k == SOBRC_TILE_WIDE || q.ndim == 2));
}
constexpr int kTileShapes = 3;
}  // namespace

extern "C" {

int32_t tile_autotune_workspace_size(const sobrc_params* params, size_t* bytes)
{
    if (!params || !bytes)
        return fail(SOBRC_EINVAL, "params and bytes must be non-NULL");
    size_t most = 0;
    for (int k = 0; k < kTileShapes; ++k) {
        sobrc_params q = *params;
        q.tile = k;
        size_t n = 0;
        if (!tile_admitted(q, k))
            continue;  // not tried
        SOBRC_TRY(workspace_size(&q, &n));
        most = n > most ? n : most;
    }
    *bytes = most;
    return SOBRC_OK;
}

int32_t tile_autotune(const sobrc_params* params, const void* d_image, const int32_t* d_labels, int32_t iters,
                      int32_t mode, void* d_workspace, size_t bytes, int32_t* h_tile, double* h_ms, void* stream)
{
    if (!params || !d_image || !d_labels || !d_workspace || !h_tile || !h_ms)
        return fail(SOBRC_EINVAL, "NULL argument");
    if (iters < 1 || iters > 1000)
        return fail(SOBRC_EINVAL, "iters must lie in [1, 1000] (got %d)", iters);
    if (mode != SOBRC_MODE_SOBOLEV && mode != SOBRC_MODE_L2 && mode != SOBRC_MODE_AUTO)
        return fail(SOBRC_EINVAL, "mode must be SOBRC_MODE_SOBOLEV, SOBRC_MODE_L2 or SOBRC_MODE_AUTO");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SOBRC_HIP(hipEventCreate(&e0), "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(SOBRC_EDEVICE, "hipEventCreate");
    }
    int32_t rc = SOBRC_OK;
    for (int k = 0; k < kTileShapes; ++k)
        h_ms[k] = -1.0;
    // two rounds, shapes alternating; each shape keeps its faster round
    for (int round = 0; round < 2 && rc == SOBRC_OK; ++round)
        for (int k = 0; k < kTileShapes && rc == SOBRC_OK; ++k) {
            sobrc_params q = *params;
            q.tile = k;
            if (!tile_admitted(q, k))
                continue;
            sobrc_ctx* c = nullptr;
            rc = ctx_create(&q, d_workspace, bytes, &c);
            if (rc != SOBRC_OK)
                break;
            int32_t done = 0;
            // warm-up (graph capture), then the timed iterations from the same start
            rc = init_labels(c, d_image, d_labels, stream);
            if (rc == SOBRC_OK)
                rc = run(c, iters < 2 ? iters : 2, 0.0, mode, &done, stream);
            if (rc == SOBRC_OK)
                rc = init_labels(c, d_image, d_labels, stream);
            if (rc == SOBRC_OK && (hipEventRecord(e0, s) != hipSuccess))
                rc = fail(SOBRC_EDEVICE, "hipEventRecord");
            if (rc == SOBRC_OK)
                rc = run(c, iters, 0.0, mode, &done, stream);
            if (rc == SOBRC_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                rc = fail(SOBRC_EDEVICE, "hipEventRecord");
            float ms = 0.f;
            if (rc == SOBRC_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                rc = fail(SOBRC_EDEVICE, "hipEventElapsedTime");
            const int32_t dr = ctx_destroy(c);
            rc = rc == SOBRC_OK ? dr : rc;
            if (rc != SOBRC_OK)
                break;
            const double per = (double)ms / (double)(done > 0 ? done : 1);
            h_ms[k] = h_ms[k] < 0.0 || per < h_ms[k] ? per : h_ms[k];
        }
    // the fastest other shape if it beats the default by at least 1.5 % (the
    // trials' timing noise reaches about 1 %), else the default
    int best = SOBRC_TILE_DEFAULT, alt = -1;
    for (int k = 1; k < kTileShapes; ++k)
        if (h_ms[k] >= 0.0 && (alt < 0 || h_ms[k] < h_ms[alt]))
            alt = k;
    if (alt >= 0 && h_ms[alt] < 0.985 * h_ms[SOBRC_TILE_DEFAULT])
        best = alt;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == SOBRC_OK)
        *h_tile = best;
    return rc;
}

}  // extern "C"

// ------------------------------------------------------------------ batches

namespace {

struct BLayout {
    size_t desc, par, off, state, tpre, total;
};

BLayout batch_layout(int nslot)
{
    BLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = align256(o + bytes);
        return r;
    };
    L.desc = take(sizeof(ImgDesc) * (size_t)nslot);
    L.par = take(4 * (size_t)nslot);
    L.off = take(4 * (size_t)kNumPh * (size_t)(nslot + 1));
    L.state = take(16 * (size_t)nslot);
    L.tpre = take(4 * (size_t)(nslot + 1));
    L.total = o;
    return L;
}

// A slot's geometry under the batch's launch shape.  Only block counts
// change, and only downwards, so every per-block buffer of the context's
// workspace still fits: gp (particle kernels) <= the context's, ranges of at
// most kBlock tiles no smaller than the context's (ge <= the context's), any
// Sobolev block count.
Geom slot_geom(const sobrc_batch* B, const sobrc_ctx* c)
{
    Geom g = c->g;
    if (B->part_chunk > 0) {
        long long gp = ((long long)c->p.max_particles + B->part_chunk - 1) / B->part_chunk;
        gp = gp < 8 ? gp : (gp + 7) / 8 * 8;
        if (gp < 1)
            gp = 1;
        if (gp < g.gp)
            g.gp = (int)gp;
    }
    if (B->lg_range > g.lgRe) {
        int lg = B->lg_range;
        while ((1 << lg) > kBlock)
            --lg;
        g.lgRe = lg;
        g.Re = 1 << lg;
        g.ge = (g.ntiles + g.Re - 1) >> lg;
        g.dlistm = g.ge <= kMaxGrid && g.Re >= 8 ? 1 : 0;  // the list buffers are always there
    }
    if (B->sob_tiles > 0) {
        int sg = (g.ntiles + B->sob_tiles - 1) / B->sob_tiles;
        sg = (sg + 7) / 8 * 8;
        if (sg < g.sob_grid)
            g.sob_grid = sg;
    }
    return g;
}

// Item offsets of every phase from the slots' launch sizes.
void batch_offsets(sobrc_batch* B)
{
    const int n = B->nslot;
    B->off.assign((size_t)kNumPh * (n + 1), 0u);
    for (int ph = 0; ph < kNumPh; ++ph) {
        unsigned* o = B->off.data() + (size_t)ph * (n + 1);
        for (int i = 0; i < n; ++i) {
            const sobrc_ctx* c = B->slot[i];
            unsigned items = 0;
            if (c) {
                const Geom g = slot_geom(B, c);
                items = ph == kPhPart ? (unsigned)g.gp
                        : ph == kPhEmit ? (unsigned)g.ge
                        : ph == kPhSob  ? (unsigned)g.sob_grid
                        : ph == kPhList ? (g.dlistm ? (unsigned)std::min(g.ge, kBatchListItems) : 0u)
                                        : 1u;
            }
            unsigned end = o[i] + items;
            o[i + 1] = ph == kPhScan ? end : (end + 7u) / 8u * 8u;
        }
        B->totals[ph] = o[n];
    }
}

void batch_drop_graphs(sobrc_batch* B)
{
    for (auto& e : B->gexec)
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
}

int32_t batch_launch(sobrc_batch* B, int mode, float tol, hipStream_t s)
{
    BatchTab t{B->d_desc, B->d_par, B->d_off, B->d_tpre, B->nslot};
    const int l2 = mode == SOBRC_MODE_L2;
    const int flags = kGate | (mode == SOBRC_MODE_AUTO ? kAuto : 0);
    SOBRC_HIP(launch_batch_step(t, B->totals, B->g0, B->sw, l2, flags, tol, s), "batched step");
    return SOBRC_OK;
}

// Per-slot state words (iterations, stop, error bits, needed capacity), one
// gather kernel and one copy for the whole batch.  Synchronises.
int32_t batch_states(sobrc_batch* B, std::vector<uint4>& st, hipStream_t s)
{
    st.assign((size_t)B->nslot, make_uint4(0u, 0u, 0u, 0u));
    if (!B->has_class)
        return SOBRC_OK;
    BatchTab t{B->d_desc, B->d_par, B->d_off, B->d_tpre, B->nslot};
    SOBRC_HIP(launch_batch_gather(t, B->d_state, s), "kb_gather");
    SOBRC_HIP(hipMemcpyAsync(st.data(), B->d_state, st.size() * sizeof(uint4), hipMemcpyDeviceToHost, s),
              "hipMemcpyAsync");
    SOBRC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    return SOBRC_OK;
}

int32_t slot_status(const uint4& v)
{
    DevState h{};
    h.err = v.z;
    h.need = v.w;
    return status_of(h);
}

// Launch `iters` iterations of every live slot (graph replays of two
// batched steps, then single steps); clears the slots' tolerance stops first.
int32_t batch_enqueue(sobrc_batch* B, int32_t iters, float tol, int32_t mode, hipStream_t s)
{
    if (!B->has_class || iters <= 0)
        return SOBRC_OK;
    BatchTab t{B->d_desc, B->d_par, B->d_off, B->d_tpre, B->nslot};
    SOBRC_HIP(launch_batch_clear(t, s), "kb_clear");
    int k = 0;
    if (iters >= 2) {
        hipGraphExec_t& e = B->gexec[mode];
        if (e && B->gtol[mode] != tol) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
        if (!e) {
            if (!B->cap_stream)
                SOBRC_HIP(hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
            hipGraph_t graph = nullptr;
            SOBRC_HIP(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal),
                      "hipStreamBeginCapture");
            int32_t r1 = batch_launch(B, mode, tol, B->cap_stream);
            int32_t r2 = r1 == SOBRC_OK ? batch_launch(B, mode, tol, B->cap_stream) : r1;
            hipError_t ec = hipStreamEndCapture(B->cap_stream, &graph);
            if (r2 != SOBRC_OK) {
                if (graph)
                    (void)hipGraphDestroy(graph);
                return r2;
            }
            if (ec != hipSuccess)
                return dev_fail(ec, "hipStreamEndCapture");
            hipError_t ei = hipGraphInstantiate(&e, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ei != hipSuccess) {
                e = nullptr;
                return dev_fail(ei, "hipGraphInstantiate");
            }
            B->gtol[mode] = tol;
        }
        for (; k + 2 <= iters; k += 2)
            SOBRC_HIP(hipGraphLaunch(e, s), "hipGraphLaunch");
    }
    for (; k < iters; ++k)
        SOBRC_TRY(batch_launch(B, mode, tol, s));
    return SOBRC_OK;
}

}  // namespace

extern "C" {

int32_t batch_workspace_size(int32_t n_slots, size_t* bytes)
{
    if (n_slots < 1 || n_slots > 65536 || !bytes)
        return fail(SOBRC_EINVAL, "n_slots must be in [1, 65536] and bytes non-NULL");
    *bytes = batch_layout(n_slots).total;
    return SOBRC_OK;
}

int32_t batch_create(int32_t n_slots, void* d_workspace, size_t bytes, sobrc_batch** out)
{
    if (!out)
        return fail(SOBRC_EINVAL, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    SOBRC_TRY(batch_workspace_size(n_slots, &need));
    if (!d_workspace || ((uintptr_t)d_workspace & 255u) != 0)
        return fail(SOBRC_EINVAL, "workspace must be a 256-byte aligned device pointer");
    if (bytes < need)
        return fail(SOBRC_EINVAL, "workspace too small: %zu < %zu bytes", bytes, need);
    BLayout L = batch_layout(n_slots);
    sobrc_batch* B = new (std::nothrow) sobrc_batch;
    if (!B)
        return fail(SOBRC_EINVAL, "out of host memory");
    B->nslot = n_slots;
    B->ws = (char*)d_workspace;
    B->d_desc = (ImgDesc*)(B->ws + L.desc);
    B->d_par = (unsigned*)(B->ws + L.par);
    B->d_off = (unsigned*)(B->ws + L.off);
    B->d_state = (uint4*)(B->ws + L.state);
    B->d_tpre = (unsigned*)(B->ws + L.tpre);
    B->slot.assign((size_t)n_slots, nullptr);
    batch_offsets(B);
    std::vector<ImgDesc> empty((size_t)n_slots);
    memset(empty.data(), 0, empty.size() * sizeof(ImgDesc));
    hipError_t e = hipMemcpy(B->d_desc, empty.data(), empty.size() * sizeof(ImgDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(B->d_off, B->off.data(), B->off.size() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        delete B;
        return dev_fail(e, "hipMemcpy");
    }
    *out = B;
    return SOBRC_OK;
}

int32_t batch_destroy(sobrc_batch* B)
{
    if (!B)
        return fail(SOBRC_EINVAL, "batch is NULL");
    for (sobrc_ctx* c : B->slot)
        if (c)
            c->batch = nullptr;
    batch_drop_graphs(B);
    if (B->cap_stream)
        (void)hipStreamDestroy(B->cap_stream);
    delete B;
    return SOBRC_OK;
}

int32_t batch_set(sobrc_batch* B, int32_t slot, sobrc_ctx* c, void* stream)
{
    if (!B)
        return fail(SOBRC_EINVAL, "batch is NULL");
    if (slot < 0 || slot >= B->nslot)
        return fail(SOBRC_EINVAL, "slot %d outside [0, %d)", slot, B->nslot);
    hipStream_t s = (hipStream_t)stream;
    if (c) {
        if (!c->initialized)
            return fail(SOBRC_ESTATE, "context not initialised");
        if (c->g.topo || c->g.psf)
            return fail(SOBRC_EINVAL, "contexts with topological control or a PSF are not batched");
        if (c->batch && (c->batch != B || B->slot[slot] != c))
            return fail(SOBRC_ESTATE, "context is already in a batch slot");
        bool any = false;
        for (sobrc_ctx* o : B->slot)
            any = any || (o && o != B->slot[slot]);
        if (any || B->has_class) {
            const Geom& a = B->g0;
            const Geom& g = c->g;
            if (a.ndim != g.ndim || a.T != g.T || a.h != g.h || a.brick != g.brick || a.full != g.full ||
                a.wide != g.wide || a.sob_lds != g.sob_lds || memcmp(&B->sw, &c->sw, sizeof(SobW)) != 0)
                return fail(SOBRC_EINVAL, "batch slots must share ndim, E, eps and the tile shape");
        }
    }
    // leaving context: its host parity follows the device
    if (sobrc_ctx* o = B->slot[slot]) {
        DevState h;
        SOBRC_TRY(read_state(o, &h, s));
        o->cur = (int)(h.iters & 1u);
        o->batch = nullptr;
        B->slot[slot] = nullptr;
    }
    ImgDesc d;
    memset(&d, 0, sizeof d);
    if (c) {
        d.g = slot_geom(B, c);
        d.b = c->b;
        d.img = c->image;
        d.live = 1;
        if (!B->has_class) {
            B->g0 = c->g;
            B->sw = c->sw;
            B->has_class = true;
        }
        c->batch = B;
        B->slot[slot] = c;
    }
    batch_offsets(B);
    const unsigned par = c ? (unsigned)c->cur : 0u;
    SOBRC_HIP(hipMemcpyAsync(B->d_desc + slot, &d, sizeof d, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    SOBRC_HIP(hipMemcpyAsync(B->d_par + slot, &par, 4, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    SOBRC_HIP(hipMemcpyAsync(B->d_off, B->off.data(), B->off.size() * 4, hipMemcpyHostToDevice, s),
              "hipMemcpyAsync");
    SOBRC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");  // host copies above are on the stack
    return SOBRC_OK;
}

int32_t batch_step(sobrc_batch* B, int32_t mode, void* stream)
{
    if (!B)
        return fail(SOBRC_EINVAL, "batch is NULL");
    if (mode != SOBRC_MODE_SOBOLEV && mode != SOBRC_MODE_L2 && mode != SOBRC_MODE_AUTO)
        return fail(SOBRC_EINVAL, "mode must be SOBRC_MODE_SOBOLEV, SOBRC_MODE_L2 or SOBRC_MODE_AUTO");
    if (!B->has_class)
        return SOBRC_OK;
    SOBRC_TRY(batch_launch(B, mode, 0.f, (hipStream_t)stream));
    for (sobrc_ctx* c : B->slot)
        if (c)
            c->cur ^= 1;  // as step(): the device may have stopped; batch_run / batch_set re-derive it
    return SOBRC_OK;
}

int32_t batch_launch_iters(sobrc_batch* B, int32_t iters, double flip_tol, int32_t mode, void* stream)
{
    if (!B)
        return fail(SOBRC_EINVAL, "batch is NULL");
    if (mode != SOBRC_MODE_SOBOLEV && mode != SOBRC_MODE_L2 && mode != SOBRC_MODE_AUTO)
        return fail(SOBRC_EINVAL, "mode must be SOBRC_MODE_SOBOLEV, SOBRC_MODE_L2 or SOBRC_MODE_AUTO");
    if (iters < 0 || !(flip_tol >= 0.0))
        return fail(SOBRC_EINVAL, "iters must be >= 0 and flip_tol >= 0");
    return batch_enqueue(B, iters, (float)flip_tol, mode, (hipStream_t)stream);
}

int32_t batch_collect(sobrc_batch* B, int32_t* h_iters, int32_t* h_stopped, void* stream)
{
    if (!B)
        return fail(SOBRC_EINVAL, "batch is NULL");
    hipStream_t s = (hipStream_t)stream;
    std::vector<uint4> st;
    SOBRC_TRY(batch_states(B, st, s));
    int32_t status = SOBRC_OK;
    for (int i = 0; i < B->nslot; ++i) {
        const bool live = B->slot[i] != nullptr;
        const int32_t si = live ? slot_status(st[i]) : SOBRC_OK;
        if (live) {
            B->slot[i]->cur = (int)(st[i].x & 1u);
            B->slot[i]->seen_err |= st[i].z;
        }
        if (h_iters)
            h_iters[i] = live ? (int32_t)st[i].x : 0;
        if (h_stopped)
            h_stopped[i] = si != SOBRC_OK ? si : (live && st[i].y ? 1 : 0);
        if (status == SOBRC_OK)
            status = si;
    }
    if (B->has_class) {
        BatchTab t{B->d_desc, B->d_par, B->d_off, B->d_tpre, B->nslot};
        SOBRC_HIP(launch_batch_clear(t, s), "kb_clear");
    }
    return status;
}

int32_t batch_run(sobrc_batch* B, int32_t max_iters, double flip_tol, int32_t mode, int32_t* h_iters_done,
                  void* stream)
{
    if (!B)
        return fail(SOBRC_EINVAL, "batch is NULL");
    if (mode != SOBRC_MODE_SOBOLEV && mode != SOBRC_MODE_L2 && mode != SOBRC_MODE_AUTO)
        return fail(SOBRC_EINVAL, "mode must be SOBRC_MODE_SOBOLEV, SOBRC_MODE_L2 or SOBRC_MODE_AUTO");
    if (max_iters < 0 || !(flip_tol >= 0.0))
        return fail(SOBRC_EINVAL, "max_iters must be >= 0 and flip_tol >= 0");
    hipStream_t s = (hipStream_t)stream;
    const int n = B->nslot;
    std::vector<uint4> st0;
    SOBRC_TRY(batch_states(B, st0, s));
    for (int i = 0; i < n; ++i)
        if (B->slot[i])
            SOBRC_TRY(slot_status(st0[i]));
    SOBRC_TRY(batch_enqueue(B, max_iters, (float)flip_tol, mode, s));
    std::vector<int32_t> it1((size_t)n, 0);
    int32_t status = batch_collect(B, it1.data(), nullptr, stream);
    if (h_iters_done)
        for (int i = 0; i < n; ++i)
            h_iters_done[i] = B->slot[i] ? it1[i] - (int32_t)st0[i].x : 0;
    return status;
}

int32_t batch_set_shape(sobrc_batch* B, int32_t part_chunk, int32_t lg_range, int32_t sob_tiles, void* stream)
{
    if (!B)
        return fail(SOBRC_EINVAL, "batch is NULL");
    if (part_chunk < 0 || lg_range < 0 || lg_range > 8 || sob_tiles < 0)
        return fail(SOBRC_EINVAL, "bad launch shape");
    hipStream_t s = (hipStream_t)stream;
    B->part_chunk = part_chunk;
    B->lg_range = lg_range;
    B->sob_tiles = sob_tiles;
    batch_offsets(B);
    std::vector<ImgDesc> d((size_t)B->nslot);
    memset(d.data(), 0, d.size() * sizeof(ImgDesc));
    for (int i = 0; i < B->nslot; ++i)
        if (sobrc_ctx* c = B->slot[i]) {
            d[i].g = slot_geom(B, c);
            d[i].b = c->b;
            d[i].img = c->image;
            d[i].live = 1;
        }
    SOBRC_HIP(hipMemcpyAsync(B->d_desc, d.data(), d.size() * sizeof(ImgDesc), hipMemcpyHostToDevice, s),
              "hipMemcpyAsync");
    SOBRC_HIP(hipMemcpyAsync(B->d_off, B->off.data(), B->off.size() * 4, hipMemcpyHostToDevice, s),
              "hipMemcpyAsync");
    SOBRC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    batch_drop_graphs(B);  // grid sizes follow the item counts
    return SOBRC_OK;
}

int32_t batch_autotune(sobrc_batch* B, int32_t mode, int32_t iters_per_trial, int32_t* h_shape,
                       int32_t* h_iters_done, void* stream)
{
    if (!B || iters_per_trial < 1)
        return fail(SOBRC_EINVAL, "batch is NULL or iters_per_trial < 1");
    if (mode != SOBRC_MODE_SOBOLEV && mode != SOBRC_MODE_L2 && mode != SOBRC_MODE_AUTO)
        return fail(SOBRC_EINVAL, "mode must be SOBRC_MODE_SOBOLEV, SOBRC_MODE_L2 or SOBRC_MODE_AUTO");
    hipStream_t s = (hipStream_t)stream;
    // candidates: the contexts' own shape, then coarser items
    const int cand[][3] = {{0, 0, 0},     {1024, 3, 4},  {1024, 5, 8},  {2048, 5, 16}, {4096, 6, 16},
                           {4096, 7, 32}, {8192, 7, 64}, {2048, 4, 8},  {8192, 8, 32}};
    const int ncand = (int)(sizeof cand / sizeof cand[0]);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SOBRC_HIP(hipEventCreate(&e0), "hipEventCreate");
    SOBRC_HIP(hipEventCreate(&e1), "hipEventCreate");
    int best = 0, done = 0;
    float best_ms = 0.f;
    int32_t rc = SOBRC_OK;
    for (int k = 0; k < ncand && rc == SOBRC_OK; ++k) {
        rc = batch_set_shape(B, cand[k][0], cand[k][1], cand[k][2], stream);
        if (rc != SOBRC_OK)
            break;
        // one untimed iteration settles the new shape, then the timed trial
        rc = batch_launch(B, mode, 0.f, s);
        for (int t = 0; t < iters_per_trial && rc == SOBRC_OK; ++t) {
            if (t == 0 && hipEventRecord(e0, s) != hipSuccess)
                rc = fail(SOBRC_EDEVICE, "hipEventRecord");
            if (rc == SOBRC_OK)
                rc = batch_launch(B, mode, 0.f, s);
        }
        if (rc != SOBRC_OK)
            break;
        float ms = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(SOBRC_EDEVICE, "event timing");
            break;
        }
        done += iters_per_trial + 1;
        if (k == 0 || ms < best_ms) {
            best_ms = ms;
            best = k;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SOBRC_OK)
        return rc;
    SOBRC_TRY(batch_set_shape(B, cand[best][0], cand[best][1], cand[best][2], stream));
    for (int i = 0; i < B->nslot; ++i)
        if (sobrc_ctx* c = B->slot[i]) {
            DevState h;
            SOBRC_TRY(read_state(c, &h, s));
            c->cur = (int)(h.iters & 1u);
        }
    if (h_shape) {
        h_shape[0] = cand[best][0];
        h_shape[1] = cand[best][1];
        h_shape[2] = cand[best][2];
    }
    if (h_iters_done)
        *h_iters_done = done;
    return SOBRC_OK;
}

}  // extern "C"

// ---------------------------------------------- stateless Eq. (6) on given particles

namespace {
struct PLayout {
    size_t ts, act, tcnt, fill, rec, vin, vout, origin, W, ds, total;
};
PLayout make_playout(const Geom& g, long long n)
{
    PLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = align256(o + bytes);
        return r;
    };
    long long m = n > 0 ? n : 1;
    L.ts = take((size_t)(g.ntiles + 1) * 4);
    L.act = take((size_t)g.ntiles * 4);
    L.tcnt = take((size_t)g.ntiles * 4);
    L.fill = take((size_t)g.ntiles * 4);
    L.rec = take((size_t)m * 8);
    L.vin = take((size_t)m * 4);
    L.vout = take((size_t)m * 4);
    L.origin = take((size_t)m * 4);
    L.W = take((size_t)kMaxT * 4);
    L.ds = take(sizeof(DevState));
    L.total = o;
    return L;
}
}  // namespace

extern "C" {

int32_t sobolev_particles_workspace_size(const sobrc_params* params, int64_t n, size_t* bytes)
{
    sobrc_params q = *params;
    q.max_particles = 1;
    SOBRC_TRY(validate(&q));
    if (!bytes || n < 0 || n > 0x7fffffffLL)
        return fail(SOBRC_EINVAL, "bad particle count or NULL bytes");
    *bytes = make_playout(make_geom(params), n).total;
    return SOBRC_OK;
}

}  // extern "C"

namespace {

// Eq. (6) on caller-given particles with the scratch memory at d_ws
// (ws_bytes, 256-byte aligned): bins the particles by tile, runs the staged
// Sobolev kernel, writes d_out in input order.
int32_t smooth_particles_ws(const sobrc_params* params, int64_t n, const int32_t* d_lin, const int32_t* d_a,
                            const int32_t* d_b, const float* d_in, float* d_out, void* d_ws, size_t ws_bytes,
                            void* stream)
{
    if (!params)
        return fail(SOBRC_EINVAL, "params is NULL");
    sobrc_params q = *params;
    q.max_particles = 1;
    SOBRC_TRY(validate(&q));
    if (n < 0 || n > 0x7fffffffLL)
        return fail(SOBRC_EINVAL, "particle count out of range");
    if (n == 0)
        return SOBRC_OK;
    if (!d_lin || !d_a || !d_b || !d_in || !d_out || !d_ws)
        return fail(SOBRC_EINVAL, "NULL device pointer");
    if (((uintptr_t)d_ws & 255u) != 0)
        return fail(SOBRC_EINVAL, "workspace must be 256-byte aligned");
    Geom g = make_geom(params);
    if (g.T > kMaxT)
        return fail(SOBRC_EINVAL, "kernel support too large");
    PLayout L = make_playout(g, n);
    if (ws_bytes < L.total)
        return fail(SOBRC_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
    char* base = (char*)d_ws;
    Bufs b{};
    b.tstart[0] = b.tstart[1] = (unsigned*)(base + L.ts);
    b.active[0] = b.active[1] = (unsigned*)(base + L.act);
    b.tcnt = (unsigned*)(base + L.tcnt);
    b.rec[0] = b.rec[1] = (uint2*)(base + L.rec);
    b.dE = (float*)(base + L.vin);
    b.gH1 = (float*)(base + L.vout);
    b.W = (float*)(base + L.W);
    b.ds = (DevState*)(base + L.ds);
    b.cap = (unsigned)n;
    unsigned* fill = (unsigned*)(base + L.fill);
    unsigned* origin = (unsigned*)(base + L.origin);
    hipStream_t s = (hipStream_t)stream;
    SobW sw{};
    SOBRC_TRY(upload_tables(g, params->E, params->eps, b.W, &sw, s));
    static_assert(sizeof(DevState) % 4 == 0, "state block in words");
    SOBRC_HIP(launch_fill_u32((unsigned*)b.ds, 0u, sizeof(DevState) / 4, s), "k_fill_u32");
    SOBRC_HIP(launch_fill_u32(b.tcnt, 0u, (size_t)g.ntiles, s), "k_fill_u32");
    SOBRC_HIP(launch_fill_u32(fill, 0u, (size_t)g.ntiles, s), "k_fill_u32");
    SOBRC_HIP(launch_bin_count(g, b, n, d_lin, d_a, d_b, s), "k_bin_count");
    DevState h;
    SOBRC_HIP(hipMemcpyAsync(&h, b.ds, sizeof h, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    SOBRC_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (h.err & kErrInput)
        return fail(SOBRC_EINVAL, "particle outside the image or with a bad label pair");
    SOBRC_HIP(launch_bin_scan(g, b, s), "k_bin_scan");
    SOBRC_HIP(launch_bin_scatter(g, b, n, d_lin, d_a, d_b, d_in, fill, origin, s), "k_bin_scatter");
    SOBRC_HIP(launch_sobolev(g, b, sw, 0, b.dE, b.gH1, 0, 0, s), "k_sobolev");
    SOBRC_HIP(launch_unbin(b, n, origin, b.gH1, d_out, s), "k_unbin");
    return SOBRC_OK;
}

}  // namespace

extern "C" {

int32_t sobolev_smooth_particles(const sobrc_params* params, int64_t n, const int32_t* d_lin, const int32_t* d_a,
                                 const int32_t* d_b, const float* d_in, float* d_out, void* d_ws, size_t ws_bytes,
                                 void* stream)
{
    return smooth_particles_ws(params, n, d_lin, d_a, d_b, d_in, d_out, d_ws, ws_bytes, stream);
}

}  // extern "C"

// ------------------------------------------- stateless update without allocation
//
// Scratch memory of sobolev_smooth_particles_static: a file-scope device
// array, one copy per GPU for the life of the process.  Host code never
// passes the array's name to a kernel (in host code it is a stand-in, not a
// device address): each device's address comes from hipGetSymbolAddress,
// taken once per device with that device current.
static __device__ __align__(256) char scratch[SOBRC_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int32_t scratch_address(void** out)
{
    int dev = 0;
    SOBRC_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(SOBRC_EDEVICE, "device %d outside the %d devices the scratch table holds", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        SOBRC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
        if (!p)
            return fail(SOBRC_EDEVICE, "no device address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SOBRC_OK;
}

}  // namespace

extern "C" {

int32_t sobolev_smooth_particles_static(const sobrc_params* params, int64_t n, const int32_t* d_lin,
                                        const int32_t* d_a, const int32_t* d_b, const float* d_in, float* d_out,
                                        void* stream)
{
    if (!params)
        return fail(SOBRC_EINVAL, "params is NULL");
    size_t need = 0;
    SOBRC_TRY(sobolev_particles_workspace_size(params, n, &need));
    if (need > (size_t)SOBRC_STATIC_SCRATCH_BYTES)
        return fail(SOBRC_EINVAL, "%lld particles on this grid need %zu bytes of scratch > the static %zu bytes",
                    (long long)n, need, (size_t)SOBRC_STATIC_SCRATCH_BYTES);
    if (n == 0)
        return SOBRC_OK;
    if (!d_lin || !d_a || !d_b || !d_in || !d_out)
        return fail(SOBRC_EINVAL, "NULL device pointer");
    void* ws = nullptr;
    SOBRC_TRY(scratch_address(&ws));
    return smooth_particles_ws(params, n, d_lin, d_a, d_b, d_in, d_out, ws, (size_t)SOBRC_STATIC_SCRATCH_BYTES,
                               stream);
}

// ------------------------------------------------------------------ profiling

int32_t profile_enable(sobrc_ctx* c, int32_t on)
{
    if (!c)
        return fail(SOBRC_EINVAL, "ctx is NULL");
    if (on && c->ev.empty()) {
        try {
            c->ev.resize(2 * kEventPairs);
            c->ev_kind.resize(kEventPairs);
        } catch (...) {
            return fail(SOBRC_EINVAL, "out of host memory");
        }
        for (auto& e : c->ev)
            SOBRC_HIP(hipEventCreate(&e), "hipEventCreate");
    }
    c->prof = on != 0;
    return SOBRC_OK;
}

int32_t profile_read(sobrc_ctx* c, double* h_ms, int64_t* h_launches, int32_t reset)
{
    if (!c)
        return fail(SOBRC_EINVAL, "ctx is NULL");
    for (size_t k = 0; k < c->ev_used; ++k) {
        SOBRC_HIP(hipEventSynchronize(c->ev[2 * k + 1]), "hipEventSynchronize");
        float ms = 0.f;
        SOBRC_HIP(hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]), "hipEventElapsedTime");
        c->prof_ms[c->ev_kind[k]] += ms;
        c->prof_n[c->ev_kind[k]] += 1;
    }
    c->ev_used = 0;
    for (int k = 0; k < SOBRC_K_NKINDS; ++k) {
        if (h_ms)
            h_ms[k] = c->prof_ms[k];
        if (h_launches)
            h_launches[k] = c->prof_n[k];
        if (reset) {
            c->prof_ms[k] = 0.0;
            c->prof_n[k] = 0;
        }
    }
    return SOBRC_OK;
}

}  // extern "C"
