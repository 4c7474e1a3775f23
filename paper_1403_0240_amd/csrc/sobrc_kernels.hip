// sobrc_kernels.hip -- gfx950 kernels of one Region Competition iteration with
// particle-approximated Sobolev gradients (arXiv:1403.0240).
//
// Data layout in HBM (one context):
//   lab        u16 label field [nz][ny][nx]
//   rec[2]     particle records {pos, a | b << 16}, tile-major order; pos packs
//              x | y << sy | z << sz.  Two buffers: state t and state t+1.
//   tstart[2]  per-tile offsets into rec (cell list with cells = tiles)
//   active[2]  list of non-empty tiles
//   dE, gH1    fp32 L2 and Sobolev gradients, one per particle
//   st_n/st_s1 exact region statistics (int64 counts, fixed-point sums)
// All kernels are wave64; reductions and compactions use ballots, mbcnt and
// cross-lane shuffles.  No kernel here is a dense contraction, so none uses MFMA.
#include "sobrc_dev.h"

namespace sobrc {

// ----------------------------------------------------------------- helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// number of set bits of m below this lane
__device__ __forceinline__ unsigned lanes_below(unsigned long long m)
{
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ __forceinline__ long long wave_sum_ll(long long v)
{
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ unsigned wave_sum_u(unsigned v)
{
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ void unpack(const Geom& g, unsigned pos, int& x, int& y, int& z)
{
    x = (int)(pos & g.mx);
    y = (int)((pos >> g.sy) & g.my);
    z = (int)((pos >> g.sz) & g.mz);
}

__device__ __forceinline__ unsigned pack(const Geom& g, int x, int y, int z)
{
    return (unsigned)x | ((unsigned)y << g.sy) | ((unsigned)z << g.sz);
}

__device__ __forceinline__ long long lin_of(const Geom& g, int x, int y, int z)
{
    return (long long)x + (long long)g.nx * ((long long)y + (long long)g.ny * z);
}

// Pixel (x, y, z) in a tile-major per-pixel field: the tile's pixels are
// contiguous (x fastest), tiles in tile order.
__device__ __forceinline__ size_t tile_major(const Geom& g, int x, int y, int z)
{
    const unsigned t = (unsigned)(x >> g.tsx) +
                       (unsigned)g.ntx * ((unsigned)(y >> g.tsy) + (unsigned)g.nty * (unsigned)(z >> g.tsz));
    const unsigned l = (unsigned)(x & ((1 << g.tsx) - 1)) | ((unsigned)(y & ((1 << g.tsy) - 1)) << g.tsx) |
                       ((unsigned)(z & ((1 << g.tsz) - 1)) << (g.tsx + g.tsy));
    return ((size_t)t << (g.tsx + g.tsy + g.tsz)) | l;
}

__device__ __forceinline__ float img_at(const Geom& g, const void* img, long long i)
{
    return g.img_u16 ? (float)((const unsigned short*)img)[i] : ((const float*)img)[i];
}

// intensity in the fixed point used for exact region sums
__device__ __forceinline__ long long qvalue(const Geom& g, const void* img, long long i)
{
    if (g.img_u16)
        return (long long)((const unsigned short*)img)[i];
    return __double2ll_rn((double)((const float*)img)[i] * g.fx_scale);
}

__device__ __forceinline__ bool stopped(const DevState* ds)
{
    return (ds->err | ds->converged) != 0;
}

// A step that overflowed the particle capacity was rolled back: labels,
// records and region sums are those of the previous state again, but the
// emission slots of its dirty tiles and the per-label table still describe
// the rejected state.  The stand-alone gradient kernels then write NaN for
// every particle instead of reading them (until init_labels clears the error).
__device__ __forceinline__ bool fill_nan_after_rollback(const Bufs& b, int cur, float* out, VB vb)
{
    const DevState* ds = b.ds;
    if (!(ds->err & kErrCapacity))
        return false;
    const unsigned long long n = ds->n[cur];
    const float qnan = __int_as_float(0x7fc00000);
    for (unsigned long long i = (unsigned long long)vb.id * blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)vb.n * blockDim.x)
        out[i] = qnan;
    return true;
}

// ------------------------------------------------------------ init kernels

__global__ __launch_bounds__(kBlock) void k_init_labels(Geom g, Bufs b, const int32_t* __restrict__ lin_labels,
                                                        const void* img, long long nvox)
{
    long long stride = (long long)gridDim.x * kBlock;
    unsigned mx = 0, bad = 0;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < nvox; i += stride) {
        int l = lin_labels[i];
        if (l < 0 || l >= g.max_labels) {
            bad = 1;
            l = 0;
        }
        b.lab[i] = (unsigned short)l;
        {
            const int x = (int)(i % g.nx), y = (int)((i / g.nx) % g.ny), z = (int)(i / ((long long)g.nx * g.ny));
            b.labt[tile_major(g, x, y, z)] = (unsigned short)l;
        }
        if (!g.img_u16) {
            unsigned bits = __float_as_uint(((const float*)img)[i]) & 0x7fffffffu;
            mx = bits > mx ? bits : mx;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        unsigned t = __shfl_xor(mx, o);
        mx = t > mx ? t : mx;
    }
    unsigned long long anybad = __ballot(bad != 0);
    if (lane_id() == 0) {
        if (mx)
            atomicMax(&b.ds->maxbits, mx);
        if (anybad)
            atomicOr(&b.ds->err, kErrLabel);
    }
}

// Region statistics n_l and sum I over the label field (photometric estimate
// theta_l = region mean).  Equal labels inside a wave are merged first.
__global__ __launch_bounds__(kBlock) void k_stats_init(Geom g, Bufs b, const void* img, long long nvox)
{
    __shared__ long long s_n[kSmallM], s_q[kSmallM];
    if (threadIdx.x < kSmallM) {
        s_n[threadIdx.x] = 0;
        s_q[threadIdx.x] = 0;
    }
    __syncthreads();
    long long stride = (long long)gridDim.x * kBlock;
    for (long long base = (long long)blockIdx.x * kBlock; base < nvox; base += stride) {
        long long i = base + threadIdx.x;
        bool pend = i < nvox;
        int l = pend ? b.lab[i] : -1;
        long long q = pend ? qvalue(g, img, i) : 0;
        unsigned long long m;
        while ((m = __ballot(pend)) != 0) {
            int leader = __ffsll((long long)m) - 1;
            int key = __shfl(l, leader);
            bool match = pend && l == key;
            long long c = wave_sum_ll(match ? 1 : 0);
            long long s = wave_sum_ll(match ? q : 0);
            if (lane_id() == leader) {
                if (g.small_m) {
                    atomicAdd((unsigned long long*)&s_n[key], (unsigned long long)c);
                    atomicAdd((unsigned long long*)&s_q[key], (unsigned long long)s);
                } else {
                    atomicAdd((unsigned long long*)&b.st_n[key], (unsigned long long)c);
                    atomicAdd((unsigned long long*)&b.st_s1[key], (unsigned long long)s);
                }
            }
            pend = pend && !match;
        }
    }
    __syncthreads();
    if (g.small_m && (int)threadIdx.x < g.max_labels && s_n[threadIdx.x]) {
        atomicAdd((unsigned long long*)&b.st_n[threadIdx.x], (unsigned long long)s_n[threadIdx.x]);
        atomicAdd((unsigned long long*)&b.st_s1[threadIdx.x], (unsigned long long)s_q[threadIdx.x]);
    }
}

// ------------------------------------------------------- particle emission
//
// A pixel carries one particle per distinct label b != L(x) among its
// in-bounds full neighbours (8 in 2D, 26 in 3D).  Tiles are scanned with the
// tile plus a one-pixel halo of labels staged in LDS; pixels outside the image
// hold the sentinel 0xFFFF (labels are < 65535).

constexpr int kBoxMax = 4096;  // bytes of a wave's label box (u16): 18 x 10 x 10 fits
constexpr unsigned short kNone = 0xFFFF;

struct TileInfo {
    int tx, ty, tz;        // tile coordinates
    int TX, TY, TZ;        // tile edge
    int BX, BY, BZ, hz;    // LDS box (tile + halo), z halo (0 in 2D)
};

__device__ __forceinline__ TileInfo tile_info(const Geom& g, unsigned t)
{
    TileInfo ti;
    ti.tx = (int)(t % (unsigned)g.ntx);
    ti.ty = (int)((t / (unsigned)g.ntx) % (unsigned)g.nty);
    ti.tz = (int)(t / ((unsigned)g.ntx * (unsigned)g.nty));
    ti.TX = 1 << g.tsx;
    ti.TY = 1 << g.tsy;
    ti.TZ = 1 << g.tsz;
    ti.hz = g.ndim == 3 ? 1 : 0;
    ti.BX = ti.TX + 2;
    ti.BY = ti.TY + 2;
    ti.BZ = ti.TZ + 2 * ti.hz;
    return ti;
}

__device__ void load_label_box(const Geom& g, const unsigned short* __restrict__ lab, unsigned short* s,
                               const TileInfo& ti)
{
    int nbox = ti.BX * ti.BY * ti.BZ;
    int ox = ti.tx * ti.TX - 1, oy = ti.ty * ti.TY - 1, oz = ti.tz * ti.TZ - ti.hz;
    for (int k = threadIdx.x; k < nbox; k += kBlock) {
        int bx = k % ti.BX, by = (k / ti.BX) % ti.BY, bz = k / (ti.BX * ti.BY);
        int x = ox + bx, y = oy + by, z = oz + bz;
        bool in = x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
        s[k] = in ? lab[lin_of(g, x, y, z)] : kNone;
    }
}

// Distinct neighbour labels of box cell c that differ from `own`: returns how
// many; the smallest and largest are left in lo/hi.
__device__ __forceinline__ int neighbour_span(const unsigned short* s, int c, int BX, int BXY, int zr,
                                              int own, int& lo, int& hi)
{
    lo = 0x10000;
    hi = -1;
    for (int dz = -zr; dz <= zr; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int l = s[c + dx + BX * dy + BXY * dz];
                if (l != own && l != kNone) {
                    lo = l < lo ? l : lo;
                    hi = l > hi ? l : hi;
                }
            }
    if (hi < 0)
        return 0;
    if (lo == hi)
        return 1;
    int cnt = 1, prev = lo;
    for (;;) {
        int nxt = 0x10000;
        for (int dz = -zr; dz <= zr; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int l = s[c + dx + BX * dy + BXY * dz];
                    if (l != own && l != kNone && l > prev && l < nxt)
                        nxt = l;
                }
        if (nxt == 0x10000)
            break;
        ++cnt;
        prev = nxt;
    }
    return cnt;
}

// next distinct neighbour label above `prev` (0x10000 if none)
__device__ __forceinline__ int neighbour_next(const unsigned short* s, int c, int BX, int BXY, int zr,
                                              int own, int prev)
{
    int nxt = 0x10000;
    for (int dz = -zr; dz <= zr; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int l = s[c + dx + BX * dy + BXY * dz];
                if (l != own && l != kNone && l > prev && l < nxt)
                    nxt = l;
            }
    return nxt;
}

__device__ __forceinline__ unsigned block_sum_u(unsigned v, unsigned* s_red)
{
    v = wave_sum_u(v);
    int w = threadIdx.x >> 6;
    __syncthreads();
    if (lane_id() == 0)
        s_red[w] = v;
    __syncthreads();
    unsigned t = 0;
    for (int i = 0; i < kBlock / 64; ++i)
        t += s_red[i];
    return t;
}

// exclusive prefix over the block (thread order); *total receives the sum
// Block barrier that orders LDS only: global loads already issued stay in
// flight across it (a full __syncthreads waits for them).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Exclusive block scan whose barriers leave outstanding global loads alone.
__device__ __forceinline__ unsigned block_exscan_lds(unsigned v, unsigned* s_red, unsigned* total)
{
    int lane = lane_id(), w = threadIdx.x >> 6;
    unsigned inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        unsigned t = __shfl_up(inc, o);
        if (lane >= o)
            inc += t;
    }
    lds_barrier();
    if (lane == 63)
        s_red[w] = inc;
    lds_barrier();
    unsigned off = 0, tot = 0;
    for (int i = 0; i < kBlock / 64; ++i) {
        unsigned c = s_red[i];
        off += i < w ? c : 0;
        tot += c;
    }
    *total = tot;
    return off + inc - v;
}

__device__ __forceinline__ unsigned block_exscan_u(unsigned v, unsigned* s_red, unsigned* total)
{
    int lane = lane_id(), w = threadIdx.x >> 6;
    unsigned inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        unsigned t = __shfl_up(inc, o);
        if (lane >= o)
            inc += t;
    }
    __syncthreads();
    if (lane == 63)
        s_red[w] = inc;
    __syncthreads();
    unsigned off = 0, tot = 0;
    for (int i = 0; i < kBlock / 64; ++i) {
        unsigned c = s_red[i];
        off += i < w ? c : 0;
        tot += c;
    }
    *total = tot;
    return off + inc - v;
}


__device__ __forceinline__ unsigned block_reduce_u(unsigned v, unsigned* s_red, int op)
{
    for (int o = 32; o > 0; o >>= 1) {
        unsigned t = __shfl_xor(v, o);
        v = op == 0 ? (t < v ? t : v) : (op == 1 ? (t > v ? t : v) : (t | v));
    }
    int w = threadIdx.x >> 6;
    __syncthreads();
    if (lane_id() == 0)
        s_red[w] = v;
    __syncthreads();
    unsigned r = s_red[0];
    for (int i = 1; i < kBlock / 64; ++i) {
        unsigned t = s_red[i];
        r = op == 0 ? (t < r ? t : r) : (op == 1 ? (t > r ? t : r) : (t | r));
    }
    return r;
}

// Per-wave LDS of one tile's emission: the label box and per-row label masks.
struct WaveEmit {
    unsigned short box[kBoxMax / 2];
    unsigned mlo[128], mhi[128];
};

// Order LDS writes of this wave before its later reads (a wave's LDS
// operations complete in order; this keeps the compiler from reordering).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ unsigned wave_excl_scan_u(unsigned v, unsigned& total)
{
    const int lane = lane_id();
    unsigned inc = v;
    for (int d = 1; d < 64; d <<= 1) {
        unsigned u = __shfl_up(inc, d);
        if (lane >= d)
            inc += u;
    }
    total = __shfl(inc, 63);
    return inc - v;
}

// Label box of a tile (tile + one-pixel halo) into LDS by one wave: all of a
// lane's loads are issued before any is stored, so their latencies overlap.
__device__ void wave_load_box(const Geom& g, const unsigned short* __restrict__ lab, unsigned short* box,
                              const TileInfo& ti)
{
    constexpr int kPer = 16;  // box entries per lane and pass (1024 per pass)
    const int nbox = ti.BX * ti.BY * ti.BZ;  // <= kBoxMax / 2
    const int ox = ti.tx * ti.TX - 1, oy = ti.ty * ti.TY - 1, oz = ti.tz * ti.TZ - ti.hz;
    const int lane = lane_id();
    // walk the box in (x, y, z) steps of 64 cells without divisions per entry
    int bx = lane % ti.BX, by = (lane / ti.BX) % ti.BY, bz = lane / (ti.BX * ti.BY);
    const int sx = 64 % ti.BX, sy = (64 / ti.BX) % ti.BY, sz = 64 / (ti.BX * ti.BY);
    for (int k0 = 0; k0 < nbox; k0 += 64 * kPer) {
        unsigned short v[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int k = k0 + lane + 64 * u;
            int x = ox + bx, y = oy + by, z = oz + bz;
            bool in = k < nbox && x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
            v[u] = in ? lab[lin_of(g, x, y, z)] : kNone;
            bx += sx;
            int cy = bx >= ti.BX;
            bx -= cy ? ti.BX : 0;
            by += sy + cy;
            int cz = by >= ti.BY;
            by -= cz ? ti.BY : 0;
            bz += sz + cz;
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int k = k0 + lane + 64 * u;
            if (k < nbox)
                box[k] = v[u];
        }
    }
    wave_lds_sync();
}

// Particles of tile t under the current labels, counted by one wave.  Each
// lane holds whole rows of the box (tile + one-pixel halo) in registers: the
// box's labels, whether it holds two labels lo < hi or more, and the per-row
// masks of "label == lo" and "label == hi" come out of registers without LDS
// round trips.  With two labels a pixel is a particle iff its 3x3(x3)
// neighbourhood holds both, i.e. iff the OR of the dilated masks over the
// neighbourhood is set in both.  The tile's slot keeps, per tile row, the
// particle bits, the bits of pixels labelled lo and the particles before the
// row, so records can be written later without the labels; boxes with more
// labels are enumerated from an LDS copy and marked for a full re-enumeration
// (slot word 0 = 0xFFFF).
template <int ND, int WIDE>
__device__ unsigned wave_count_tile(const Geom& g, const unsigned short* __restrict__ lab,
                                    const unsigned short* __restrict__ labt, unsigned t, WaveEmit& W,
                                    unsigned* __restrict__ slot)
{
    constexpr int TX = tile_ex(ND, WIDE), TY = tile_ey(ND, WIDE), TZ = tile_ez(ND), HZ = ND == 3 ? 1 : 0;
    constexpr int BX = TX + 2, BY = TY + 2, BZ = TZ + 2 * HZ, NROW = BY * BZ;
    constexpr int RPL = (NROW + 63) / 64;  // box rows per lane
    static_assert(BX * BY * BZ <= kBoxMax / 2 && NROW <= 128, "box too large");
    const int lane = lane_id();
    const int tx = (int)(t % (unsigned)g.ntx), ty = (int)((t / (unsigned)g.ntx) % (unsigned)g.nty);
    const int tz = (int)(t / ((unsigned)g.ntx * (unsigned)g.nty));
    const int ox = tx * TX - 1, oy = ty * TY - 1, oz = tz * TZ - HZ;
    // every lane issues all of its loads before using any.  With rows of a
    // multiple of 8 labels a box row is read as the aligned 16-byte chunks
    // of [tx*TX - 8, tx*TX + TX + 8) from the tile-major copy (each a piece
    // of one tile row: the tile's own rows are one contiguous block); chunks
    // outside the row are not read.  Otherwise each label is read on its own.
    constexpr int NCH = (TX + 16) / 8;  // 16-byte chunks per box row
    unsigned v[RPL][BX];
    if ((g.nx & 7) == 0) {
        uint4 ch[RPL][NCH];
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int r = lane + 64 * i;
            const int by = r % BY, bz = r / BY;
            const int y = oy + by, z = oz + bz;
            const bool rin = r < NROW && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
            const int yc = rin ? y : 0, zc = rin ? z : 0;
            // tile row (y, z) of tile column x = 0, in 16-byte units
            const size_t rbase = (((size_t)g.ntx * ((size_t)(yc >> g.tsy) + (size_t)g.nty * (size_t)(zc >> g.tsz)))
                                  << (g.tsx + g.tsy + g.tsz)) +
                                 ((size_t)((yc & (TY - 1)) + TY * (zc & (TZ - 1))) << g.tsx);
            const uint4* tl = (const uint4*)labt;
            const int c0 = tx * (TX / 8) - 1;  // chunk index of x = tx*TX - 8
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int cc = c0 + c;
                const bool cin = rin && cc >= 0 && 8 * cc + 8 <= g.nx;
                const int x0 = 8 * (cin ? cc : 0);  // first pixel of the chunk
                const size_t at = (rbase + ((size_t)(x0 >> g.tsx) << (g.tsx + g.tsy + g.tsz)) + (size_t)(x0 & (TX - 1))) >> 3;
                ch[i][c] = cin ? tl[at] : make_uint4(0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu);
            }
        }
#pragma unroll
        for (int i = 0; i < RPL; ++i)
#pragma unroll
            for (int bx = 0; bx < BX; ++bx) {
                const int e = 7 + bx;  // label index inside the 8 * NCH window
                const uint4 q = ch[i][e >> 3];
                const int w = (e >> 1) & 3;
                const unsigned word = w == 0 ? q.x : w == 1 ? q.y : w == 2 ? q.z : q.w;
                v[i][bx] = (e & 1) ? (word >> 16) : (word & 0xffffu);
            }
    } else {
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int r = lane + 64 * i;
            const int by = r % BY, bz = r / BY;
            const int y = oy + by, z = oz + bz;
            const bool rin = r < NROW && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
            const long long base = rin ? lin_of(g, 0, y, z) : 0;
#pragma unroll
            for (int bx = 0; bx < BX; ++bx) {
                const int x = ox + bx;
                v[i][bx] = (rin && x >= 0 && x < g.nx) ? (unsigned)lab[base + x] : (unsigned)kNone;
            }
        }
    }
    unsigned mn = 0xffffu, mx = 0u;
#pragma unroll
    for (int i = 0; i < RPL; ++i)
#pragma unroll
        for (int bx = 0; bx < BX; ++bx) {
            const unsigned l = v[i][bx];
            if (l != kNone) {
                mn = l < mn ? l : mn;
                mx = l > mx ? l : mx;
            }
        }
    for (int o = 32; o > 0; o >>= 1) {
        unsigned a = __shfl_xor(mn, o), c = __shfl_xor(mx, o);
        mn = a < mn ? a : mn;
        mx = c > mx ? c : mx;
    }
    if (mx <= mn) {  // one label: no contour in this tile
        if (lane < TY * TZ)
            slot[1 + lane] = 0u;  // no particle bits (the brick kernels read neighbours' rows unguarded)
        return 0;
    }
    bool third = false;
#pragma unroll
    for (int i = 0; i < RPL; ++i)
#pragma unroll
        for (int bx = 0; bx < BX; ++bx) {
            const unsigned l = v[i][bx];
            third = third || (l != kNone && l != mn && l != mx);
        }
    constexpr int BXY = BX * BY;
    if (__ballot(third) != 0) {
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int r = lane + 64 * i;
            if (r < NROW)
#pragma unroll
                for (int bx = 0; bx < BX; ++bx)
                    W.box[r * BX + bx] = (unsigned short)v[i][bx];
        }
        wave_lds_sync();
        unsigned cc = 0;
        for (int q = lane; q < TX * TY * TZ; q += 64) {
            const int lx = q % TX, ly = (q / TX) % TY, lz = q / (TX * TY);
            const int x = tx * TX + lx, y = ty * TY + ly, z = tz * TZ + lz;
            if (x >= g.nx || y >= g.ny || z >= g.nz)
                continue;
            const int cidx = (lx + 1) + BX * ((ly + 1) + BY * (lz + HZ));
            int lo, hi;
            cc += neighbour_span(W.box, cidx, BX, BXY, HZ, W.box[cidx], lo, hi);
        }
        if (lane == 0)
            slot[0] = 0xffffu;
        return wave_sum_u(cc);
    }
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        const int r = lane + 64 * i;
        unsigned ml = 0, mh = 0;
#pragma unroll
        for (int bx = 0; bx < BX; ++bx) {
            ml |= (v[i][bx] == mn ? 1u : 0u) << bx;
            mh |= (v[i][bx] == mx ? 1u : 0u) << bx;
        }
        if (r < NROW) {
            W.mlo[r] = ml;
            W.mhi[r] = mh;
        }
    }
    wave_lds_sync();
    unsigned pb = 0;
    if (lane < TY * TZ) {  // one interior row per lane (at most 64)
        const int by = lane % TY + 1, bz = lane / TY + HZ;
        unsigned ol = 0, oh = 0;
#pragma unroll
        for (int dz = -HZ; dz <= HZ; ++dz)
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const int r = (by + dy) + BY * (bz + dz);
                const unsigned ml = W.mlo[r], mh = W.mhi[r];
                ol |= ml | (ml << 1) | (ml >> 1);
                oh |= mh | (mh << 1) | (mh >> 1);
            }
        const int rc = by + BY * bz;
        const unsigned cl = W.mlo[rc], ch = W.mhi[rc];
        constexpr unsigned tmask = (1u << TX) - 1u;
        pb = ((ol & oh & (cl | ch)) >> 1) & tmask;
        slot[1 + lane] = pb | (((cl >> 1) & tmask) << 16);
    }
    unsigned tot;
    const unsigned pre = wave_excl_scan_u((unsigned)__popc(pb), tot);
    if (lane < TY * TZ)
        slot[1 + kSlotRows + lane] = pre;
    if (lane == 0)
        slot[0] = mn | (mx << 16);
    return tot;
}

// Write the records of tile t (counted by wave_count_tile) at rec[o...], one
// wave, canonical order: position inside the tile (x fastest), then b.  The
// caller loads the tile slot's header (hdr = slot[0]) and this lane's row word
// (slot[1 + lane], every lane: the slot has kSlotWords > 64 words) together
// with the tile's offset, so that their latencies overlap.
__device__ void wave_write_tile(const Geom& g, const unsigned short* __restrict__ lab, unsigned t, WaveEmit& W,
                                unsigned hdr, unsigned word, uint2* __restrict__ rec, unsigned o)
{
    static_assert(kSlotWords > 64, "a row word per lane");
    const int lane = lane_id();
    TileInfo ti = tile_info(g, t);
    if ((hdr & 0xffffu) != 0xffffu) {
        const unsigned lo = hdr & 0xffffu, hi = hdr >> 16;
        word = lane < ti.TY * ti.TZ ? word : 0u;
        unsigned pb = word & 0xffffu, own_lo = word >> 16;
        unsigned tot;
        unsigned oo = o + wave_excl_scan_u((unsigned)__popc(pb), tot);
        int y = ti.ty * ti.TY + (lane & (ti.TY - 1)), z = ti.tz * ti.TZ + (lane >> g.tsy);
        while (pb) {
            int lx = __ffs(pb) - 1;
            pb &= pb - 1;
            bool isl = (own_lo >> lx) & 1u;
            unsigned own = isl ? lo : hi, oth = isl ? hi : lo;
            rec[oo++] = make_uint2(pack(g, ti.tx * ti.TX + lx, y, z), own | (oth << 16));
        }
        return;
    }
    // several labels: enumerate distinct neighbour labels per pixel
    wave_load_box(g, lab, W.box, ti);
    const int BXY = ti.BX * ti.BY, zr = ti.hz;
    const int nv = ti.TX * ti.TY * ti.TZ;
    const int per = (nv + 63) / 64;  // contiguous run of voxels per lane
    const int v0 = lane * per, v1 = min(v0 + per, nv);
    unsigned cc = 0;
    for (int v = v0; v < v1; ++v) {
        int lx = v & (ti.TX - 1), ly = (v >> g.tsx) & (ti.TY - 1), lz = v >> (g.tsx + g.tsy);
        int x = ti.tx * ti.TX + lx, y = ti.ty * ti.TY + ly, z = ti.tz * ti.TZ + lz;
        if (x >= g.nx || y >= g.ny || z >= g.nz)
            continue;
        int cidx = (lx + 1) + ti.BX * ((ly + 1) + ti.BY * (lz + ti.hz));
        int lo, hi;
        cc += neighbour_span(W.box, cidx, ti.BX, BXY, zr, W.box[cidx], lo, hi);
    }
    unsigned tot;
    unsigned oo = o + wave_excl_scan_u(cc, tot);
    for (int v = v0; v < v1; ++v) {
        int lx = v & (ti.TX - 1), ly = (v >> g.tsx) & (ti.TY - 1), lz = v >> (g.tsx + g.tsy);
        int x = ti.tx * ti.TX + lx, y = ti.ty * ti.TY + ly, z = ti.tz * ti.TZ + lz;
        if (x >= g.nx || y >= g.ny || z >= g.nz)
            continue;
        int cidx = (lx + 1) + ti.BX * ((ly + 1) + ti.BY * (lz + ti.hz));
        int own = W.box[cidx];
        unsigned pos = pack(g, x, y, z);
        int l = neighbour_next(W.box, cidx, ti.BX, BXY, zr, own, -1);
        while (l != 0x10000) {
            rec[oo++] = make_uint2(pos, (unsigned)own | ((unsigned)l << 16));
            l = neighbour_next(W.box, cidx, ti.BX, BXY, zr, own, l);
        }
    }
}

// Emission ranges: range r holds tiles [r*Re, (r+1)*Re) (Re = 2^lgRe <=
// kBlock); the scan works on per-range totals.  Dirty tiles (a flip within one
// pixel this iteration, or every tile at initialisation) are re-emitted one
// wave per tile.  Slot j (block j mod gridDim) takes tile
//   t = s * Ls + u,   s = j mod 8,  u = j / 8,  Ls = ceil(ntiles / 8),
// so with a grid that is a multiple of 8 every XCD works on one contiguous
// eighth of the tile order (neighbouring tiles share label rows, and so lines
// of that XCD's L2), while consecutive tiles go to consecutive blocks of the
// XCD (a surface crossing a run of tiles spreads over many blocks).
__device__ __forceinline__ bool slot_tile(const Geom& g, unsigned j, unsigned& t)
{
    const unsigned ls = ((unsigned)g.ntiles + 7u) >> 3;
    const unsigned u = j >> 3;
    t = (j & 7u) * ls + u;
    return u < ls && t < (unsigned)g.ntiles;
}

// Items [a0, a1) of [0, na) for this block: contiguous chunks, consecutive
// chunks on the same XCD (blocks are dealt to the 8 XCDs round-robin), so
// that work on neighbouring tiles shares one L2.  Grids that are not a
// multiple of 8 take chunks in block order.
__device__ __forceinline__ void xcd_chunk(unsigned na, VB vb, unsigned& a0, unsigned& a1)
{
    const unsigned G = vb.n;
    const unsigned L = (G & 7u) ? vb.id : (vb.id & 7u) * (G >> 3) + (vb.id >> 3);
    if (G < (1u << 20)) {
        // floor(L na / G) through one double division: the product is below
        // 2^52 (exact), the quotient below 2^32, so the correctly rounded
        // quotient is within 2^-21 of the exact one while a fractional part
        // is at least 1/G > 2^-20 from the next integer -- truncation is exact
        const double dn = (double)na, dG = (double)G;
        a0 = (unsigned)((double)L * dn / dG);
        a1 = (unsigned)((double)(L + 1) * dn / dG);
    } else {
        a0 = (unsigned)((unsigned long long)L * na / G);
        a1 = (unsigned)((unsigned long long)(L + 1) * na / G);
    }
}

__device__ __forceinline__ bool tile_dirty(const Bufs& b, unsigned t, unsigned epoch, int all_dirty)
{
    return all_dirty || b.dirty[t] == epoch;
}

// Particle count of every tile of the next state, accumulated per range.
// Clean tiles keep their previous count.
template <int ND, int WIDE>
__device__ __forceinline__ void count_body(const Geom& g, const Bufs& b, int cur, int gated, int all_dirty, VB vb)
{
    __shared__ WaveEmit W[kBlock / 64];
    __shared__ unsigned s_dl[kBlock];
    __shared__ unsigned s_ndl;
    __shared__ unsigned s_red[kBlock / 64];
    if (g.dlistm) {
        // The dirty tiles go to a flat list that count_list_body counts: the
        // block takes its emission range as a contiguous run of tiles (Re <=
        // kBlock), lists the range's dirty tiles in tile order and forms the
        // range's sums of the clean tiles itself (no atomics).  The loads go
        // out with the stop flag (in bounds either way).
        const int tr = (int)(vb.id << g.lgRe) + (int)threadIdx.x;
        const bool in = (int)threadIdx.x < g.Re && tr < g.ntiles;
        const unsigned tdv = in ? b.dirty[tr] : 0u;
        const unsigned ts0 = in ? b.tstart[cur][tr] : 0u, ts1 = in ? b.tstart[cur][tr + 1] : 0u;
        const unsigned epoch = b.ds->epoch;
        if (gated && stopped(b.ds))
            return;
        const bool dirty = in && (all_dirty || tdv == epoch);
        const unsigned c = in && !dirty ? ts1 - ts0 : 0u;
        if (in && !dirty)
            b.tcnt[tr] = c;
        unsigned packed, sum;
        const unsigned pre = block_exscan_u((dirty ? 1u : 0u) | (c ? 1u << 16 : 0u), s_red, &packed);
        if (dirty)
            b.dlist[(size_t)vb.id * kBlock + (pre & 0xffffu)] = (unsigned)tr;
        (void)block_exscan_u(c, s_red, &sum);
        if (threadIdx.x == 0) {
            b.dcnt[vb.id] = packed & 0xffffu;
            b.part_cnt[vb.id] = sum;  // count_list_body adds the dirty tiles' counts
            b.part_act[vb.id] = packed >> 16;
        }
        return;
    }
    const unsigned G = vb.n;
    const unsigned j = vb.id + threadIdx.x * G;  // G * kBlock >= 8 * ceil(ntiles / 8)
    unsigned t;
    const bool has = slot_tile(g, j, t);
    // the tile's loads go out with the stop flag (in bounds either way)
    const unsigned tdv = has ? b.dirty[t] : 0u;
    const unsigned ts0 = has ? b.tstart[cur][t] : 0u, ts1 = has ? b.tstart[cur][t + 1] : 0u;
    if (gated && stopped(b.ds))
        return;
    const unsigned epoch = b.ds->epoch;
    if (threadIdx.x == 0)
        s_ndl = 0;
    __syncthreads();
    if (has) {
        if (all_dirty || tdv == epoch) {
            s_dl[atomicAdd(&s_ndl, 1u)] = t;
        } else {
            unsigned c = ts1 - ts0;
            b.tcnt[t] = c;
            if (c) {
                atomicAdd(&b.part_cnt[t >> g.lgRe], c);
                atomicAdd(&b.part_act[t >> g.lgRe], 1u);
            }
        }
    }
    __syncthreads();
    const unsigned ndl = s_ndl;
    const int wv = threadIdx.x >> 6;
    for (unsigned i = wv; i < ndl; i += kBlock / 64) {
        const unsigned td = s_dl[i];
        unsigned cc = wave_count_tile<ND, WIDE>(g, b.lab, b.labt, td, W[wv], b.tslot + (size_t)td * kSlotWords);
        if (lane_id() == 0) {
            b.tcnt[td] = cc;
            if (cc) {
                atomicAdd(&b.part_cnt[td >> g.lgRe], cc);
                atomicAdd(&b.part_act[td >> g.lgRe], 1u);
            }
        }
    }
}

template <int ND, int WIDE>
__global__ __launch_bounds__(kBlock) void k_count(Geom g, Bufs b, int cur, int gated, int all_dirty)
{
    count_body<ND, WIDE>(g, b, cur, gated, all_dirty, VB{blockIdx.x, gridDim.x});
}

// Dirty tiles listed by count_body, counted with one wave each.  Emission
// block j lists the dirty tiles of range j in tile order, so the lists
// concatenated in block order are the dirty tiles in tile order.  Every block
// forms the exclusive prefix of the list lengths (two 16-byte loads per
// thread) and takes an XCD-contiguous, equal share of the items, one per wave
// in turn: the dirty tiles of one region are counted on one XCD (their label
// boxes overlap, so they share lines of its L2), and every wave has at most
// one more item than any other.  The items also go to a flat list (tile ids)
// for the write kernel.
template <int ND, int WIDE>
__device__ __forceinline__ void count_list_body(const Geom& g, const Bufs& b, int gated, VB vb)
{
    __shared__ WaveEmit W[kBlock / 64];
    __shared__ unsigned s_pre[kMaxGrid + 1];
    __shared__ unsigned s_red[kBlock / 64];
    static_assert(kMaxGrid == 8 * kBlock, "eight list lengths per thread");
    static_assert(kMaxGrid <= 64 * 64, "two probes of 64 positions cover the prefix");
    const int ge = g.ge;
    const int i0 = (int)threadIdx.x * 8;
    const uint4* dc = (const uint4*)b.dcnt;  // kMaxGrid entries; only those < ge are read
    // the list lengths are loaded with the stop flag (in bounds either way)
    const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
    const uint4 q0 = i0 < ge ? dc[2 * threadIdx.x] : z4, q1 = i0 + 4 < ge ? dc[2 * threadIdx.x + 1] : z4;
    if (gated && stopped(b.ds))
        return;
    unsigned c[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
    unsigned sum = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        c[k] = i0 + k < ge ? c[k] : 0u;
        sum += c[k];
    }
    unsigned tot;
    unsigned ex = block_exscan_u(sum, s_red, &tot);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (i0 + k < ge)
            s_pre[i0 + k] = ex;
        ex += c[k];
    }
    if (threadIdx.x == 0)
        s_pre[ge] = tot;
    __syncthreads();
    if (vb.id == 0 && threadIdx.x == 0)
        b.ds->ndirty = tot;
    const int wv = threadIdx.x >> 6, lane = lane_id();
    unsigned a0, a1;
    xcd_chunk(tot, vb, a0, a1);
    for (unsigned item = a0 + wv; item < a1; item += kBlock / 64) {
        // list block holding item: the largest lo with s_pre[lo] <= item.  The
        // prefix is non-decreasing with s_pre[0] = 0, so the wave finds it in
        // two probes of 64 positions (chunks of S, then within the chunk)
        // instead of a chain of dependent LDS reads
        const int S = (ge + 63) >> 6;
        const int p1 = lane * S;
        const bool c1 = p1 < ge && s_pre[p1] <= item;
        const int lo1 = (__popcll(__ballot(c1)) - 1) * S;
        const int p2 = lo1 + lane;
        const bool c2 = lane < S && p2 < ge && s_pre[p2] <= item;
        const int lo = lo1 + __popcll(__ballot(c2)) - 1;
        const unsigned pos = (unsigned)lo * kBlock + (item - s_pre[lo]);
        const unsigned td = b.dlist[pos];
        unsigned cc = wave_count_tile<ND, WIDE>(g, b.lab, b.labt, td, W[wv], b.tslot + (size_t)td * kSlotWords);
        if (lane_id() == 0) {
            b.dflat[item] = td;
            b.tcnt[td] = cc;
            if (cc) {
                atomicAdd(&b.part_cnt[td >> g.lgRe], cc);
                atomicAdd(&b.part_act[td >> g.lgRe], 1u);
            }
        }
    }
}

template <int ND, int WIDE>
__global__ __launch_bounds__(kBlock) void k_count_list(Geom g, Bufs b, int gated)
{
    count_list_body<ND, WIDE>(g, b, gated, VB{blockIdx.x, gridDim.x});
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o);
    return v;
}

// Single block: fold the flip partials into the region statistics, refresh the
// per-label table of the L2 gradient, scan the emission partials into block
// offsets, check the capacity (requesting a roll-back if it is exceeded), and
// record telemetry and the convergence test.  The block is latency bound: all
// partials are loaded before the first wait (the first two emission partials
// of each thread stay in registers), and the per-label statistics partials are
// split over every wave, kScanThreads / 64 / max_labels waves per label.
__device__ __forceinline__ void scan_body(const Geom& g, const Bufs& b, int cur, int nxt, int is_init, float tol, int32_t* d_nflips, int gated, int flags, VB vb)
{
    constexpr int kW = kScanThreads / 64;
    static_assert(kMaxGrid <= 2 * kScanThreads, "two flip partials per thread");
    __shared__ unsigned long long s_sum[kW];
    __shared__ unsigned s_nz[kW];
    __shared__ unsigned s_f[kW], s_r[kW];
    __shared__ long long s_dn[kW], s_dq[kW];
    DevState* ds = b.ds;
    if (gated && stopped(ds))
        return;
    const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
    const int per = (g.ge + kScanThreads - 1) / kScanThreads;  // emission partials per thread (<= 2 typ.)
    const int i0 = tid * per, i1 = min(i0 + per, g.ge);
    const bool has0 = i0 < i1, has1 = i0 + 1 < i1;
    const unsigned c0 = has0 ? b.part_cnt[i0] : 0u, z0 = has0 ? b.part_act[i0] : 0u;
    const unsigned c1 = has1 ? b.part_cnt[i0 + 1] : 0u, z1 = has1 ? b.part_act[i0 + 1] : 0u;
    unsigned f = 0, rv = 0;
    if (!is_init) {
        const int j1 = tid + kScanThreads;
        f = (tid < g.gp ? b.part_f[tid] : 0u) + (j1 < g.gp ? b.part_f[j1] : 0u);
        rv = (tid < g.gp ? b.part_f[g.gp + tid] : 0u) + (j1 < g.gp ? b.part_f[g.gp + j1] : 0u);
    }
    // statistics of few labels: wave w takes chunk cw of label lw
    const int L = g.small_m ? g.max_labels : 0;
    const int wpl = L ? kW / L : 0;
    const int lw = (wpl && w < L * wpl) ? w / wpl : -1;
    const int cw = wpl ? w % wpl : 0;
    const bool lead = lw >= 0 && cw == 0 && lane == 0;
    long long n0 = 0, q0 = 0, dn = 0, dq = 0;
    if (lead) {
        n0 = b.st_n[lw];
        q0 = b.st_s1[lw];
    }
    // many labels: the statistics are final already (atomics in k_flip); a
    // thread's first label goes out with the other loads
    long long ln0 = 0, ls0 = 0;
    if (!g.small_m && tid < g.max_labels) {
        ln0 = b.st_n[tid];
        ls0 = b.st_s1[tid];
    }
    unsigned pre_n = 0, pre_it = 0, pre_lm = 0, pre_sw = 0;
    if (tid == 0 && !is_init) {
        pre_n = ds->n[cur];
        pre_it = ds->iters;
        pre_lm = ds->lmode;
        pre_sw = ds->switch_it;
    }
    if (!is_init && lw >= 0) {
        const int lo = (int)((long long)cw * g.gp / wpl), hi = (int)((long long)(cw + 1) * g.gp / wpl);
        const long long* pn = b.part_n + (long long)lw * g.gp;
        const long long* pq = b.part_q + (long long)lw * g.gp;
        for (int k0 = lo + lane; k0 < hi; k0 += 8 * 64) {
            long long an[8], aq[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = k0 + 64 * u;
                an[u] = i < hi ? pn[i] : 0;
                aq[u] = i < hi ? pq[i] : 0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                dn += an[u];
                dq += aq[u];
            }
        }
    }
    unsigned long long sum = (unsigned long long)c0 + c1;
    unsigned nz = z0 + z1;
    for (int i = i0 + 2; i < i1; ++i) {  // very large images only
        sum += b.part_cnt[i];
        nz += b.part_act[i];
    }
    unsigned nf = 0;
    if (!is_init) {
        f = wave_sum(f);
        rv = wave_sum(rv);
        if (lane == 0) {
            s_f[w] = f;
            s_r[w] = rv;
        }
    }
    if (!is_init && lw >= 0) {
        dn = wave_sum(dn);
        dq = wave_sum(dq);
        if (lane == 0) {
            s_dn[w] = dn;
            s_dq[w] = dq;
        }
    }
    if (!g.small_m) {  // statistics already final (atomics in k_flip)
        for (int l = tid; l < g.max_labels; l += kScanThreads) {
            const long long n = l == tid ? ln0 : b.st_n[l];
            const long long q = l == tid ? ls0 : b.st_s1[l];
            double d = (double)n;
            float mu = n > 0 ? (float)((double)q * g.fx_inv / d) : 0.f;
            float fa = n > 1 ? (float)(d / (d - 1.0)) : 0.f;
            float fb = (float)(d / (d + 1.0));
            b.lstat[l] = make_float4(mu, fa, fb, 0.f);
        }
    }
    // exclusive scan of the emission partials
    unsigned long long isum = sum;
    unsigned inz = nz;
    for (int o = 1; o < 64; o <<= 1) {
        unsigned long long a = __shfl_up(isum, o);
        unsigned z = __shfl_up(inz, o);
        if (lane >= o) {
            isum += a;
            inz += z;
        }
    }
    if (lane == 63) {
        s_sum[w] = isum;
        s_nz[w] = inz;
    }
    __syncthreads();
    if (lead) {
        long long n = n0, q = q0;
        if (!is_init) {
            for (int k = 0; k < wpl; ++k) {
                n += s_dn[w + k];
                q += s_dq[w + k];
            }
            b.st_n[lw] = n;
            b.st_s1[lw] = q;
        }
        double d = (double)n;
        float mu = n > 0 ? (float)((double)q * g.fx_inv / d) : 0.f;
        float fa = n > 1 ? (float)(d / (d - 1.0)) : 0.f;
        float fb = (float)(d / (d + 1.0));
        b.lstat[lw] = make_float4(mu, fa, fb, 0.f);
    }
    unsigned nb = 0;  // reversals
    if (!is_init)
        for (int i = 0; i < kW; ++i) {
            nf += s_f[i];
            nb += s_r[i];
        }
    unsigned long long off = 0, total = 0;
    unsigned offz = 0, totz = 0;
    for (int i = 0; i < kW; ++i) {
        off += i < w ? s_sum[i] : 0;
        offz += i < w ? s_nz[i] : 0;
        total += s_sum[i];
        totz += s_nz[i];
    }
    off += isum - sum;
    offz += inz - nz;
    const bool overflow = total > (unsigned long long)b.cap;
    for (int i = i0; i < i1; ++i) {
        const unsigned c = i == i0 ? c0 : (i == i0 + 1 ? c1 : b.part_cnt[i]);
        const unsigned z = i == i0 ? z0 : (i == i0 + 1 ? z1 : b.part_act[i]);
        if (!overflow) {
            b.part_off[i] = (unsigned)off;
            b.part_aoff[i] = offz;
        }
        off += c;
        offz += z;
        b.part_cnt[i] = 0;  // the next count accumulates afresh
        b.part_act[i] = 0;
    }
    if (overflow && !is_init) {
        for (int t = tid; t <= g.ntiles; t += kScanThreads)
            b.tstart[nxt][t] = b.tstart[cur][t];
        unsigned na = ds->n_active[cur];
        for (unsigned t = tid; t < na; t += kScanThreads)
            b.active[nxt][t] = b.active[cur][t];
    }
    if (tid == 0) {
        if (overflow) {
            ds->err |= kErrCapacity;
            ds->need = total > 0xffffffffull ? 0xffffffffu : (unsigned)total;
            if (!is_init) {
                ds->undo = 1;
                ds->n[nxt] = pre_n;
                ds->n_active[nxt] = ds->n_active[cur];
            }
        } else {
            ds->n[nxt] = (unsigned)total;
            ds->n_active[nxt] = totz;
            ds->go = 1;
        }
        if (!is_init) {
            ds->nflips = nf;
            if (!overflow) {
                const unsigned ncur = pre_n, it = pre_it;
                b.hist[it % kHist] = ncur;
                b.hist[kHist + it % kHist] = nf;
                b.hist[2 * kHist + it % kHist] = nb;
                ds->iters = it + 1;
                if (d_nflips)
                    *d_nflips = (int32_t)nf;
                if (tol > 0.f && (double)nf < (double)tol * (double)ncur)
                    ds->converged = 1;
                // oscillation: at least half of the flips are reversals, in
                // this step and the one before; auto mode then uses L2
                // gradients from the next step on
                const bool osc = nf > 0u && 2ull * nb >= (unsigned long long)nf;
                const bool cycle = nf > 0u && nb == nf;  // every flip undoes the previous step's
                const unsigned lm = pre_lm, sw = pre_sw;
                // this step and the one before ran with L2 gradients
                const bool l2_both = sw != 0u && sw <= it;
                if ((flags & kAuto) && tol > 0.f && l2_both && cycle && (lm & 4u))
                    ds->converged = 1;  // a settled cycle under L2 too: a pixel-resolution minimum
                if ((flags & kAuto) && sw == 0u && osc && (lm & 2u))
                    ds->switch_it = it + 2u;
                ds->lmode = (lm & 1u) | (osc ? 2u : 0u) | (cycle ? 4u : 0u);
            }
        }
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan(Geom g, Bufs b, int cur, int nxt, int is_init, float tol,
                                                      int32_t* d_nflips, int gated, int flags)
{
    scan_body(g, b, cur, nxt, is_init, tol, d_nflips, gated, flags, VB{blockIdx.x, gridDim.x});
}

// Per-pixel move decision of state t (shared by k_flip and the roll-back):
// particle p starts its pixel's run of records; the smallest negative
// gradient of the run wins, ties going to the first (smaller target label).
__device__ __forceinline__ bool decide_move(const uint2* rec, const float* grad, unsigned n, unsigned p,
                                            uint2& r, int& target)
{
    r = rec[p];
    if (p > 0 && rec[p - 1].x == r.x)
        return false;
    int best = -1;
    float bg = 0.f;
    for (unsigned j = p; j < n; ++j) {
        uint2 rj = rec[j];
        if (rj.x != r.x)
            break;
        float gj = grad[j];
        if (gj < 0.f && (best < 0 || gj < bg)) {
            best = (int)j;
            bg = gj;
            target = (int)(rj.y >> 16);
        }
    }
    return best >= 0;
}

// Write the particle records of the next state: dirty tiles are re-emitted
// from the labels in canonical order, clean tiles copy their records from
// state t.  On an overflowing step, restore state t instead.
__device__ __forceinline__ void write_body(const Geom& g, const Bufs& b, const void* img, int cur, int nxt, const float* __restrict__ grad_sob, const float* __restrict__ grad_l2, int flags, int all_dirty, VB vb)
{
    __shared__ WaveEmit W[kBlock / 64];
    __shared__ unsigned s_red[kBlock / 64];
    __shared__ unsigned s_pre[kBlock + 1];
    __shared__ unsigned s_old[kBlock];
    __shared__ unsigned s_dl[kBlock];
    __shared__ unsigned s_ndl;
    DevState* ds = b.ds;
    // the block's emission range: consecutive ranges on one XCD (with a grid
    // that is a multiple of 8), so that the record lines two neighbouring
    // ranges share are written through one L2.  This thread's tile of the
    // range: its loads go out with the state flags (in bounds whichever way
    // the flags decide)
    const unsigned rg = (vb.n & 7u) ? vb.id : (vb.id & 7u) * (vb.n >> 3) + (vb.id >> 3);
    const int t0 = (int)rg << g.lgRe, t1 = min(t0 + g.Re, g.ntiles);
    const int t = t0 + (int)threadIdx.x;
    const bool in = t < t1;
    const unsigned c = in ? b.tcnt[t] : 0;
    const unsigned tdv = in ? b.dirty[t] : 0u;
    const unsigned tso = in ? b.tstart[cur][t] : 0u;
    const unsigned base = b.part_off[rg], abase = b.part_aoff[rg];
    // this block's XCD-contiguous share of the flat list of dirty tiles (in
    // the count's order: neighbouring tiles, whose records are neighbours too,
    // are written through one L2), one item per wave in turn; the first
    // item's loads are issued now, so that they overlap the range's work below
    const int wv = threadIdx.x >> 6, lane = lane_id();
    const unsigned nd0 = g.dlistm ? ds->ndirty : 0u;
    unsigned ia0, ia1;
    xcd_chunk(nd0, vb, ia0, ia1);
    const unsigned item0 = ia0 + (unsigned)wv;
    const unsigned tt0 = item0 < ia1 ? b.dflat[item0] : 0u;
    if (ds->undo) {
        // the same gradients k_flip decided on in this step
        const float* grad = ((flags & kAuto) && (ds->lmode & 1u)) ? grad_l2 : grad_sob;
        long long stride = (long long)vb.n * kBlock;
        unsigned n = ds->n[cur];
        for (long long i = (long long)vb.id * kBlock + threadIdx.x; i < n; i += stride) {
            b.rec[nxt][i] = b.rec[cur][i];
            uint2 r;
            int bb = 0;
            bool mv;
            if (g.topo) {
                r = b.rec[cur][i];
                bb = (int)(r.y >> 16);
                mv = b.tstate[i] == 2;
            } else {
                mv = decide_move(b.rec[cur], grad, n, (unsigned)i, r, bb);
            }
            if (mv) {
                int x, y, z;
                unpack(g, r.x, x, y, z);
                long long lin = lin_of(g, x, y, z);
                int a = (int)(r.y & 0xffffu);
                b.lab[lin] = (unsigned short)a;
                b.labt[tile_major(g, x, y, z)] = (unsigned short)a;
                long long q = qvalue(g, img, lin);
                atomicAdd((unsigned long long*)&b.st_n[a], 1ull);
                atomicAdd((unsigned long long*)&b.st_n[bb], (unsigned long long)(-1ll));
                atomicAdd((unsigned long long*)&b.st_s1[a], (unsigned long long)q);
                atomicAdd((unsigned long long*)&b.st_s1[bb], (unsigned long long)(-q));
            }
        }
        return;
    }
    if (!ds->go)
        return;
    const unsigned epoch = ds->epoch;
    unsigned ctt0 = 0u, pbase0 = 0u, hdr0 = 0u, word0 = 0u, part0 = 0u;
    if (item0 < ia1) {
        ctt0 = b.tcnt[tt0];
        pbase0 = b.part_off[tt0 >> g.lgRe];
        const unsigned* slot = b.tslot + (size_t)tt0 * kSlotWords;
        hdr0 = slot[0];
        word0 = slot[1 + lane];
        const int r0 = (int)(tt0 >> g.lgRe) << g.lgRe;
        for (int k = r0 + lane; k < (int)tt0; k += 64)
            part0 += b.tcnt[k];
    }
    // range rg: offsets, non-empty tile list, and the clean tiles'
    // records moved unchanged to their new offsets
    const bool dirty = in && (all_dirty || tdv == epoch);
    unsigned tot, totz;
    const unsigned ex = block_exscan_lds(c, s_red, &tot);
    const unsigned exz = block_exscan_lds(c != 0 ? 1u : 0u, s_red, &totz);
    if (in) {
        b.tstart[nxt][t] = base + ex;
        if (c)
            b.active[nxt][abase + exz] = (unsigned)t;
        if (t == g.ntiles - 1)
            b.tstart[nxt][g.ntiles] = base + ex + c;
    }
    s_pre[threadIdx.x] = ex;
    if (threadIdx.x == kBlock - 1)
        s_pre[kBlock] = ex + c;
    s_old[threadIdx.x] = (in && !dirty) ? tso : 0xffffffffu;
    if (threadIdx.x == 0)
        s_ndl = 0;
    lds_barrier();
    uint2* rec = b.rec[nxt];
    const uint2* orec = b.rec[cur];
    int j = 0;
    for (unsigned k0 = 0; k0 < tot; k0 += 4 * kBlock) {
        uint2 r[4];
        unsigned dst[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            unsigned k = k0 + u * kBlock + threadIdx.x;
            dst[u] = 0xffffffffu;
            if (k < tot) {
                while (s_pre[j + 1] <= k)
                    ++j;
                unsigned so = s_old[j];
                if (so != 0xffffffffu) {
                    r[u] = orec[so + (k - s_pre[j])];
                    dst[u] = base + k;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (dst[u] != 0xffffffffu)
                rec[dst[u]] = r[u];
    }
    if (g.dlistm) {
        // the block's dirty tiles from the flat list, one per wave in turn;
        // the first one's loads went out at the start
        if (item0 < ia1 && ctt0)
            wave_write_tile(g, b.lab, tt0, W[wv], hdr0, word0, rec, pbase0 + wave_sum_u(part0));
        for (unsigned item = item0 + kBlock / 64; item < ia1; item += kBlock / 64) {
            const unsigned tt = b.dflat[item];
            // every load of the tile is issued before any is used
            const unsigned ctt = b.tcnt[tt];
            const unsigned pbase = b.part_off[tt >> g.lgRe];
            const unsigned* slot = b.tslot + (size_t)tt * kSlotWords;
            const unsigned hdr = slot[0], word = slot[1 + lane];
            const int r0 = (int)(tt >> g.lgRe) << g.lgRe;
            unsigned part = 0;  // offset: the range's base plus the counts before tt in the range
            for (int k = r0 + lane; k < (int)tt; k += 64)
                part += b.tcnt[k];
            const unsigned o = pbase + wave_sum_u(part);
            if (ctt)
                wave_write_tile(g, b.lab, tt, W[wv], hdr, word, rec, o);
        }
        return;
    }
    // dirty tiles of this block's round-robin share are re-emitted from the labels
    const unsigned G = vb.n;
    const unsigned jd = vb.id + threadIdx.x * G;
    unsigned td;
    if (slot_tile(g, jd, td) && b.tcnt[td] && tile_dirty(b, td, epoch, all_dirty))
        s_dl[atomicAdd(&s_ndl, 1u)] = td;
    __syncthreads();
    const unsigned ndl = s_ndl;
    for (unsigned i = wv; i < ndl; i += kBlock / 64) {
        const unsigned tt = s_dl[i];
        const int r0 = (int)(tt >> g.lgRe) << g.lgRe;
        // offset of tile tt: its range's base plus the counts before it in the range
        unsigned part = 0;
        for (int k = r0 + lane; k < (int)tt; k += 64)
            part += b.tcnt[k];
        unsigned o = b.part_off[tt >> g.lgRe] + wave_sum_u(part);
        const unsigned* slot = b.tslot + (size_t)tt * kSlotWords;
        wave_write_tile(g, b.lab, tt, W[wv], slot[0], slot[1 + lane], rec, o);
    }
}

__global__ __launch_bounds__(kBlock) void k_write(Geom g, Bufs b, const void* img, int cur, int nxt,
                                                 const float* __restrict__ grad_sob,
                                                 const float* __restrict__ grad_l2, int flags, int all_dirty)
{
    write_body(g, b, img, cur, nxt, grad_sob, grad_l2, flags, all_dirty, VB{blockIdx.x, gridDim.x});
}

// --------------------------------------------------- L2 gradient per particle
//
// Energy change of one move a -> b at pixel x with value v (Eqs. (10)-(11)):
//   PC: n_b/(n_b+1) (v - mu_b)^2 - n_a/(n_a-1) (v - mu_a)^2   (means re-estimated)
//   PS: (v - m_b(x))^2 - (v - m_a(x))^2, m_l = mean of label l in the ball |y-x| <= R
//   + lambda (c_a - c_b), c_l = face neighbours with label l (contour length).
// Poisson pixel energy J - v log J of a move from expected intensity m_a to
// m_b, both held at their current values, J raised to at least 1e-6.
__device__ __forceinline__ float poisson_move(float v, float m_a, float m_b)
{
    const float ja = fmaxf(m_a, 1e-6f), jb = fmaxf(m_b, 1e-6f);
    return (jb - ja) - v * (logf(jb) - logf(ja));
}

// PSF: the deconvolving model (a compile-time switch keeps the plain path lean)
template <bool PSF>
__device__ __forceinline__ void l2diff_body(const Geom& g, const Bufs& b, const void* img, int cur, float* __restrict__ out, int gated, VB vb)
{
    DevState* ds = b.ds;
    if (gated && vb.id == 0 && threadIdx.x == 0) {
        ds->go = 0;
        ds->undo = 0;
        ds->epoch = ds->epoch + 1;
        ds->lmode = (ds->lmode & ~1u) | (ds->switch_it != 0 ? 1u : 0u);
    }
    if (gated && stopped(ds))
        return;
    if (!gated && fill_nan_after_rollback(b, cur, out, vb))
        return;
    unsigned n = ds->n[cur];
    const uint2* rec = b.rec[cur];
    unsigned p0, p1;
    xcd_chunk(n, vb, p0, p1);
    for (unsigned p = p0 + threadIdx.x; p < p1; p += kBlock) {
        uint2 r = rec[p];
        int x, y, z;
        unpack(g, r.x, x, y, z);
        int a = (int)(r.y & 0xffffu), bl = (int)(r.y >> 16);
        long long i = lin_of(g, x, y, z);
        float v = img_at(g, img, i);
        int ca = 0, cb = 0;
        {
            // face neighbours in the tile-major label copy: inside the tile a
            // fixed offset, across its border the facing pixel of the next tile
            const long long TX = 1ll << g.tsx, TXY = 1ll << (g.tsx + g.tsy), TV = 1ll << (g.tsx + g.tsy + g.tsz);
            const int lx = x & ((1 << g.tsx) - 1), ly = y & ((1 << g.tsy) - 1), lz = z & ((1 << g.tsz) - 1);
            const long long ti = (long long)tile_major(g, x, y, z);
            const long long sy = (long long)g.ntx * TV, sz = (long long)g.ntx * g.nty * TV;
#define SOBRC_FACE(cond, j)                    \
    if (cond) {                                \
        int l = b.labt[j];                     \
        ca += l == a;                          \
        cb += l == bl;                         \
    }
            SOBRC_FACE(x > 0, lx > 0 ? ti - 1 : ti - TV + (TX - 1))
            SOBRC_FACE(x + 1 < g.nx, lx < TX - 1 ? ti + 1 : ti + TV - (TX - 1))
            SOBRC_FACE(y > 0, ly > 0 ? ti - TX : ti - sy + (TXY - TX))
            SOBRC_FACE(y + 1 < g.ny, ly < (1 << g.tsy) - 1 ? ti + TX : ti + sy - (TXY - TX))
            SOBRC_FACE(z > 0, lz > 0 ? ti - TXY : ti - sz + (TV - TXY))
            SOBRC_FACE(z + 1 < g.nz, lz < (1 << g.tsz) - 1 ? ti + TXY : ti + sz - (TV - TXY))
#undef SOBRC_FACE
        }
        float dext;
        if (PSF) {
            // deconvolving model: delta^2 N(x) - 2 delta C(x), theta held fixed
            const float d = (float)(b.dtheta[bl] - b.dtheta[a]);
            dext = d * d * b.dN[i] - 2.f * d * b.dC[i];
        } else if (g.model == 0) {
            float4 sa = b.lstat[a], sb = b.lstat[bl];
            if (g.noise) {
                dext = poisson_move(v, sa.x, sb.x);
            } else {
                float da = v - sa.x, db = v - sb.x;
                dext = sb.z * db * db - sa.y * da * da;
            }
        } else {
            float sa = 0.f, sb = 0.f;
            int na = 0, nb = 0;
            int rz = g.ndim == 3 ? g.R : 0;
            for (int dz = -rz; dz <= rz; ++dz) {
                int zz = z + dz;
                if (zz < 0 || zz >= g.nz)
                    continue;
                for (int dy = -g.R; dy <= g.R; ++dy) {
                    int yy = y + dy;
                    if (yy < 0 || yy >= g.ny)
                        continue;
                    for (int dx = -g.R; dx <= g.R; ++dx) {
                        int xx = x + dx;
                        if (xx < 0 || xx >= g.nx || dx * dx + dy * dy + dz * dz > g.R2)
                            continue;
                        long long j = lin_of(g, xx, yy, zz);
                        int l = b.lab[j];
                        if (l == a) {
                            sa += img_at(g, img, j);
                            ++na;
                        } else if (l == bl) {
                            sb += img_at(g, img, j);
                            ++nb;
                        }
                    }
                }
            }
            float ma = sa / (float)na, mb = sb / (float)nb;
            dext = g.noise ? poisson_move(v, ma, mb) : (v - mb) * (v - mb) - (v - ma) * (v - ma);
        }
        const float dE = dext + g.lambda * (float)(ca - cb);
        out[p] = dE;
        if (b.dv)  // the brick kernels read the values by pixel (a scattered store: not kept in cache)
            __builtin_nontemporal_store(dE, b.dv + tile_major(g, x, y, z));
    }
}

template <bool PSF>
__global__ __launch_bounds__(kBlock) void k_l2diff(Geom g, Bufs b, const void* img, int cur, float* __restrict__ out,
                                                  int gated)
{
    l2diff_body<PSF>(g, b, img, cur, out, gated, VB{blockIdx.x, gridDim.x});
}

// PS model, tile-staged: one block per non-empty tile (the active-tile list,
// XCD-contiguous runs) copies the tile's box -- the tile and R pixels on every
// side, intensity and label of each pixel in one 8-byte entry -- into LDS
// once, and each of the tile's particles takes its PS ball sums and its
// face-neighbour counts from there.  Pixels outside the image carry the label
// kNone, which no particle's labels equal, so a ball row is walked over its
// whole half-width w (w^2 <= R^2 - dy^2 - dz^2) without per-pixel tests; the
// pixels that count are added in the same order as in the per-particle path
// above (the others add +0), so the sums are the same fp32 values.  The row
// half-widths are tabulated once per block.
__device__ __forceinline__ int isqrt_floor(int v)  // v >= 0
{
    int w = (int)sqrtf((float)v);
    while (w * w > v)
        --w;
    while ((w + 1) * (w + 1) <= v)
        ++w;
    return w;
}

__device__ __forceinline__ void l2diff_ps_tile_body(const Geom& g, const Bufs& b, const void* img, int cur,
                                                    float* __restrict__ out, int gated, VB vb)
{
    extern __shared__ __align__(16) char lds[];
    DevState* ds = b.ds;
    if (gated && vb.id == 0 && threadIdx.x == 0) {
        ds->go = 0;
        ds->undo = 0;
        ds->epoch = ds->epoch + 1;
        ds->lmode = (ds->lmode & ~1u) | (ds->switch_it != 0 ? 1u : 0u);
    }
    if (gated && stopped(ds))
        return;
    if (!gated && fill_nan_after_rollback(b, cur, out, vb))
        return;
    const int R = g.R, rz = g.ndim == 3 ? R : 0;
    const int TX = 1 << g.tsx, TY = 1 << g.tsy, TZ = 1 << g.tsz;
    const int BX = TX + 2 * R, BY = TY + 2 * R, BZ = TZ + 2 * rz, BXY = BX * BY;
    const int nbox = BX * BY * BZ;
    uint2* s_e = (uint2*)lds;  // (intensity bits, label)
    int* s_w = (int*)(s_e + nbox);  // half-width of ball row (dy, dz), -1 if empty
    const int nrow = (2 * R + 1) * (2 * rz + 1);
    for (int k = threadIdx.x; k < nrow; k += kBlock) {
        const int dy = k % (2 * R + 1) - R, dz = k / (2 * R + 1) - rz;
        const int rem = g.R2 - dy * dy - dz * dz;
        s_w[k] = rem < 0 ? -1 : isqrt_floor(rem);
    }
    unsigned a0, a1;
    xcd_chunk(ds->n_active[cur], vb, a0, a1);
    const unsigned* ts = b.tstart[cur];
    const uint2* rec = b.rec[cur];
    // box cell of this thread's first entry, and the step of kBlock entries
    // (divisions once per block; the box walk below only adds)
    const int bx0 = (int)threadIdx.x % BX, by0 = ((int)threadIdx.x / BX) % BY, bz0 = (int)threadIdx.x / BXY;
    const int sx = kBlock % BX, sy = (kBlock / BX) % BY, sz = kBlock / BXY;
    for (unsigned ai = a0; ai < a1; ++ai) {
        const unsigned t = b.active[cur][ai];
        const int tx = (int)(t % (unsigned)g.ntx), ty = (int)((t / (unsigned)g.ntx) % (unsigned)g.nty);
        const int tz = (int)(t / ((unsigned)g.ntx * (unsigned)g.nty));
        const int ox = tx * TX - R, oy = ty * TY - R, oz = tz * TZ - rz;
        const unsigned p0 = ts[t], p1 = ts[t + 1];
        __syncthreads();  // the previous tile is done with LDS
        // the box in passes of kPsPer entries per thread: every load of a pass
        // is issued before any entry is stored, so their latencies overlap
        constexpr int kPsPer = 8;
        int bx = bx0, by = by0, bz = bz0;
        for (int k0 = 0; k0 < nbox; k0 += kBlock * kPsPer) {
            float v[kPsPer];
            unsigned l[kPsPer];
#pragma unroll
            for (int u = 0; u < kPsPer; ++u) {
                const int k = k0 + u * kBlock + (int)threadIdx.x;
                const int x = ox + bx, y = oy + by, z = oz + bz;
                const bool in = k < nbox && x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
                const long long j = in ? lin_of(g, x, y, z) : 0;
                v[u] = in ? img_at(g, img, j) : 0.f;
                l[u] = in ? (unsigned)b.lab[j] : (unsigned)kNone;
                bx += sx;  // next entry: kBlock cells on (sx < BX, sy < BY: one carry each)
                const int cy = bx >= BX;
                bx -= cy ? BX : 0;
                by += sy + cy;
                const int cz = by >= BY;
                by -= cz ? BY : 0;
                bz += sz + cz;
            }
#pragma unroll
            for (int u = 0; u < kPsPer; ++u) {
                const int k = k0 + u * kBlock + (int)threadIdx.x;
                if (k < nbox)
                    s_e[k] = make_uint2(__float_as_uint(v[u]), l[u]);
            }
        }
        __syncthreads();
        for (unsigned p = p0 + threadIdx.x; p < p1; p += kBlock) {
            const uint2 r = rec[p];
            int x, y, z;
            unpack(g, r.x, x, y, z);
            const unsigned a = r.y & 0xffffu, bl = r.y >> 16;
            const int c = (x - ox) + BX * ((y - oy) + BY * (z - oz));
            const float v = __uint_as_float(s_e[c].x);
            int ca = 0, cb = 0;
#define SOBRC_FACE(cond, j)                    \
    if (cond) {                                \
        const unsigned l = s_e[j].y;           \
        ca += l == a;                          \
        cb += l == bl;                         \
    }
            SOBRC_FACE(x > 0, c - 1)
            SOBRC_FACE(x + 1 < g.nx, c + 1)
            SOBRC_FACE(y > 0, c - BX)
            SOBRC_FACE(y + 1 < g.ny, c + BX)
            SOBRC_FACE(z > 0, c - BXY)
            SOBRC_FACE(z + 1 < g.nz, c + BXY)
#undef SOBRC_FACE
            float sa = 0.f, sb = 0.f;
            int na = 0, nb = 0;
            for (int dz = -rz; dz <= rz; ++dz)
                for (int dy = -R; dy <= R; ++dy) {
                    const int w = s_w[(dy + R) + (2 * R + 1) * (dz + rz)];
                    if (w < 0)
                        continue;
                    const uint2* row = s_e + c + BX * (dy + BY * dz);
#pragma unroll 4
                    for (int dx = -w; dx <= w; ++dx) {
                        const uint2 e = row[dx];
                        const float val = __uint_as_float(e.x);
                        const bool ia = e.y == a, ib = e.y == bl;
                        sa += ia ? val : 0.f;
                        na += ia ? 1 : 0;
                        sb += ib ? val : 0.f;
                        nb += ib ? 1 : 0;
                    }
                }
            const float ma = sa / (float)na, mb = sb / (float)nb;
            const float dext = g.noise ? poisson_move(v, ma, mb) : (v - mb) * (v - mb) - (v - ma) * (v - ma);
            const float dE = dext + g.lambda * (float)(ca - cb);
            out[p] = dE;
            if (b.dv)
                __builtin_nontemporal_store(dE, b.dv + tile_major(g, x, y, z));
        }
    }
}

// Given L2 gradients (record order) to their pixels, for the brick kernels.
__global__ __launch_bounds__(kBlock) void k_dense_put(Geom g, Bufs b, int cur, const float* __restrict__ in)
{
    const unsigned n = b.ds->n[cur];
    const uint2* rec = b.rec[cur];
    for (unsigned p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) {
        int x, y, z;
        unpack(g, rec[p].x, x, y, z);
        __builtin_nontemporal_store(in[p], b.dv + tile_major(g, x, y, z));
    }
}

__global__ __launch_bounds__(kBlock) void k_l2diff_ps(Geom g, Bufs b, const void* img, int cur,
                                                     float* __restrict__ out, int gated)
{
    l2diff_ps_tile_body(g, b, img, cur, out, gated, VB{blockIdx.x, gridDim.x});
}

// ------------------------------------------------- Sobolev update, Eq. (6)
//
// One block per non-empty tile (the cell of the cell list); blocks are mapped
// to contiguous runs of the tile list per XCD so that neighbouring tiles share
// an L2.  The support of a core particle reaches h pixels beyond its tile.
//
// Brick kernels (one instantiation per dimension and halo h): when every
// particle in the tile's halo box carries the same unordered label pair
// {lo, hi} (so at most one particle per pixel), the box is laid out densely
// in LDS -- per pixel the value of an (lo -> hi) particle, the value of an
// (hi -> lo) particle, and both occupancy counts packed in one word -- and each
// core particle applies the compile-time stencil of all offsets with
// d^2 < (h+1)^2 to it: two FMAs and one integer add per tap give both sums of
// Eq. (6) and both set sizes.  Weights W[d^2] (0 outside the support) arrive as
// kernel arguments.
//
// Generic path (several label pairs in the box, or no brick kernel for this
// halo): the box's particles are staged in LDS in rounds and every core
// particle scans the staged set with exact integer distance tests.

__device__ void sob_generic_tile(const Geom& g, const Bufs& b, int cur, const float* __restrict__ in,
                                 float* __restrict__ out, unsigned t, char* lds)
{
    const int cap = g.stage_cap;
    unsigned* s_pos = (unsigned*)lds;
    unsigned* s_ab = s_pos + cap;
    float* s_v = (float*)(s_ab + cap);
    float* s_W = s_v + cap;
    unsigned* s_wtot = (unsigned*)(s_W + g.T);
    const unsigned* ts = b.tstart[cur];
    const uint2* rec = b.rec[cur];
    const int TX = 1 << g.tsx, TY = 1 << g.tsy, TZ = 1 << g.tsz;
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    __syncthreads();
    for (int k = threadIdx.x; k < g.T; k += kSobBlock)
        s_W[k] = b.W[k];
    int tx = (int)(t % (unsigned)g.ntx), ty = (int)((t / (unsigned)g.ntx) % (unsigned)g.nty);
    int tz = (int)(t / ((unsigned)g.ntx * (unsigned)g.nty));
    int bx0 = max(tx * TX - g.h, 0), bx1 = min(tx * TX + TX + g.h, g.nx);
    int by0 = max(ty * TY - g.h, 0), by1 = min(ty * TY + TY + g.h, g.ny);
    int bz0 = max(tz * TZ - g.h, 0), bz1 = min(tz * TZ + TZ + g.h, g.nz);
    int kx0 = bx0 >> g.tsx, nkx = ((bx1 - 1) >> g.tsx) - kx0 + 1;
    int ky0 = by0 >> g.tsy, nky = ((by1 - 1) >> g.tsy) - ky0 + 1;
    int kz0 = bz0 >> g.tsz, nkz = ((bz1 - 1) >> g.tsz) - kz0 + 1;
    int nnt = nkx * nky * nkz;
    unsigned cs = ts[t], ce = ts[t + 1];
    for (unsigned cb = cs; cb < ce; cb += kSobBlock) {
        unsigned p = cb + threadIdx.x;
        bool act = p < ce;
        int px = 0, py = 0, pz = 0;
        unsigned code = 0xffffffffu, swp = 0xffffffffu;
        if (act) {
            uint2 r = rec[p];
            unpack(g, r.x, px, py, pz);
            code = r.y;
            swp = (r.y >> 16) | (r.y << 16);
        }
        float s1 = 0.f, s2 = 0.f;
        int c1 = 0, c2 = 0;
        int k = 0;
        unsigned qs, qe;
        {
            unsigned nt = (unsigned)(kx0 + g.ntx * (ky0 + g.nty * kz0));
            qs = ts[nt];
            qe = ts[nt + 1];
        }
        for (;;) {
            int fill = 0;
            __syncthreads();
            while (k < nnt && fill <= cap - kSobBlock) {
                if (qs >= qe) {
                    ++k;
                    if (k < nnt) {
                        int kx = kx0 + k % nkx, ky = ky0 + (k / nkx) % nky, kz = kz0 + k / (nkx * nky);
                        unsigned nt = (unsigned)(kx + g.ntx * (ky + g.nty * kz));
                        qs = ts[nt];
                        qe = ts[nt + 1];
                    }
                    continue;
                }
                unsigned q = qs + threadIdx.x;
                bool inb = false;
                uint2 r = make_uint2(0u, 0u);
                float v = 0.f;
                if (q < qe) {
                    r = rec[q];
                    v = in[q];
                    int qx, qy, qz;
                    unpack(g, r.x, qx, qy, qz);
                    inb = qx >= bx0 && qx < bx1 && qy >= by0 && qy < by1 && qz >= bz0 && qz < bz1;
                }
                unsigned long long m = __ballot(inb);
                if (lane == 0)
                    s_wtot[wv] = (unsigned)__popcll(m);
                __syncthreads();
                unsigned off = 0, tot = 0;
                for (int i = 0; i < kSobBlock / 64; ++i) {
                    unsigned c = s_wtot[i];
                    off += i < wv ? c : 0;
                    tot += c;
                }
                if (inb) {
                    int slot = fill + (int)(off + lanes_below(m));
                    s_pos[slot] = r.x;
                    s_ab[slot] = r.y;
                    s_v[slot] = v;
                }
                fill += (int)tot;
                qs += kSobBlock;
                __syncthreads();
            }
            __syncthreads();
            if (act) {
                for (int j = 0; j < fill; ++j) {
                    int qx, qy, qz;
                    unpack(g, s_pos[j], qx, qy, qz);
                    int dx = qx - px, dy = qy - py, dz = qz - pz;
                    int d2 = dx * dx + dy * dy + dz * dz;
                    if (d2 < g.T) {
                        unsigned qab = s_ab[j];
                        float wv_ = s_W[d2] * s_v[j];
                        if (qab == code) {
                            s1 += wv_;
                            ++c1;
                        } else if (qab == swp) {
                            s2 += wv_;
                            ++c2;
                        }
                    }
                }
            }
            if (k >= nnt)
                break;
        }
        if (act) {
            float res = s1 / (float)c1;
            if (c2)
                res -= s2 / (float)c2;
            out[p] = res;
        }
    }
}

__device__ __forceinline__ void sobolev_generic_body(const Geom& g, const Bufs& b, int cur, const float* __restrict__ in, float* __restrict__ out, int gated, VB vb)
{
    extern __shared__ __align__(16) char lds[];
    if ((gated & kGate) && stopped(b.ds))
        return;
    if ((gated & kAuto) && (b.ds->lmode & 1u))
        return;  // L2 gradients in force: no smoothing
    if (!(gated & kGate) && fill_nan_after_rollback(b, cur, out, vb))
        return;
    unsigned a0, a1;
    xcd_chunk(b.ds->n_active[cur], vb, a0, a1);
    for (unsigned ai = a0; ai < a1; ++ai)
        sob_generic_tile(g, b, cur, in, out, b.active[cur][ai], lds);
}

__global__ __launch_bounds__(kSobBlock) void k_sobolev_generic(Geom g, Bufs b, int cur,
                                                              const float* __restrict__ in,
                                                              float* __restrict__ out, int gated)
{
    sobolev_generic_body(g, b, cur, in, out, gated, VB{blockIdx.x, gridDim.x});
}

constexpr int kTapGroup = 16;  // brick reads the stencil keeps in flight

template <int ND, int H, int WIDE>
struct BrickShape {
    static constexpr int TX = tile_ex(ND, WIDE), TY = tile_ey(ND, WIDE), TZ = tile_ez(ND);
    static constexpr int HZ = ND == 3 ? H : 0;
    static constexpr int BX = TX + 2 * H, BY = TY + 2 * H, BZ = TZ + 2 * HZ;
    // odd row stride: the rows of a tile then fall on distinct LDS banks
    // (a stride that is a multiple of 4 puts all (y, z) rows of a plane on
    // 8 of the 32 bank pairs, so a surface with one particle per row
    // conflicts 4-8 ways on every tap)
    static constexpr int SX = BX | 1;
    static constexpr int NCELL = SX * BY * BZ;
    static constexpr int LIM = (H + 1) * (H + 1);
    // half-width of the support in box row (dy, dz) when the support is
    // d^2 < (H + 1)^2: the largest k with k^2 + dy^2 + dz^2 < LIM, -1 if none
    static constexpr int full_w(int dy, int dz)
    {
        int w = -1;
        while (w + 1 <= H && (w + 1) * (w + 1) + dy * dy + dz * dz < LIM)
            ++w;
        return w;
    }
    static constexpr int count()
    {
        int n = 0;
        for (int dz = -HZ; dz <= HZ; ++dz)
            for (int dy = -H; dy <= H; ++dy)
                for (int dx = -H; dx <= H; ++dx)
                    n += dx * dx + dy * dy + dz * dz < LIM;
        return n;
    }
    static constexpr int NT = count();
};

template <int NT>
struct TapList {
    int off[NT];  // cell offset from the corner of the (2h+1)^d cube
    int d2[NT];
};

template <int ND, int H, int WIDE>
constexpr TapList<BrickShape<ND, H, WIDE>::NT> make_taps()
{
    using S = BrickShape<ND, H, WIDE>;
    TapList<S::NT> t{};
    int k = 0;
    for (int dz = -S::HZ; dz <= S::HZ; ++dz)
        for (int dy = -H; dy <= H; ++dy)
            for (int dx = -H; dx <= H; ++dx) {
                int d2 = dx * dx + dy * dy + dz * dz;
                if (d2 < S::LIM) {
                    t.off[k] = (dx + H) + S::SX * ((dy + H) + S::BY * (dz + S::HZ));
                    t.d2[k] = d2;
                    ++k;
                }
            }
    return t;
}

// Tiles active[cur][a0 .. a1) of one context through the brick kernel (the
// tile loop stays inside this function: the compiler keeps its registers
// lean that way).
template <int ND, int H, bool FULL, int WIDE>
__device__ __forceinline__ void brick_range(const Geom& g, const Bufs& b, const SobW& sw, int cur,
                                            const float* __restrict__ in, float* __restrict__ out, int gated,
                                            unsigned a0, unsigned a1)
{
    using S = BrickShape<ND, H, WIDE>;
    constexpr TapList<S::NT> taps = make_taps<ND, H, WIDE>();
    constexpr int NCORE = S::TX * S::TY * S::TZ;
    __shared__ __align__(16) char lds[brick_lds_bytes(ND, H, WIDE)];
    // own particles: brick corner cell (12 bits) | x in tile << 12 | box row of
    // the corner << 17 | side A << 31
    __shared__ unsigned s_core[NCORE];
    __shared__ unsigned s_mode, s_ncore, s_cs;
    constexpr int NROWS = S::BY * S::BZ;
    // One box row per thread.  Its L2 values come from the per-pixel field in
    // aligned 16-byte chunks: CL chunks left of the tile row, NCH in all, box
    // x = 0 at element X0 of that window.  Its particle and side bits come
    // from the slot words of the three tile rows it crosses.
    constexpr int CL = (H + 3) / 4;
    constexpr int NCH = CL + (S::TX - 1 + H) / 4 + 1;
    constexpr int X0 = 4 * CL - H;
    static_assert(NROWS <= kSobBlock, "one box row per thread");
    static_assert(S::TX % 4 == 0 && H <= S::TX && S::BX <= 32, "chunks of one tile row, three tile rows per box row");
    static_assert(S::NCELL * 8 + NROWS * 8 <= brick_lds_bytes(ND, H, WIDE), "brick does not fit its LDS");
    // fields of a core entry: corner cells and rows of the tile's own pixels;
    // the support window of a row fits one 32-bit mask
    static_assert((S::TX - 1) + S::SX * ((S::TY - 1) + S::BY * (S::TZ - 1)) < 4096 &&
                      (S::TY - 1) + S::BY * (S::TZ - 1) < 512 && S::TX <= 32 && S::BX <= 32,
                  "core entry fields");
    float2* s_v = (float2*)lds;               // (value of a lo->hi particle, value of a hi->lo particle)
    uint2* s_m = (uint2*)(s_v + S::NCELL);    // per box row: bits of lo->hi particles, of hi->lo particles
    DevState* ds = b.ds;
    if ((gated & kGate) && stopped(ds))
        return;
    if ((gated & kAuto) && (ds->lmode & 1u))
        return;  // L2 gradients in force: no smoothing
    const unsigned* ts = b.tstart[cur];
    const float* __restrict__ dv = b.dv;
    const int lane = lane_id();
    const int rr = (int)threadIdx.x;  // this thread's box row
    const int ryi = rr % S::BY, rzi = rr / S::BY;
    for (unsigned ai = a0; ai < a1; ++ai) {
        const unsigned t = b.active[cur][ai];
        const int tx = (int)(t % (unsigned)g.ntx), ty = (int)((t / (unsigned)g.ntx) % (unsigned)g.nty);
        const int tz = (int)(t / ((unsigned)g.ntx * (unsigned)g.nty));
        const int ox = tx * S::TX - H, oy = ty * S::TY - H, oz = tz * S::TZ - S::HZ;
        const int bx0 = max(ox, 0), bx1 = min(ox + S::BX, g.nx);
        const int by0 = max(oy, 0), by1 = min(oy + S::BY, g.ny);
        const int bz0 = max(oz, 0), bz1 = min(oz + S::BZ, g.nz);
        const int kx0 = bx0 / S::TX, nkx = (bx1 - 1) / S::TX - kx0 + 1;
        const int ky0 = by0 / S::TY, nky = (by1 - 1) / S::TY - ky0 + 1;
        const int kz0 = bz0 / S::TZ, nkz = (bz1 - 1) / S::TZ - kz0 + 1;
        // neighbour tiles k = kxi + 3 (kyi + 3 kzi), kxi < nkx, kyi < nky, kzi < nkz
        const int kown = (tx - kx0) + 3 * ((ty - ky0) + 3 * (tz - kz0));
        if (ai != a0)
            __syncthreads();  // the previous tile is done with LDS
        // One round trip: the box row's slot words and L2 chunks, and (the last wave)
        // the neighbour tiles' record ranges and label pairs and the tile's
        // own rows.  A row word of a tile without particles is zero, and the
        // per-pixel field holds the current L2 value at every particle, so the
        // row needs nothing else; pixels that are not particles are masked.
        const int y = oy + ryi, z = oz + rzi;
        const bool rin = rr < NROWS && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
        const int yc = rin ? y : 0, zc = rin ? z : 0;
        const unsigned trow = (unsigned)g.ntx * ((unsigned)(yc / S::TY) + (unsigned)g.nty * (unsigned)(zc / S::TZ));
        const int lrow = (yc % S::TY) + S::TY * (zc % S::TZ);
        unsigned wd[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int kx = tx - 1 + k;
            const bool ok = rin && kx >= 0 && kx < g.ntx;
            wd[k] = ok ? b.tslot[(size_t)(trow + (unsigned)kx) * kSlotWords + 1 + lrow] : 0u;
        }
        float4 ch[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int e = 4 * (c - CL);  // x of the chunk's first pixel, from the tile's
            const int kxo = e < 0 ? -1 : e / S::TX;
            const int kx = tx + kxo;
            const bool ok = rin && kx >= 0 && kx < g.ntx;
            ch[c] = ok ? *(const float4*)(dv + (size_t)(trow + (unsigned)kx) * NCORE + (e - kxo * S::TX) + S::TX * lrow)
                       : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        // the last wave (fewest box rows): label pairs of the neighbour tiles
        // (slot headers) and the tile's own rows for the core list
        unsigned hdr = 0u, nb_beg = 0u, nb_end = 0u, own_word = 0u, own_pre = 0u;
        if (threadIdx.x >= kSobBlock - 64) {
            const int kxi = lane % 3, kyi = (lane / 3) % 3, kzi = lane / 9;
            if (kxi < nkx && kyi < nky && kzi < nkz) {
                const int kx = kx0 + kxi, ky = ky0 + kyi, kz = kz0 + kzi;
                const unsigned tile = (unsigned)(kx + g.ntx * (ky + g.nty * kz));
                nb_beg = ts[tile];
                nb_end = ts[tile + 1];
                hdr = b.tslot[(size_t)tile * kSlotWords];
            }
            if (lane < S::TY * S::TZ) {
                const unsigned* sl = b.tslot + (size_t)t * kSlotWords;
                own_word = sl[1 + lane];
                own_pre = sl[1 + kSlotRows + lane];
            }
        }
        if (rr < NROWS) {
            // particle and lo-side bits of the three tile rows (x from (tx - 1) * TX),
            // then the box row's window of them
            const unsigned long long tm = (1ull << S::TX) - 1ull;
            unsigned long long pw = 0ull, lw = 0ull;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                pw |= ((unsigned long long)wd[k] & tm) << (k * S::TX);
                lw |= ((unsigned long long)(wd[k] >> 16) & tm) << (k * S::TX);
            }
            const unsigned bm = (unsigned)((1ull << S::BX) - 1ull);
            const unsigned mp = (unsigned)(pw >> (S::TX - H)) & bm, ml = (unsigned)(lw >> (S::TX - H)) & bm;
            const unsigned mA = mp & ml, mB = mp & ~ml;
            s_m[rr] = make_uint2(mA, mB);
            float2* row = s_v + S::SX * rr;
#pragma unroll
            for (int i = 0; i < S::BX; ++i) {
                const int e = X0 + i;
                const float4 q = ch[e >> 2];
                const float v = (e & 3) == 0 ? q.x : (e & 3) == 1 ? q.y : (e & 3) == 2 ? q.z : q.w;
                row[i] = make_float2(((mA >> i) & 1u) ? v : 0.f, ((mB >> i) & 1u) ? v : 0.f);
            }
        }
        if (threadIdx.x >= kSobBlock - 64) {
            // several label pairs around this tile: the staged generic scan
            const unsigned own_hdr = __shfl(hdr, kown);
            const bool has = nb_end > nb_beg;
            const bool bad = has && (hdr != own_hdr || (hdr & 0xffffu) == 0xffffu);
            const bool any_bad = __ballot(bad) != 0;
            const unsigned cs0 = __shfl(nb_beg, kown), ncore0 = __shfl(nb_end, kown) - cs0;
            // the tile's own particles, in record order, as (brick corner cell, side)
            unsigned pbits = own_word & 0xffffu;
            const unsigned own = own_word >> 16;
            const int ly = lane % S::TY, lz = lane / S::TY;
            unsigned pre = own_pre;
            const unsigned row0 = (unsigned)(ly + S::BY * lz);
            while (pbits) {
                const int lx = __ffs(pbits) - 1;
                pbits &= pbits - 1;
                s_core[pre++] = (unsigned)(lx + S::SX * (ly + S::BY * lz)) | ((unsigned)lx << 12) | (row0 << 17) |
                                (((own >> lx) & 1u) << 31);
            }
            if (lane == 0) {
                s_mode = any_bad ? 1u : 0u;
                s_ncore = ncore0;
                s_cs = cs0;
            }
        }
        __syncthreads();
        if (s_mode) {
            sob_generic_tile(g, b, cur, in, out, t, lds);
            continue;
        }
        const unsigned cs = s_cs, ncore = s_ncore;
        for (unsigned e = threadIdx.x; e < ncore; e += kSobBlock) {
            const unsigned ce = s_core[e];
            const int c0 = (int)(ce & 0xfffu), lx = (int)((ce >> 12) & 31u), row0 = (int)((ce >> 17) & 0x1ffu);
            const bool sideA = (ce >> 31) != 0;
            const float2* vb = s_v + c0;
            float sA = 0.f, sB = 0.f;
            // taps in groups: the scheduler may not hoist every brick read
            // ahead of the arithmetic (that costs registers, so occupancy)
#pragma unroll
            for (int q0 = 0; q0 < S::NT; q0 += kTapGroup) {
#pragma unroll
                for (int q = q0; q < (q0 + kTapGroup < S::NT ? q0 + kTapGroup : S::NT); ++q) {
                    const float2 cv = vb[taps.off[q]];
                    const float wk = sw.w[taps.d2[q]];
                    sA = fmaf(wk, cv.x, sA);
                    sB = fmaf(wk, cv.y, sB);
                }
                __asm__ volatile("" ::: "memory");  // no brick read moves across a group
            }
            // |Q_p| and |Q'_p|: particles of each side in the support, a window
            // of every support row's side masks
            unsigned nA = 0u, nB = 0u;
#pragma unroll
            for (int dz = -S::HZ; dz <= S::HZ; ++dz)
#pragma unroll
                for (int dy = -H; dy <= H; ++dy) {
                    // a row outside the support (w < 0) gets an empty window: no branch,
                    // so the row reads of one particle issue together.  With every
                    // offset of the box inside the support (FULL) the half-widths
                    // are compile-time constants and empty rows are not read.
                    if (FULL && S::full_w(dy, dz) < 0)
                        continue;
                    const int w = FULL ? S::full_w(dy, dz) : sw.rw[(dy + H) + (2 * H + 1) * (dz + S::HZ)];
                    const unsigned wm = w >= 0 ? (2u << (2 * w)) - 1u : 0u;
                    const uint2 m = s_m[row0 + (dy + H) + S::BY * (dz + S::HZ)];
                    const unsigned win = wm << (lx + H - (w >= 0 ? w : 0));
                    nA += (unsigned)__popc(m.x & win);
                    nB += (unsigned)__popc(m.y & win);
                }
            const float same = sideA ? sA : sB, other = sideA ? sB : sA;
            const unsigned nS = sideA ? nA : nB, nO = sideA ? nB : nA;
            float res = same / (float)nS;
            if (nO)
                res -= other / (float)nO;
            out[cs + e] = res;
        }
    }
}

template <int ND, int H, bool FULL, int WIDE>
__device__ __forceinline__ void sobolev_brick_body(const Geom& g, const Bufs& b, const SobW& sw, int cur, const float* __restrict__ in, float* __restrict__ out, int gated, VB vb)
{
    if (!(gated & kGate) && fill_nan_after_rollback(b, cur, out, vb))
        return;
    unsigned a0, a1;
    xcd_chunk(b.ds->n_active[cur], vb, a0, a1);
    brick_range<ND, H, FULL, WIDE>(g, b, sw, cur, in, out, gated, a0, a1);
}

template <int ND, int H, bool FULL, int WIDE>
__global__ __launch_bounds__(kSobBlock) void k_sobolev_brick(Geom g, Bufs b, SobW sw, int cur,
                                                            const float* __restrict__ in,
                                                            float* __restrict__ out, int gated)
{
    sobolev_brick_body<ND, H, FULL, WIDE>(g, b, sw, cur, in, out, gated, VB{blockIdx.x, gridDim.x});
}

// ------------------------------------------------------- acceptance of moves
//
// Every particle with gradient < 0 is a candidate; per pixel the smallest
// gradient wins (ties: first in order, i.e. smaller b).  Decisions read only
// gradients and records of state t, so the label field is updated in place.
// Region statistics follow exactly (integer deltas): per-block partials for
// few labels, wave-merged atomics otherwise.  Tiles within one pixel of a
// flip are marked dirty for the particle-set update.
// TOPO: the moves were decided by the ranked acceptance (compile-time switch)
template <bool TOPO>
__device__ __forceinline__ void flip_body(const Geom& g, const Bufs& b, const void* img, int cur, const float* __restrict__ grad_sob, const float* __restrict__ grad_l2, int flags, VB vb)
{
    __shared__ long long s_dn[kSmallM], s_dq[kSmallM];
    __shared__ unsigned s_f, s_rv;
    DevState* ds = b.ds;
    if (stopped(ds))
        return;
    if (threadIdx.x < kSmallM) {
        s_dn[threadIdx.x] = 0;
        s_dq[threadIdx.x] = 0;
    }
    if (threadIdx.x == 0) {
        s_f = 0;
        s_rv = 0;
    }
    if (TOPO && vb.id == 0 && threadIdx.x <= (unsigned)kTopoRounds)
        ds->topo_cnt[threadIdx.x] = 0;  // the ranked acceptance of this step is done
    __syncthreads();
    const unsigned n = ds->n[cur];
    const unsigned epoch = ds->epoch, it = ds->iters;
    const float* grad = ((flags & kAuto) && (ds->lmode & 1u)) ? grad_l2 : grad_sob;
    const uint2* rec = b.rec[cur];
    const int lane = lane_id();
    const int TX = 1 << g.tsx, TY = 1 << g.tsy, TZ = 1 << g.tsz;
    unsigned p0, p1;
    xcd_chunk(n, vb, p0, p1);
    for (unsigned base = p0; base < p1; base += kBlock) {
        unsigned p = base + threadIdx.x;
        bool f = false, rev = false;
        unsigned lin = 0;
        int a = 0, bb = 0;
        if (p < p1) {
            uint2 r;
            bool mv;
            if (TOPO) {
                // decided by the ranked acceptance; its per-pixel words are cleared here
                const unsigned char st = b.tstate[p];
                r = rec[p];
                bb = (int)(r.y >> 16);
                mv = st == 2;
                if (st != 0) {
                    int xx, yy, zz;
                    unpack(g, r.x, xx, yy, zz);
                    b.pmap[lin_of(g, xx, yy, zz)] = ~0ull;
                }
            } else {
                mv = decide_move(rec, grad, n, p, r, bb);
            }
            if (mv) {
                f = true;
                int x, y, z;
                unpack(g, r.x, x, y, z);
                lin = (unsigned)lin_of(g, x, y, z);
                a = (int)(r.y & 0xffffu);
                b.lab[lin] = (unsigned short)bb;
                b.labt[tile_major(g, x, y, z)] = (unsigned short)bb;
                const unsigned st = b.fstamp[lin];
                rev = st != 0u && st == it;  // this pixel also changed in the previous iteration
                b.fstamp[lin] = it + 1u;
                int tx = x >> g.tsx, ty = y >> g.tsy, tz = z >> g.tsz;
                int lx = x & (TX - 1), ly = y & (TY - 1), lz = z & (TZ - 1);
                int x0 = (lx == 0 && tx > 0) ? -1 : 0, x1 = (lx == TX - 1 && tx + 1 < g.ntx) ? 1 : 0;
                int y0 = (ly == 0 && ty > 0) ? -1 : 0, y1 = (ly == TY - 1 && ty + 1 < g.nty) ? 1 : 0;
                int z0 = (lz == 0 && tz > 0) ? -1 : 0, z1 = (lz == TZ - 1 && tz + 1 < g.ntz) ? 1 : 0;
                for (int dz = z0; dz <= z1; ++dz)
                    for (int dy = y0; dy <= y1; ++dy)
                        for (int dx = x0; dx <= x1; ++dx)
                            b.dirty[(tx + dx) + g.ntx * ((ty + dy) + g.nty * (tz + dz))] = epoch;
            }
        }
        unsigned long long m = __ballot(f);
        if (m == 0)
            continue;
        int leader = __ffsll((long long)m) - 1;
        const unsigned long long mr = __ballot(rev);
        if (lane == leader) {
            atomicAdd(&s_f, (unsigned)__popcll(m));
            if (mr)
                atomicAdd(&s_rv, (unsigned)__popcll(mr));
        }
        long long q = f ? qvalue(g, img, lin) : 0;
        unsigned key = f ? ((unsigned)min(a, bb) | ((unsigned)max(a, bb) << 16)) : 0u;
        long long sgn = bb > a ? 1 : -1;  // +1: move from the smaller to the larger label
        bool pend = f;
        unsigned long long mm;
        while ((mm = __ballot(pend)) != 0) {
            int l2 = __ffsll((long long)mm) - 1;
            unsigned k = __shfl(key, l2);
            bool match = pend && key == k;
            long long dn = wave_sum_ll(match ? sgn : 0);
            long long dq = wave_sum_ll(match ? sgn * q : 0);
            if (lane == l2) {
                int lo = (int)(k & 0xffffu), hi = (int)(k >> 16);
                if (g.small_m) {
                    atomicAdd((unsigned long long*)&s_dn[hi], (unsigned long long)dn);
                    atomicAdd((unsigned long long*)&s_dn[lo], (unsigned long long)(-dn));
                    atomicAdd((unsigned long long*)&s_dq[hi], (unsigned long long)dq);
                    atomicAdd((unsigned long long*)&s_dq[lo], (unsigned long long)(-dq));
                } else {
                    atomicAdd((unsigned long long*)&b.st_n[hi], (unsigned long long)dn);
                    atomicAdd((unsigned long long*)&b.st_n[lo], (unsigned long long)(-dn));
                    atomicAdd((unsigned long long*)&b.st_s1[hi], (unsigned long long)dq);
                    atomicAdd((unsigned long long*)&b.st_s1[lo], (unsigned long long)(-dq));
                }
            }
            pend = pend && !match;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        b.part_f[vb.id] = s_f;
        b.part_f[vb.n + vb.id] = s_rv;
    }
    if (g.small_m && (int)threadIdx.x < g.max_labels) {
        b.part_n[(long long)threadIdx.x * vb.n + vb.id] = s_dn[threadIdx.x];
        b.part_q[(long long)threadIdx.x * vb.n + vb.id] = s_dq[threadIdx.x];
    }
}

template <bool TOPO>
__global__ __launch_bounds__(kBlock) void k_flip(Geom g, Bufs b, const void* img, int cur,
                                                const float* __restrict__ grad_sob,
                                                const float* __restrict__ grad_l2, int flags)
{
    flip_body<TOPO>(g, b, img, cur, grad_sob, grad_l2, flags, VB{blockIdx.x, gridDim.x});
}

// ------------------------------------- ranked acceptance, topological control
//
// Candidates (gradient < 0) run in the order of (gradient, pixel, target
// label); a move is executed only if its pixel still has the label it started
// from and is a simple point of the foreground regions it leaves and joins
// (26/6 connectivity, 8/4 in 2D; label 0 is not controlled).  The sequential
// result is reproduced exactly in parallel: a candidate is decided as soon as
// every candidate ranked before it within its 3x3(x3) neighbourhood has been
// decided.  Its decision reads only labels of that neighbourhood, which are
// final for it by then, and two candidates decided together never lie in each
// other's neighbourhood.
//
// Per candidate pixel a word holds the smallest undecided key (orderable
// gradient << 16 | target label) and the pixel's current label.  Each word is
// a complete state of its pixel: when its key ranks after a candidate, its
// label is final for that candidate, whenever it was read.  Each block stages
// a tile with its one-pixel halo in LDS and decides, in local rounds, what its
// staged words allow; round launches take the tiles with undecided candidates
// left, and after kTopoRounds launches one block finishes the rest.

constexpr unsigned long long kKeyInf = 0xFFFFFFFFFFFFull;  // 48-bit key of a pixel with no undecided candidate
constexpr int kTopoBox = 1000;                            // 10^3 box (3D); 18^2 = 324 in 2D
constexpr int kTopoCand = 512;                            // candidates of a tile staged in LDS
// per-iteration tile stamp, odd so that a cleared mark (0) never matches
__device__ __forceinline__ unsigned topo_stamp(unsigned it) { return (it << 1) | 1u; }

// gradients < 0: the more negative, the smaller the key; ties by target label
__device__ __forceinline__ unsigned long long cand_key(float gv, int bb)
{
    return ((unsigned long long)(~__float_as_uint(gv)) << 16) | (unsigned)bb;
}

// 3x3(x3) neighbourhood as a bit set: bit k = (dx+1) + 3(dy+1) [+ 9(dz+1)]
template <int ND>
struct NbBits {
    static constexpr int N = ND == 3 ? 27 : 9;
    static constexpr int CENTRE = N / 2;
    static constexpr unsigned ALL = (1u << N) - 1u;
    static constexpr int dist(int k)  // number of non-zero offsets
    {
        return (k % 3 != 1) + ((k / 3) % 3 != 1) + (ND == 3 ? (k / 9 != 1) : 0);
    }
    static constexpr unsigned x_at(int xi)
    {
        unsigned m = 0;
        for (int k = 0; k < N; ++k)
            if (k % 3 == xi)
                m |= 1u << k;
        return m;
    }
    static constexpr unsigned y_at(int yi)
    {
        unsigned m = 0;
        for (int k = 0; k < N; ++k)
            if ((k / 3) % 3 == yi)
                m |= 1u << k;
        return m;
    }
    static constexpr unsigned faces()
    {
        unsigned m = 0;
        for (int k = 0; k < N; ++k)
            if (dist(k) == 1)
                m |= 1u << k;
        return m;
    }
    // where the complement is examined: 18-neighbourhood (3D), 8 (2D)
    static constexpr unsigned bg_domain()
    {
        unsigned m = 0;
        for (int k = 0; k < N; ++k)
            if (dist(k) >= 1 && (ND == 2 || dist(k) <= 2))
                m |= 1u << k;
        return m;
    }
};

// one step of growth under full (8/26) or face (4/6) adjacency
template <int ND>
__device__ __forceinline__ unsigned grow_full(unsigned s)
{
    using M = NbBits<ND>;
    // each axis step keeps to the N bits: a bit shifted past the top would
    // come back into range with the next axis' right shift
    s = (s | ((s << 1) & ~M::x_at(0)) | ((s >> 1) & ~M::x_at(2))) & M::ALL;
    s = (s | ((s << 3) & ~M::y_at(0)) | ((s >> 3) & ~M::y_at(2))) & M::ALL;
    if (ND == 3)
        s = (s | (s << 9) | (s >> 9)) & M::ALL;
    return s;
}

template <int ND>
__device__ __forceinline__ unsigned grow_face(unsigned s)
{
    using M = NbBits<ND>;
    unsigned r = s | ((s << 1) & ~M::x_at(0)) | ((s >> 1) & ~M::x_at(2)) | ((s << 3) & ~M::y_at(0)) |
                 ((s >> 3) & ~M::y_at(2));
    if (ND == 3)
        r |= (s << 9) | (s >> 9);
    return r & M::ALL;
}

// Simple point: m = the neighbours (centre excluded) inside the region.  The
// region's part of the neighbourhood is one full-adjacency component, and the
// complement's face-adjacency components within the 18- (8-) neighbourhood
// that touch a face neighbour are exactly one.
template <int ND>
__device__ __forceinline__ bool simple_point(unsigned m)
{
    using M = NbBits<ND>;
    if (m == 0)
        return false;
    unsigned c = m & (0u - m), p;
    do {
        p = c;
        c = grow_full<ND>(c) & m;
    } while (c != p);
    if (c != m)
        return false;
    const unsigned dom = ~m & M::bg_domain();
    const unsigned f = dom & M::faces();
    if (f == 0)
        return false;
    c = f & (0u - f);
    do {
        p = c;
        c = grow_face<ND>(c) & dom;
    } while (c != p);
    return (f & ~c) == 0;
}

// Per-pixel words are read and written at device scope, so that blocks on
// other XCDs see a word soon after it is stored.
__device__ __forceinline__ unsigned long long word_load(const unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void word_store(unsigned long long* p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Decide what can be decided of tile t from the per-pixel words of the tile
// and its halo, in local rounds on LDS; the tile's own words are written
// back.  Returns (block-uniform) whether undecided candidates remain.
// A tile's undecided candidates during its local rounds (LDS).
struct TopoCand {
    unsigned n;
    unsigned p[kTopoCand];              // record index
    unsigned rw[kTopoCand];             // a | b << 16
    unsigned long long key[kTopoCand];  // rank key
    unsigned short cell[kTopoCand];     // box cell
    unsigned char st[kTopoCand];        // 1 undecided, 2 executed, 3 refused
};

template <int ND>
__device__ bool topo_tile(const Geom& g, const Bufs& b, int cur, unsigned t, const float* __restrict__ grad,
                          unsigned long long* words, unsigned short* s_lab, unsigned long long* s_key, TopoCand& C)
{
    using M = NbBits<ND>;
    const TileInfo ti = tile_info(g, t);
    const int nbox = ti.BX * ti.BY * ti.BZ, BXY = ti.BX * ti.BY;
    const int ox = ti.tx * ti.TX - 1, oy = ti.ty * ti.TY - 1, oz = ti.tz * ti.TZ - ti.hz;
    // the tile's record range and the box's words and labels in one round
    // trip: every load is issued before any is used (a pixel's label is
    // loaded beside its word and kept if the word carries none)
    const unsigned r0 = b.tstart[cur][t], r1 = b.tstart[cur][t + 1];
    constexpr int kPer = (kTopoBox + kBlock - 1) / kBlock;  // box cells per thread
    unsigned long long wv[kPer];
    unsigned short lv[kPer];
    bool inb[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int k = (int)threadIdx.x + u * kBlock;
        const int bx = k % ti.BX, by = (k / ti.BX) % ti.BY, bz = k / BXY;
        const int x = ox + bx, y = oy + by, z = oz + bz;
        inb[u] = k < nbox && x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
        wv[u] = 0ull;
        lv[u] = kNone;
        if (inb[u]) {
            const long long i = lin_of(g, x, y, z);
            wv[u] = word_load(words + i);
            lv[u] = b.lab[i];
        }
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int k = (int)threadIdx.x + u * kBlock;
        if (k < nbox) {
            const unsigned long long w = wv[u];
            s_lab[k] = !inb[u] ? kNone : (w & 0xFFFFu) != 0xFFFFu ? (unsigned short)(w & 0xFFFFu) : lv[u];
            s_key[k] = inb[u] ? w >> 16 : kKeyInf;
        }
    }
    __syncthreads();
    const uint2* rec = b.rec[cur];
    auto cell_of = [&](unsigned pos) {
        int x, y, z;
        unpack(g, pos, x, y, z);
        return (x - ox) + ti.BX * ((y - oy) + ti.BY * (z - oz));
    };
    auto nb_off = [&](int k) {
        return (k % 3 - 1) + ti.BX * ((k / 3) % 3 - 1) + (ND == 3 ? BXY * (k / 9 - 1) : 0);
    };
    // one undecided candidate: 0 while a candidate ranked before it is
    // undecided within its neighbourhood, else 2 (executed) or 3 (refused)
    auto decide = [&](unsigned rw, int c, unsigned long long kc) -> unsigned char {
        if (s_key[c] != kc)
            return 0;  // an undecided move of this pixel ranks first
        const unsigned gc = (unsigned)(kc >> 16);
        bool ready = true;  // all neighbours read: no branch per neighbour
#pragma unroll
        for (int k = 0; k < M::N; ++k) {
            if (k == M::CENTRE)
                continue;
            const unsigned gy = (unsigned)(s_key[c + nb_off(k)] >> 16);
            // a neighbour ranks first: smaller gradient, or equal and earlier in raster order
            ready = ready && !(gy < gc || (gy == gc && k < M::CENTRE));
        }
        if (!ready)
            return 0;
        const int a = (int)(rw & 0xFFFFu), bb = (int)(rw >> 16);
        bool ok = s_lab[c] == a;
        if (ok) {
            unsigned ma = 0, mb = 0;
#pragma unroll
            for (int k = 0; k < M::N; ++k) {
                if (k == M::CENTRE)
                    continue;
                const unsigned short l = s_lab[c + nb_off(k)];
                ma |= (unsigned)(l == a) << k;
                mb |= (unsigned)(l == bb) << k;
            }
            ok = (a == 0 || simple_point<ND>(ma)) && (bb == 0 || simple_point<ND>(mb));
        }
        if (ok)
            s_lab[c] = (unsigned short)bb;
        return ok ? 2 : 3;
    };
    auto clear_own_keys = [&]() {
        const int ntile = ti.TX * ti.TY * ti.TZ;
        for (int k = threadIdx.x; k < ntile; k += kBlock) {
            const int lx = k % ti.TX, ly = (k / ti.TX) % ti.TY, lz = k / (ti.TX * ti.TY);
            s_key[(lx + 1) + ti.BX * ((ly + 1) + ti.BY * (lz + ti.hz))] = kKeyInf;
        }
    };
    // the tile's undecided candidates, staged in LDS when they fit
    if (threadIdx.x == 0)
        C.n = 0;
    __syncthreads();
    for (unsigned p = r0 + threadIdx.x; p < r1; p += kBlock) {
        // the record and gradient go out with the state (in bounds either way)
        const unsigned char st = b.tstate[p];
        const uint2 r = rec[p];
        const float gp = grad[p];
        if (st == 1) {
            const unsigned j = atomicAdd(&C.n, 1u);
            if (j < (unsigned)kTopoCand) {
                C.p[j] = p;
                C.cell[j] = (unsigned short)cell_of(r.x);
                C.rw[j] = r.y;
                C.key[j] = cand_key(gp, (int)(r.y >> 16));
                C.st[j] = 1;
            }
        }
    }
    __syncthreads();
    const unsigned nc = C.n;
    int pend = 0;
    if (nc <= (unsigned)kTopoCand) {
        for (;;) {
            int prog = 0;
            for (unsigned j = threadIdx.x; j < nc; j += kBlock)
                if (C.st[j] == 1) {
                    const unsigned char d = decide(C.rw[j], C.cell[j], C.key[j]);
                    if (d) {
                        C.st[j] = d;
                        prog = 1;
                    }
                }
            if (!__syncthreads_or(prog))
                break;
            clear_own_keys();
            __syncthreads();
            for (unsigned j = threadIdx.x; j < nc; j += kBlock)
                if (C.st[j] == 1)
                    atomicMin(&s_key[C.cell[j]], C.key[j]);
            __syncthreads();
        }
        // states back; words of the candidates' pixels published (the other
        // pixels of the tile kept theirs)
        for (unsigned j = threadIdx.x; j < nc; j += kBlock) {
            const unsigned p = C.p[j];
            const unsigned char st = C.st[j];
            pend |= st == 1;
            if (st != 1)
                b.tstate[p] = st;
            int x, y, z;
            unpack(g, rec[p].x, x, y, z);
            const int c = C.cell[j];
            word_store(words + lin_of(g, x, y, z), (s_key[c] << 16) | s_lab[c]);
        }
        return __syncthreads_or(pend) != 0;
    }
    // many candidates: states kept in memory
    for (;;) {
        int prog = 0;
        for (unsigned p = r0 + threadIdx.x; p < r1; p += kBlock) {
            if (b.tstate[p] != 1)
                continue;
            const uint2 r = rec[p];
            const unsigned char d = decide(r.y, cell_of(r.x), cand_key(grad[p], (int)(r.y >> 16)));
            if (d) {
                b.tstate[p] = d;
                prog = 1;
            }
        }
        if (!__syncthreads_or(prog))
            break;
        clear_own_keys();
        __syncthreads();
        for (unsigned p = r0 + threadIdx.x; p < r1; p += kBlock)
            if (b.tstate[p] == 1) {
                const uint2 r = rec[p];
                atomicMin(&s_key[cell_of(r.x)], cand_key(grad[p], (int)(r.y >> 16)));
            }
        __syncthreads();
    }
    for (unsigned p = r0 + threadIdx.x; p < r1; p += kBlock) {
        const unsigned char st = b.tstate[p];
        if (st == 0)
            continue;
        pend |= st == 1;
        const uint2 r = rec[p];
        const int c = cell_of(r.x);
        int x, y, z;
        unpack(g, r.x, x, y, z);
        word_store(words + lin_of(g, x, y, z), (s_key[c] << 16) | s_lab[c]);
    }
    return __syncthreads_or(pend) != 0;
}

// Candidates of state t: state, per-pixel smallest key, and the stamp of the
// tiles holding candidates (round 0's work).
__global__ __launch_bounds__(kBlock) void k_topo_prep(Geom g, Bufs b, int cur, const float* __restrict__ grad_sob,
                                                     const float* __restrict__ grad_l2, int flags)
{
    DevState* ds = b.ds;
    if (stopped(ds))
        return;
    const float* grad = ((flags & kAuto) && (ds->lmode & 1u)) ? grad_l2 : grad_sob;
    const unsigned n = ds->n[cur], stamp = topo_stamp(ds->iters);
    unsigned p0, p1;
    xcd_chunk(n, VB{blockIdx.x, gridDim.x}, p0, p1);
    for (unsigned base = p0; base < p1; base += kBlock) {
        const unsigned p = base + threadIdx.x;
        unsigned tile = 0xFFFFFFFFu;
        if (p < p1) {
            const float gv = grad[p];
            const bool cand = gv < 0.f;
            b.tstate[p] = cand ? 1 : 0;
            if (cand) {
                const uint2 r = b.rec[cur][p];
                int x, y, z;
                unpack(g, r.x, x, y, z);
                atomicMin(&b.pmap[lin_of(g, x, y, z)], (cand_key(gv, (int)(r.y >> 16)) << 16) | 0xFFFFull);
                tile = (unsigned)((x >> g.tsx) + g.ntx * ((y >> g.tsy) + g.nty * (z >> g.tsz)));
            }
        }
        // records are tile-sorted: the first candidate lane of each run of
        // one tile stamps it (round 0 walks the non-empty tiles and takes
        // the stamped ones)
        const unsigned prev = __shfl_up(tile, 1);
        if (tile != 0xFFFFFFFFu && (lane_id() == 0 || prev != tile))
            b.tmark[tile] = stamp;
    }
}

// Round r: the tiles listed by round r - 1 (for r = 0 the non-empty tiles
// the preparation stamped); those with undecided candidates left are listed
// for round r + 1.  The
// per-pixel words are updated in place: a block may see a neighbour's words
// from before or after that neighbour's work in this round, and either is a
// valid state of those pixels for every decision taken from it.
template <int ND>
__global__ __launch_bounds__(kBlock) void k_topo_round(Geom g, Bufs b, int cur, const float* __restrict__ grad_sob,
                                                      const float* __restrict__ grad_l2, int flags, int r)
{
    __shared__ unsigned short s_lab[kTopoBox];
    __shared__ unsigned long long s_key[kTopoBox];
    __shared__ TopoCand s_cand;
    DevState* ds = b.ds;
    if (stopped(ds))
        return;
    // round 0: the non-empty tiles, those stamped by the preparation
    const unsigned n = r == 0 ? ds->n_active[cur] : ds->topo_cnt[r];
    const unsigned stamp = topo_stamp(ds->iters);
    // consecutive list entries (neighbouring tiles, mostly) on one XCD
    const unsigned G = gridDim.x;
    const unsigned L = (G & 7u) ? blockIdx.x : (blockIdx.x & 7u) * (G >> 3) + (blockIdx.x >> 3);
    if (L >= n)
        return;
    const float* grad = ((flags & kAuto) && (ds->lmode & 1u)) ? grad_l2 : grad_sob;
    const unsigned* list = r == 0 ? b.active[cur] : b.tlist[r & 1];
    unsigned* next = b.tlist[(r + 1) & 1];
    for (unsigned i = L; i < n; i += G) {
        const unsigned t = list[i];
        if (r == 0 && b.tmark[t] != stamp)
            continue;  // no candidate in this tile
        const bool pend = topo_tile<ND>(g, b, cur, t, grad, b.pmap, s_lab, s_key, s_cand);
        if (pend && threadIdx.x == 0)
            next[atomicAdd(&ds->topo_cnt[r + 1], 1u)] = t;
        __syncthreads();  // LDS reuse by the next tile
    }
}

// One block: the tiles left after the parallel rounds, until none has
// undecided candidates.  Every pass decides at least the first-ranked
// undecided candidate.
template <int ND>
__global__ __launch_bounds__(kBlock) void k_topo_finish(Geom g, Bufs b, int cur, const float* __restrict__ grad_sob,
                                                       const float* __restrict__ grad_l2, int flags)
{
    __shared__ unsigned short s_lab[kTopoBox];
    __shared__ unsigned long long s_key[kTopoBox];
    __shared__ TopoCand s_cand;
    __shared__ unsigned s_mk;
    DevState* ds = b.ds;
    if (stopped(ds))
        return;
    const unsigned nleft = ds->topo_cnt[kTopoRounds];
    if (nleft == 0)
        return;
    const float* grad = ((flags & kAuto) && (ds->lmode & 1u)) ? grad_l2 : grad_sob;
    const unsigned done = topo_stamp(ds->iters) + 1u;  // even: never a stamp
    const unsigned* list = b.tlist[kTopoRounds & 1];
    for (int pass = 0;; ++pass) {
        if (pass == kTopoMaxPasses) {
            // a chain of dependent candidates across more tiles than this is
            // not expected; report instead of running on
            if (threadIdx.x == 0)
                atomicOr(&ds->err, kErrTopo);
            return;
        }
        bool any = false;
        for (unsigned i = 0; i < nleft; ++i) {
            const unsigned t = list[i];
            if (threadIdx.x == 0)
                s_mk = b.tmark[t];
            __syncthreads();
            const unsigned mk = s_mk;  // one value for the whole block
            __syncthreads();
            if (mk == done)
                continue;
            any = true;
            const bool pend = topo_tile<ND>(g, b, cur, t, grad, b.pmap, s_lab, s_key, s_cand);
            __syncthreads();
            if (threadIdx.x == 0 && !pend)
                b.tmark[t] = done;
            __syncthreads();
        }
        if (!any)
            break;
    }
}

// ------------------------------------------------------------- export / io

__global__ __launch_bounds__(kBlock) void k_unpack(Geom g, Bufs b, int cur, int32_t* lin, int32_t* a, int32_t* bb)
{
    unsigned n = b.ds->n[cur];
    for (unsigned p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) {
        uint2 r = b.rec[cur][p];
        int x, y, z;
        unpack(g, r.x, x, y, z);
        if (lin)
            lin[p] = (int32_t)lin_of(g, x, y, z);
        if (a)
            a[p] = (int32_t)(r.y & 0xffffu);
        if (bb)
            bb[p] = (int32_t)(r.y >> 16);
    }
}

__global__ __launch_bounds__(kBlock) void k_labels_out(Bufs b, int32_t* out, long long nvox)
{
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < nvox; i += (long long)gridDim.x * kBlock)
        out[i] = b.lab[i];
}

// -------------------------------------- stateless binning (caller particles)

__device__ __forceinline__ unsigned tile_of(const Geom& g, int x, int y, int z)
{
    return (unsigned)((x >> g.tsx) + g.ntx * ((y >> g.tsy) + g.nty * (z >> g.tsz)));
}

__global__ __launch_bounds__(kBlock) void k_bin_count(Geom g, Bufs b, long long n, const int32_t* lin,
                                                     const int32_t* a, const int32_t* bb)
{
    long long nvox = (long long)g.nx * g.ny * g.nz;
    for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < n; k += (long long)gridDim.x * kBlock) {
        long long i = lin[k];
        int la = a[k], lb = bb[k];
        if (i < 0 || i >= nvox || la < 0 || la >= g.max_labels || lb < 0 || lb >= g.max_labels || la == lb) {
            atomicOr(&b.ds->err, kErrInput);
            continue;
        }
        int x = (int)(i % g.nx), y = (int)((i / g.nx) % g.ny), z = (int)(i / ((long long)g.nx * g.ny));
        atomicAdd(&b.tcnt[tile_of(g, x, y, z)], 1u);
    }
}

// Exclusive scan of per-tile counts into tstart[0] and the non-empty tile
// list (single block; used by the stateless smoothing entry point).
__global__ __launch_bounds__(kScanThreads) void k_bin_scan(Geom g, Bufs b)
{
    __shared__ unsigned long long s_sum[kScanThreads / 64];
    __shared__ unsigned s_nz[kScanThreads / 64];
    int nt = g.ntiles, tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
    int per = (nt + kScanThreads - 1) / kScanThreads;
    int t0 = tid * per, t1 = min(t0 + per, nt);
    unsigned long long sum = 0;
    unsigned nz = 0;
    for (int t = t0; t < t1; ++t) {
        unsigned c = b.tcnt[t];
        sum += c;
        nz += c != 0;
    }
    unsigned long long isum = sum;
    unsigned inz = nz;
    for (int o = 1; o < 64; o <<= 1) {
        unsigned long long a = __shfl_up(isum, o);
        unsigned z = __shfl_up(inz, o);
        if (lane >= o) {
            isum += a;
            inz += z;
        }
    }
    if (lane == 63) {
        s_sum[w] = isum;
        s_nz[w] = inz;
    }
    __syncthreads();
    unsigned long long off = 0, total = 0;
    unsigned offz = 0, totz = 0;
    for (int i = 0; i < kScanThreads / 64; ++i) {
        off += i < w ? s_sum[i] : 0;
        offz += i < w ? s_nz[i] : 0;
        total += s_sum[i];
        totz += s_nz[i];
    }
    off += isum - sum;
    offz += inz - nz;
    unsigned long long run = off;
    unsigned an = offz;
    for (int t = t0; t < t1; ++t) {
        unsigned c = b.tcnt[t];
        b.tstart[0][t] = (unsigned)run;
        if (c)
            b.active[0][an++] = (unsigned)t;
        run += c;
    }
    if (tid == 0) {
        b.tstart[0][nt] = (unsigned)total;
        b.ds->n[0] = (unsigned)total;
        b.ds->n_active[0] = totz;
    }
}

__global__ __launch_bounds__(kBlock) void k_bin_scatter(Geom g, Bufs b, long long n, const int32_t* lin,
                                                       const int32_t* a, const int32_t* bb, const float* in,
                                                       unsigned* fill, unsigned* origin)
{
    for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < n; k += (long long)gridDim.x * kBlock) {
        long long i = lin[k];
        int x = (int)(i % g.nx), y = (int)((i / g.nx) % g.ny), z = (int)(i / ((long long)g.nx * g.ny));
        unsigned t = tile_of(g, x, y, z);
        unsigned slot = b.tstart[0][t] + atomicAdd(&fill[t], 1u);
        b.rec[0][slot] = make_uint2(pack(g, x, y, z), (unsigned)a[k] | ((unsigned)bb[k] << 16));
        b.dE[slot] = in[k];
        origin[slot] = (unsigned)k;
    }
}

__global__ __launch_bounds__(kBlock) void k_unbin(long long n, const unsigned* origin, const float* binned, float* out)
{
    for (long long s = (long long)blockIdx.x * kBlock + threadIdx.x; s < n; s += (long long)gridDim.x * kBlock)
        out[origin[s]] = binned[s];
}

// ------------------------------------------------------------ launchers

static int grid_for(long long n, int cap)
{
    long long gsz = (n + kBlock - 1) / kBlock;
    if (gsz < 1)
        gsz = 1;
    return (int)(gsz > cap ? cap : gsz);
}

hipError_t launch_init_labels(const Geom& g, const Bufs& b, const int32_t* labels_in, const void* img,
                              hipStream_t s)
{
    long long nvox = (long long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_init_labels, dim3(grid_for(nvox, 4096)), dim3(kBlock), 0, s, g, b, labels_in, img, nvox);
    return hipGetLastError();
}

hipError_t launch_stats_init(const Geom& g, const Bufs& b, const void* img, hipStream_t s)
{
    long long nvox = (long long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_stats_init, dim3(grid_for(nvox, 1024)), dim3(kBlock), 0, s, g, b, img, nvox);
    return hipGetLastError();
}

hipError_t launch_dense_put(const Geom& g, const Bufs& b, int cur, const float* in, hipStream_t s)
{
    if (!b.dv)
        return hipSuccess;
    hipLaunchKernelGGL(k_dense_put, dim3(g.gp), dim3(kBlock), 0, s, g, b, cur, in);
    return hipGetLastError();
}

hipError_t launch_l2diff(const Geom& g, const Bufs& b, const void* img, int cur, float* out, int gated,
                         hipStream_t s)
{
    if (g.psf)
        hipLaunchKernelGGL(k_l2diff<true>, dim3(g.gp), dim3(kBlock), 0, s, g, b, img, cur, out, gated);
    else if (g.ps_lds)
        hipLaunchKernelGGL(k_l2diff_ps, dim3(g.sob_grid), dim3(kBlock), g.ps_lds, s, g, b, img, cur, out, gated);
    else
        hipLaunchKernelGGL(k_l2diff<false>, dim3(g.gp), dim3(kBlock), 0, s, g, b, img, cur, out, gated);
    return hipGetLastError();
}

// Word fill (clears of scratch memory by a kernel, which stream capture
// records as an ordinary kernel node).
__global__ __launch_bounds__(kBlock) void k_fill_u32(unsigned* __restrict__ p, unsigned v, unsigned long long n)
{
    for (unsigned long long i = (unsigned long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * kBlock)
        p[i] = v;
}

hipError_t launch_fill_u32(unsigned* p, unsigned v, size_t n, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    size_t blocks = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(kBlock), 0, s, p, v,
                       (unsigned long long)n);
    return hipGetLastError();
}

hipError_t launch_sobolev(const Geom& g, const Bufs& b, const SobW& sw, int cur, const float* in, float* out,
                          int gated, int use_slots, hipStream_t s)
{
    dim3 gd(g.sob_grid), bd(kSobBlock);
    if (!g.brick || !use_slots) {
        hipLaunchKernelGGL(k_sobolev_generic, gd, bd, g.sob_lds, s, g, b, cur, in, out, gated);
        return hipGetLastError();
    }
    gd = dim3(g.brick_grid);
#define SOBRC_BRICK_W(ND, H, WIDE)                                                                 \
    if (g.ndim == ND && g.h == H && g.wide == WIDE) {                                              \
        if (g.full)                                                                                \
            hipLaunchKernelGGL((k_sobolev_brick<ND, H, true, WIDE>), gd, bd, 0, s, g, b, sw, cur, in, out, gated); \
        else                                                                                       \
            hipLaunchKernelGGL((k_sobolev_brick<ND, H, false, WIDE>), gd, bd, 0, s, g, b, sw, cur, in, out, gated); \
        return hipGetLastError();                                                                  \
    }
#define SOBRC_BRICK(ND, H) SOBRC_BRICK_W(ND, H, 0) SOBRC_BRICK_W(ND, H, 1) SOBRC_BRICK_TALL##ND(H)
#define SOBRC_BRICK_TALL3(H)
#define SOBRC_BRICK_TALL2(H) SOBRC_BRICK_W(2, H, 2)
    SOBRC_BRICK(3, 1) SOBRC_BRICK(3, 2) SOBRC_BRICK(3, 3) SOBRC_BRICK(3, 4)
    SOBRC_BRICK(2, 1) SOBRC_BRICK(2, 2) SOBRC_BRICK(2, 3) SOBRC_BRICK(2, 4)
    SOBRC_BRICK(2, 5) SOBRC_BRICK(2, 6) SOBRC_BRICK(2, 7) SOBRC_BRICK(2, 8)
#undef SOBRC_BRICK
#undef SOBRC_BRICK_W
#undef SOBRC_BRICK_TALL3
#undef SOBRC_BRICK_TALL2
    return hipErrorInvalidValue;
}

hipError_t launch_flip(const Geom& g, const Bufs& b, const void* img, int cur, const float* grad,
                       const float* grad_l2, int flags, hipStream_t s)
{
    if (g.topo)
        hipLaunchKernelGGL(k_flip<true>, dim3(g.gp), dim3(kBlock), 0, s, g, b, img, cur, grad, grad_l2, flags);
    else
        hipLaunchKernelGGL(k_flip<false>, dim3(g.gp), dim3(kBlock), 0, s, g, b, img, cur, grad, grad_l2, flags);
    return hipGetLastError();
}

hipError_t launch_topo(const Geom& g, const Bufs& b, int cur, const float* grad, const float* grad_l2, int flags,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_topo_prep, dim3(g.gp), dim3(kBlock), 0, s, g, b, cur, grad, grad_l2, flags);
    for (int r = 0; r < kTopoRounds; ++r) {
        // later rounds have fewer tiles left: smaller grids (multiples of 8),
        // but never so small that a block works through many tiles in turn
        int G = g.sob_grid >> (r < 2 ? r : 2);
        G = G < 8 ? 8 : (G + 7) / 8 * 8;
        if (g.ndim == 3)
            hipLaunchKernelGGL(k_topo_round<3>, dim3(G), dim3(kBlock), 0, s, g, b, cur, grad, grad_l2, flags, r);
        else
            hipLaunchKernelGGL(k_topo_round<2>, dim3(G), dim3(kBlock), 0, s, g, b, cur, grad, grad_l2, flags, r);
    }
    if (g.ndim == 3)
        hipLaunchKernelGGL(k_topo_finish<3>, dim3(1), dim3(kBlock), 0, s, g, b, cur, grad, grad_l2, flags);
    else
        hipLaunchKernelGGL(k_topo_finish<2>, dim3(1), dim3(kBlock), 0, s, g, b, cur, grad, grad_l2, flags);
    return hipGetLastError();
}

hipError_t launch_count(const Geom& g, const Bufs& b, int cur, int gated, int all_dirty, hipStream_t s)
{
#define SOBRC_COUNT(ND, WIDE)                                                                              \
    if (g.ndim == ND && g.wide == WIDE) {                                                                  \
        hipLaunchKernelGGL((k_count<ND, WIDE>), dim3(g.ge), dim3(kBlock), 0, s, g, b, cur, gated, all_dirty); \
        if (g.dlistm) {                                                                                    \
            const unsigned gl = g.ge < kListGrid ? (unsigned)g.ge : (unsigned)kListGrid;                 \
            hipLaunchKernelGGL((k_count_list<ND, WIDE>), dim3(gl), dim3(kBlock), 0, s, g, b, gated);      \
        }                                                                                                  \
    }
    SOBRC_COUNT(3, 0) SOBRC_COUNT(3, 1) SOBRC_COUNT(2, 0) SOBRC_COUNT(2, 1) SOBRC_COUNT(2, 2)
#undef SOBRC_COUNT
    return hipGetLastError();
}

hipError_t launch_scan(const Geom& g, const Bufs& b, int cur, int nxt, int is_init, float tol, int32_t* d_nflips,
                       int gated, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, g, b, cur, nxt, is_init, tol, d_nflips,
                       gated & kGate, gated & kAuto);
    return hipGetLastError();
}

hipError_t launch_write(const Geom& g, const Bufs& b, const void* img, int cur, int nxt, const float* grad,
                        const float* grad_l2, int flags, int all_dirty, hipStream_t s)
{
    hipLaunchKernelGGL(k_write, dim3(g.ge), dim3(kBlock), 0, s, g, b, img, cur, nxt, grad, grad_l2, flags,
                       all_dirty);
    return hipGetLastError();
}

hipError_t launch_unpack(const Geom& g, const Bufs& b, int cur, int32_t* lin, int32_t* a, int32_t* bb,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_unpack, dim3(grid_for(b.cap, 2048)), dim3(kBlock), 0, s, g, b, cur, lin, a, bb);
    return hipGetLastError();
}

hipError_t launch_labels_out(const Geom& g, const Bufs& b, int32_t* out, hipStream_t s)
{
    long long nvox = (long long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_labels_out, dim3(grid_for(nvox, 4096)), dim3(kBlock), 0, s, b, out, nvox);
    return hipGetLastError();
}

hipError_t launch_bin_count(const Geom& g, const Bufs& b, long long n, const int32_t* lin, const int32_t* a,
                            const int32_t* bb, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin_count, dim3(grid_for(n, 4096)), dim3(kBlock), 0, s, g, b, n, lin, a, bb);
    return hipGetLastError();
}

hipError_t launch_bin_scan(const Geom& g, const Bufs& b, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(kScanThreads), 0, s, g, b);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(const Geom& g, const Bufs& b, long long n, const int32_t* lin, const int32_t* a,
                              const int32_t* bb, const float* in, unsigned* fill, unsigned* origin, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin_scatter, dim3(grid_for(n, 4096)), dim3(kBlock), 0, s, g, b, n, lin, a, bb, in, fill,
                       origin);
    return hipGetLastError();
}

hipError_t launch_unbin(const Bufs& b, long long n, const unsigned* origin, const float* binned, float* out,
                        hipStream_t s)
{
    (void)b;
    hipLaunchKernelGGL(k_unbin, dim3(grid_for(n, 4096)), dim3(kBlock), 0, s, n, origin, binned, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ batches
//
// A batched launch runs the stand-alone kernel bodies for every live slot of a
// batch: a persistent grid (a multiple of 8 blocks, at most kPersist) walks the
// concatenated item space of the phase, and each item becomes the block
// (index, count) that the slot's own launch would have had.  A slot's results
// are therefore the ones of its stand-alone run, bit for bit.

// Slot holding `item`: the largest i < nslot with off[i] <= item (empty
// slots have off[i] == off[i + 1] and are skipped; off[0] = 0).  Called with
// the same item by every lane of a wave: 64 candidates are tested per round
// with one load each and a ballot, so up to 64 slots take one dependent load
// (a binary search would take log2(nslot)).
__device__ __forceinline__ int slot_of(const unsigned* __restrict__ off, int nslot, unsigned item)
{
    const int lane = lane_id();
    int lo = 0, span = nslot;  // the answer lies in [lo, lo + span) and off[lo] <= item
    while (span > 1) {
        const int step = (span + 63) >> 6;
        const int c = lane * step;
        const bool ok = c < span && off[lo + c] <= item;
        const unsigned long long m = __ballot(ok);  // lane 0 always holds
        const int last = 63 - __clzll((long long)m);
        lo += last * step;
        span = min(step, span - last * step);
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void kb_l2diff(const ImgDesc* __restrict__ d, const unsigned* __restrict__ par,
                                                   const unsigned* __restrict__ offs, int nslot,
                                                   unsigned* __restrict__ tpre)
{
    if (blockIdx.x == 0) {
        // prefix of the slots' non-empty tile counts (state par[i]) for the
        // batched Sobolev kernel, which deals the batch's tiles to its blocks
        __shared__ unsigned s_red[kBlock / 64];
        unsigned carry = 0;
        for (int i0 = 0; i0 < nslot; i0 += kBlock) {
            const int i = i0 + (int)threadIdx.x;
            const unsigned n = (i < nslot && d[i].live) ? d[i].b.ds->n_active[par[i]] : 0u;
            unsigned tot;
            const unsigned ex = block_exscan_u(n, s_red, &tot);
            if (i < nslot)
                tpre[i] = carry + ex;
            carry += tot;
        }
        if (threadIdx.x == 0)
            tpre[nslot] = carry;
    }
    const unsigned* off = offs + kPhPart * (nslot + 1);
    const unsigned total = off[nslot];
    for (unsigned item = blockIdx.x; item < total; item += gridDim.x) {
        const int i = slot_of(off, nslot, item);
        const ImgDesc& D = d[i];
        const unsigned v = item - off[i];
        if (v < (unsigned)D.g.gp)
            l2diff_body<false>(D.g, D.b, D.img, (int)par[i], D.b.dE, 1, VB{v, (unsigned)D.g.gp});
    }
}

__global__ __launch_bounds__(kSobBlock) void kb_sobolev_generic(const ImgDesc* __restrict__ d,
                                                               const unsigned* __restrict__ par,
                                                               const unsigned* __restrict__ offs, int nslot,
                                                               int gated)
{
    const unsigned* off = offs + kPhSob * (nslot + 1);
    const unsigned total = off[nslot];
    for (unsigned item = blockIdx.x; item < total; item += gridDim.x) {
        const int i = slot_of(off, nslot, item);
        const ImgDesc& D = d[i];
        const unsigned v = item - off[i];
        if (v < (unsigned)D.g.sob_grid)
            sobolev_generic_body(D.g, D.b, (int)par[i], D.b.dE, D.b.gH1, gated, VB{v, (unsigned)D.g.sob_grid});
        __syncthreads();
    }
}

template <int ND, int H, bool FULL, int WIDE>
// The batch's non-empty tiles, numbered through all slots (tpre: the prefix
// of their counts, written by kb_l2diff), are dealt to the blocks in
// contiguous runs (XCD-contiguous as in a stand-alone launch): the blocks
// follow the tiles that hold particles in this iteration instead of a fixed
// share of every image's tiles.
__global__ __launch_bounds__(kSobBlock) void kb_sobolev_brick(const ImgDesc* __restrict__ d,
                                                             const unsigned* __restrict__ par,
                                                             const unsigned* __restrict__ tpre, int nslot, SobW sw,
                                                             int gated)
{
    unsigned a0, a1;
    xcd_chunk(tpre[nslot], VB{blockIdx.x, gridDim.x}, a0, a1);
    for (unsigned k = a0; k < a1;) {
        const int i = slot_of(tpre, nslot, k);  // slot whose run holds tile k (never an empty one)
        const unsigned e = min(a1, tpre[i + 1]);
        const ImgDesc& D = d[i];
        if (k != a0)
            __syncthreads();  // the previous slot's tiles are done with LDS
        brick_range<ND, H, FULL, WIDE>(D.g, D.b, sw, (int)par[i], D.b.dE, D.b.gH1, gated, k - tpre[i], e - tpre[i]);
        k = e;
    }
}

__global__ __launch_bounds__(kBlock) void kb_flip(const ImgDesc* __restrict__ d, const unsigned* __restrict__ par,
                                                 const unsigned* __restrict__ offs, int nslot, int l2, int flags)
{
    const unsigned* off = offs + kPhPart * (nslot + 1);
    const unsigned total = off[nslot];
    for (unsigned item = blockIdx.x; item < total; item += gridDim.x) {
        const int i = slot_of(off, nslot, item);
        const ImgDesc& D = d[i];
        const unsigned v = item - off[i];
        if (v < (unsigned)D.g.gp)
            flip_body<false>(D.g, D.b, D.img, (int)par[i], l2 ? D.b.dE : D.b.gH1, D.b.dE, flags,
                      VB{v, (unsigned)D.g.gp});
        __syncthreads();
    }
}

template <int ND, int WIDE>
__global__ __launch_bounds__(kBlock) void kb_count(const ImgDesc* __restrict__ d, const unsigned* __restrict__ par,
                                                  const unsigned* __restrict__ offs, int nslot)
{
    const unsigned* off = offs + kPhEmit * (nslot + 1);
    const unsigned total = off[nslot];
    for (unsigned item = blockIdx.x; item < total; item += gridDim.x) {
        const int i = slot_of(off, nslot, item);
        const ImgDesc& D = d[i];
        const unsigned v = item - off[i];
        if (v < (unsigned)D.g.ge)
            count_body<ND, WIDE>(D.g, D.b, (int)par[i], 1, 0, VB{v, (unsigned)D.g.ge});
        __syncthreads();
    }
}

template <int ND, int WIDE>
__global__ __launch_bounds__(kBlock) void kb_count_list(const ImgDesc* __restrict__ d,
                                                       const unsigned* __restrict__ offs, int nslot)
{
    const unsigned* off = offs + kPhList * (nslot + 1);
    const unsigned total = off[nslot];
    for (unsigned item = blockIdx.x; item < total; item += gridDim.x) {
        const int i = slot_of(off, nslot, item);
        const ImgDesc& D = d[i];
        const unsigned v = item - off[i];
        const unsigned nb = (unsigned)min(D.g.ge, kBatchListItems);
        if (v < nb && D.g.dlistm)
            count_list_body<ND, WIDE>(D.g, D.b, 1, VB{v, nb});
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanThreads) void kb_scan(const ImgDesc* __restrict__ d,
                                                       const unsigned* __restrict__ par,
                                                       const unsigned* __restrict__ offs, int nslot, float tol,
                                                       int flags)
{
    const unsigned* off = offs + kPhScan * (nslot + 1);
    const unsigned total = off[nslot];
    for (unsigned item = blockIdx.x; item < total; item += gridDim.x) {
        const int i = slot_of(off, nslot, item);
        const ImgDesc& D = d[i];
        const int cur = (int)par[i];
        scan_body(D.g, D.b, cur, 1 - cur, 0, tol, nullptr, 1, flags & kAuto, VB{0, 1});
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void kb_write(const ImgDesc* __restrict__ d, const unsigned* __restrict__ par,
                                                  const unsigned* __restrict__ offs, int nslot, int l2, int flags)
{
    const unsigned* off = offs + kPhEmit * (nslot + 1);
    const unsigned total = off[nslot];
    for (unsigned item = blockIdx.x; item < total; item += gridDim.x) {
        const int i = slot_of(off, nslot, item);
        const ImgDesc& D = d[i];
        const unsigned v = item - off[i];
        const int cur = (int)par[i];
        if (v < (unsigned)D.g.ge)
            write_body(D.g, D.b, D.img, cur, 1 - cur, l2 ? D.b.dE : D.b.gH1, D.b.dE, flags, 0,
                       VB{v, (unsigned)D.g.ge});
        __syncthreads();
    }
}

// End of a batched step: every live slot's current state is at the parity of
// its committed iterations (a stopped or rolled-back step leaves it).
__global__ __launch_bounds__(kBlock) void kb_advance(const ImgDesc* __restrict__ d, unsigned* __restrict__ par,
                                                    int nslot)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < nslot; i += gridDim.x * kBlock)
        if (d[i].live)
            par[i] = d[i].b.ds->iters & 1u;
}

// Start of a batched run: clear every live slot's tolerance stop.
__global__ __launch_bounds__(kBlock) void kb_clear(const ImgDesc* __restrict__ d, int nslot)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < nslot; i += gridDim.x * kBlock)
        if (d[i].live)
            d[i].b.ds->converged = 0u;
}

// Per live slot, the words a collecting host needs: committed iterations,
// stop flag, error bits, particle count that did not fit.
__global__ __launch_bounds__(kBlock) void kb_gather(const ImgDesc* __restrict__ d, int nslot,
                                                   uint4* __restrict__ out)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < nslot; i += gridDim.x * kBlock) {
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (d[i].live) {
            const DevState* ds = d[i].b.ds;
            v = make_uint4(ds->iters, ds->converged, ds->err, ds->need);
        }
        out[i] = v;
    }
}

namespace {
dim3 persistent_grid(unsigned items)
{
    unsigned g = (items + 7u) / 8u * 8u;
    return dim3(g < 8u ? 8u : (g > (unsigned)kPersist ? (unsigned)kPersist : g));
}
}  // namespace

hipError_t launch_batch_step(const BatchTab& t, const unsigned* totals, const Geom& g0, const SobW& sw, int l2,
                             int flags, float tol, hipStream_t s)
{
    const int ns = t.nslot;
    hipLaunchKernelGGL(kb_l2diff, persistent_grid(totals[kPhPart]), dim3(kBlock), 0, s, t.d, t.par, t.off, ns,
                       t.tpre);
    if (!l2) {
        const dim3 gd = persistent_grid(totals[kPhSob]);
        bool done = false;
        if (g0.brick) {
#define SOBRC_BRICK_W(ND, H, WIDE)                                                                          \
    if (!done && g0.ndim == ND && g0.h == H && g0.wide == WIDE) {                                             \
        if (g0.full)                                                                                          \
            hipLaunchKernelGGL((kb_sobolev_brick<ND, H, true, WIDE>), dim3(kPersist), dim3(kSobBlock), 0, s,  \
                               t.d, t.par, t.tpre, ns, sw, flags);                                            \
        else                                                                                                  \
            hipLaunchKernelGGL((kb_sobolev_brick<ND, H, false, WIDE>), dim3(kPersist), dim3(kSobBlock), 0, s, \
                               t.d, t.par, t.tpre, ns, sw, flags);                                            \
        done = true;                                                                                          \
    }
#define SOBRC_BRICK(ND, H) SOBRC_BRICK_W(ND, H, 0) SOBRC_BRICK_W(ND, H, 1) SOBRC_BRICK_TALL##ND(H)
#define SOBRC_BRICK_TALL3(H)
#define SOBRC_BRICK_TALL2(H) SOBRC_BRICK_W(2, H, 2)
            SOBRC_BRICK(3, 1) SOBRC_BRICK(3, 2) SOBRC_BRICK(3, 3) SOBRC_BRICK(3, 4)
            SOBRC_BRICK(2, 1) SOBRC_BRICK(2, 2) SOBRC_BRICK(2, 3) SOBRC_BRICK(2, 4)
            SOBRC_BRICK(2, 5) SOBRC_BRICK(2, 6) SOBRC_BRICK(2, 7) SOBRC_BRICK(2, 8)
#undef SOBRC_BRICK
#undef SOBRC_BRICK_W
#undef SOBRC_BRICK_TALL3
#undef SOBRC_BRICK_TALL2
        }
        if (!done)
            hipLaunchKernelGGL(kb_sobolev_generic, gd, dim3(kSobBlock), g0.sob_lds, s, t.d, t.par, t.off, ns,
                               flags);
    }
    hipLaunchKernelGGL(kb_flip, persistent_grid(totals[kPhPart]), dim3(kBlock), 0, s, t.d, t.par, t.off, ns, l2,
                       flags);
    const unsigned nsc = totals[kPhScan] < 256u ? (totals[kPhScan] ? totals[kPhScan] : 1u) : 256u;
#define SOBRC_COUNT(ND, WIDE)                                                                                \
    if (g0.ndim == ND && g0.wide == WIDE) {                                                                  \
        hipLaunchKernelGGL((kb_count<ND, WIDE>), persistent_grid(totals[kPhEmit]), dim3(kBlock), 0, s, t.d,  \
                           t.par, t.off, ns);                                                                \
        hipLaunchKernelGGL((kb_count_list<ND, WIDE>), persistent_grid(totals[kPhList]), dim3(kBlock), 0, s,  \
                           t.d, t.off, ns);                                                                  \
    }
    SOBRC_COUNT(3, 0) SOBRC_COUNT(3, 1) SOBRC_COUNT(2, 0) SOBRC_COUNT(2, 1) SOBRC_COUNT(2, 2)
#undef SOBRC_COUNT
    hipLaunchKernelGGL(kb_scan, dim3(nsc), dim3(kScanThreads), 0, s, t.d, t.par, t.off, ns, tol, flags);
    hipLaunchKernelGGL(kb_write, persistent_grid(totals[kPhEmit]), dim3(kBlock), 0, s, t.d, t.par, t.off, ns, l2,
                       flags);
    hipLaunchKernelGGL(kb_advance, dim3((ns + kBlock - 1) / kBlock), dim3(kBlock), 0, s, t.d, t.par, ns);
    return hipGetLastError();
}

hipError_t launch_batch_gather(const BatchTab& t, uint4* out, hipStream_t s)
{
    hipLaunchKernelGGL(kb_gather, dim3((t.nslot + kBlock - 1) / kBlock), dim3(kBlock), 0, s, t.d, t.nslot, out);
    return hipGetLastError();
}

hipError_t launch_batch_clear(const BatchTab& t, hipStream_t s)
{
    hipLaunchKernelGGL(kb_clear, dim3((t.nslot + kBlock - 1) / kBlock), dim3(kBlock), 0, s, t.d, t.nslot);
    return hipGetLastError();
}

}  // namespace sobrc
