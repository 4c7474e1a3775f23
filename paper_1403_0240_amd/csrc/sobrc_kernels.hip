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

constexpr int kBoxMax = 2048;
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

struct EmitLds {
    unsigned short box[kBoxMax];
    unsigned red[kBlock / 64];
    unsigned mlo[128], mhi[128];
    unsigned total;
};

// Particles of tile t under the current labels.  Counts them (WRITE = false)
// or writes their records in canonical order starting at rec[o] (WRITE = true).
// A box (tile + one-pixel halo) holding only two labels lo < hi takes the bit
// path: per box row, masks of "label == lo" and "label == hi"; a pixel is a
// particle iff its 3x3(x3) neighbourhood holds both labels, i.e. iff the OR of
// both dilated masks over the neighbourhood is set in both.  Other boxes
// enumerate the distinct neighbour labels of every pixel.
template <bool WRITE>
__device__ unsigned emit_tile(const Geom& g, const unsigned short* __restrict__ lab, unsigned t, EmitLds& L,
                              uint2* rec, unsigned o)
{
    TileInfo ti = tile_info(g, t);
    __syncthreads();
    load_label_box(g, lab, L.box, ti);
    __syncthreads();
    const int nbox = ti.BX * ti.BY * ti.BZ;
    unsigned mn = 0xffffu, mx = 0u;
    for (int k = threadIdx.x; k < nbox; k += kBlock) {
        unsigned l = L.box[k];
        if (l != kNone) {
            mn = l < mn ? l : mn;
            mx = l > mx ? l : mx;
        }
    }
    mn = block_reduce_u(mn, L.red, 0);
    mx = block_reduce_u(mx, L.red, 1);
    if (mx <= mn)
        return 0;  // one label (or none): no contour in this tile
    unsigned third = 0;
    for (int k = threadIdx.x; k < nbox; k += kBlock) {
        unsigned l = L.box[k];
        third |= (l != kNone && l != mn && l != mx) ? 1u : 0u;
    }
    third = block_reduce_u(third, L.red, 2);
    const int BXY = ti.BX * ti.BY, zr = ti.hz;
    if (!third) {
        const int nrow = ti.BY * ti.BZ;
        for (int r = threadIdx.x; r < nrow; r += kBlock) {
            unsigned ml = 0, mh = 0;
            for (int bx = 0; bx < ti.BX; ++bx) {
                unsigned l = L.box[r * ti.BX + bx];
                ml |= (l == mn ? 1u : 0u) << bx;
                mh |= (l == mx ? 1u : 0u) << bx;
            }
            L.mlo[r] = ml;
            L.mhi[r] = mh;
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const int nr = ti.TY * ti.TZ;  // interior rows, at most 64
            const int lane = threadIdx.x;
            unsigned pb = 0, own_lo = 0;
            int ly = 0, lz = 0;
            if (lane < nr) {
                ly = lane & (ti.TY - 1);
                lz = lane >> g.tsy;
                int by = ly + 1, bz = lz + ti.hz;
                unsigned ol = 0, oh = 0;
                for (int dz = -zr; dz <= zr; ++dz)
                    for (int dy = -1; dy <= 1; ++dy) {
                        int r = (by + dy) + ti.BY * (bz + dz);
                        unsigned ml = L.mlo[r], mh = L.mhi[r];
                        ol |= ml | (ml << 1) | (ml >> 1);
                        oh |= mh | (mh << 1) | (mh >> 1);
                    }
                int rc = by + ti.BY * bz;
                unsigned cl = L.mlo[rc], ch = L.mhi[rc];
                pb = ((ol & oh & (cl | ch)) >> 1) & ((1u << ti.TX) - 1u);
                own_lo = cl >> 1;
            }
            unsigned cnt = (unsigned)__popc(pb);
            if (WRITE) {
                unsigned inc = cnt;
                for (int d = 1; d < 64; d <<= 1) {
                    unsigned u = __shfl_up(inc, d);
                    if (lane >= d)
                        inc += u;
                }
                unsigned oo = o + inc - cnt;
                int y = ti.ty * ti.TY + ly, z = ti.tz * ti.TZ + lz;
                while (pb) {
                    int lx = __ffs(pb) - 1;
                    pb &= pb - 1;
                    bool isl = (own_lo >> lx) & 1u;
                    unsigned own = isl ? mn : mx, oth = isl ? mx : mn;
                    rec[oo++] = make_uint2(pack(g, ti.tx * ti.TX + lx, y, z), own | (oth << 16));
                }
            }
            cnt = wave_sum_u(cnt);
            if (lane == 0)
                L.total = cnt;
        }
        __syncthreads();
        return L.total;
    }
    // several labels: enumerate distinct neighbour labels per pixel
    const int nv = ti.TX * ti.TY * ti.TZ;
    const int per = (nv + kBlock - 1) / kBlock;  // contiguous run of voxels per thread
    const int v0 = threadIdx.x * per, v1 = min(v0 + per, nv);
    unsigned cc = 0;
    for (int v = v0; v < v1; ++v) {
        int lx = v & (ti.TX - 1), ly = (v >> g.tsx) & (ti.TY - 1), lz = v >> (g.tsx + g.tsy);
        int x = ti.tx * ti.TX + lx, y = ti.ty * ti.TY + ly, z = ti.tz * ti.TZ + lz;
        if (x >= g.nx || y >= g.ny || z >= g.nz)
            continue;
        int cidx = (lx + 1) + ti.BX * ((ly + 1) + ti.BY * (lz + ti.hz));
        int lo, hi;
        cc += neighbour_span(L.box, cidx, ti.BX, BXY, zr, L.box[cidx], lo, hi);
    }
    unsigned tot;
    unsigned oo = o + block_exscan_u(cc, L.red, &tot);
    if (WRITE) {
        for (int v = v0; v < v1; ++v) {
            int lx = v & (ti.TX - 1), ly = (v >> g.tsx) & (ti.TY - 1), lz = v >> (g.tsx + g.tsy);
            int x = ti.tx * ti.TX + lx, y = ti.ty * ti.TY + ly, z = ti.tz * ti.TZ + lz;
            if (x >= g.nx || y >= g.ny || z >= g.nz)
                continue;
            int cidx = (lx + 1) + ti.BX * ((ly + 1) + ti.BY * (lz + ti.hz));
            int own = L.box[cidx];
            unsigned pos = pack(g, x, y, z);
            int l = neighbour_next(L.box, cidx, ti.BX, BXY, zr, own, -1);
            while (l != 0x10000) {
                rec[oo++] = make_uint2(pos, (unsigned)own | ((unsigned)l << 16));
                l = neighbour_next(L.box, cidx, ti.BX, BXY, zr, own, l);
            }
        }
    }
    return tot;
}

// Emission ranges: range r holds tiles [r*Re, (r+1)*Re) (Re = 2^lgRe <=
// kBlock); the scan works on per-range totals.  Dirty tiles (a flip within one
// pixel this iteration, or every tile at initialisation) are shared among the
// blocks round-robin -- block b takes tiles t = b (mod gridDim) -- so that a
// surface crossing many neighbouring tiles does not pile up on one block.
__device__ __forceinline__ bool tile_dirty(const Bufs& b, unsigned t, unsigned epoch, int all_dirty)
{
    return all_dirty || b.dirty[t] == epoch;
}

// Particle count of every tile of the next state, accumulated per range.
// Clean tiles keep their previous count.
__global__ __launch_bounds__(kBlock) void k_count(Geom g, Bufs b, int cur, int gated, int all_dirty)
{
    __shared__ EmitLds L;
    __shared__ unsigned s_dl[kBlock];
    __shared__ unsigned s_ndl;
    if (gated && stopped(b.ds))
        return;
    const unsigned epoch = b.ds->epoch;
    const unsigned G = gridDim.x;
    if (threadIdx.x == 0)
        s_ndl = 0;
    __syncthreads();
    const unsigned t = blockIdx.x + threadIdx.x * G;  // at most Re <= kBlock tiles per block
    if (t < (unsigned)g.ntiles) {
        if (tile_dirty(b, t, epoch, all_dirty)) {
            s_dl[atomicAdd(&s_ndl, 1u)] = t;
        } else {
            unsigned c = b.tstart[cur][t + 1] - b.tstart[cur][t];
            b.tcnt[t] = c;
            if (c) {
                atomicAdd(&b.part_cnt[t >> g.lgRe], c);
                atomicAdd(&b.part_act[t >> g.lgRe], 1u);
            }
        }
    }
    __syncthreads();
    const unsigned ndl = s_ndl;
    for (unsigned i = 0; i < ndl; ++i) {
        unsigned td = s_dl[i];
        unsigned cc = emit_tile<false>(g, b.lab, td, L, nullptr, 0);
        if (threadIdx.x == 0) {
            b.tcnt[td] = cc;
            if (cc) {
                atomicAdd(&b.part_cnt[td >> g.lgRe], cc);
                atomicAdd(&b.part_act[td >> g.lgRe], 1u);
            }
        }
    }
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
// record telemetry and the convergence test.
__global__ __launch_bounds__(kScanThreads) void k_scan(Geom g, Bufs b, int cur, int nxt, int is_init, float tol,
                                                      int32_t* d_nflips, int gated)
{
    __shared__ unsigned long long s_sum[kScanThreads / 64];
    __shared__ unsigned s_nz[kScanThreads / 64];
    __shared__ unsigned s_f[kScanThreads / 64];
    DevState* ds = b.ds;
    if (gated && stopped(ds))
        return;
    const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
    unsigned nf = 0;
    if (!is_init) {
        unsigned f = 0;
        for (int i = tid; i < g.gp; i += kScanThreads)
            f += b.part_f[i];
        f = wave_sum(f);
        if (lane == 0)
            s_f[w] = f;
        if (g.small_m && w < g.max_labels) {
            long long dn = 0, dq = 0;
            for (int i = lane; i < g.gp; i += 64) {
                dn += b.part_n[(long long)w * g.gp + i];
                dq += b.part_q[(long long)w * g.gp + i];
            }
            dn = wave_sum(dn);
            dq = wave_sum(dq);
            if (lane == 0) {
                b.st_n[w] += dn;
                b.st_s1[w] += dq;
            }
        }
        __syncthreads();
        for (int i = 0; i < kScanThreads / 64; ++i)
            nf += s_f[i];
    }
    // per-label table of the piecewise-constant data term
    for (int l = tid; l < g.max_labels; l += kScanThreads) {
        long long n = b.st_n[l];
        double dn = (double)n;
        float mu = n > 0 ? (float)((double)b.st_s1[l] * g.fx_inv / dn) : 0.f;
        float fa = n > 1 ? (float)(dn / (dn - 1.0)) : 0.f;
        float fb = (float)(dn / (dn + 1.0));
        b.lstat[l] = make_float4(mu, fa, fb, 0.f);
    }
    // exclusive scan of the emission partials (a contiguous chunk per thread)
    const int per = (g.ge + kScanThreads - 1) / kScanThreads;
    const int i0 = tid * per, i1 = min(i0 + per, g.ge);
    unsigned long long sum = 0;
    unsigned nz = 0;
    for (int i = i0; i < i1; ++i) {
        sum += b.part_cnt[i];
        nz += b.part_act[i];
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
    bool overflow = total > (unsigned long long)b.cap;
    if (!overflow) {
        for (int i = i0; i < i1; ++i) {
            b.part_off[i] = (unsigned)off;
            b.part_aoff[i] = offz;
            off += b.part_cnt[i];
            offz += b.part_act[i];
        }
    }
    __syncthreads();
    for (int i = i0; i < i1; ++i) {  // the next count accumulates afresh
        b.part_cnt[i] = 0;
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
                ds->n[nxt] = ds->n[cur];
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
                unsigned ncur = ds->n[cur], it = ds->iters;
                b.hist[it % kHist] = ncur;
                b.hist[kHist + it % kHist] = nf;
                ds->iters = it + 1;
                if (d_nflips)
                    *d_nflips = (int32_t)nf;
                if (tol > 0.f && (double)nf < (double)tol * (double)ncur)
                    ds->converged = 1;
            }
        }
    }
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
__global__ __launch_bounds__(kBlock) void k_write(Geom g, Bufs b, const void* img, int cur, int nxt,
                                                 const float* __restrict__ grad, int all_dirty)
{
    __shared__ EmitLds L;
    __shared__ unsigned s_pre[kBlock + 1];
    __shared__ unsigned s_old[kBlock];
    __shared__ unsigned s_dl[kBlock];
    __shared__ unsigned s_ndl;
    DevState* ds = b.ds;
    if (ds->undo) {
        long long stride = (long long)gridDim.x * kBlock;
        unsigned n = ds->n[cur];
        for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
            b.rec[nxt][i] = b.rec[cur][i];
            uint2 r;
            int bb = 0;
            if (decide_move(b.rec[cur], grad, n, (unsigned)i, r, bb)) {
                int x, y, z;
                unpack(g, r.x, x, y, z);
                long long lin = lin_of(g, x, y, z);
                int a = (int)(r.y & 0xffffu);
                b.lab[lin] = (unsigned short)a;
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
    // range blockIdx.x: offsets, non-empty tile list, and the clean tiles'
    // records moved unchanged to their new offsets
    const int t0 = blockIdx.x << g.lgRe, t1 = min(t0 + g.Re, g.ntiles);
    const int t = t0 + (int)threadIdx.x;
    const bool in = t < t1;
    const unsigned c = in ? b.tcnt[t] : 0;
    const bool dirty = in && tile_dirty(b, (unsigned)t, epoch, all_dirty);
    unsigned tot, totz;
    const unsigned ex = block_exscan_u(c, L.red, &tot);
    const unsigned exz = block_exscan_u(c != 0 ? 1u : 0u, L.red, &totz);
    const unsigned base = b.part_off[blockIdx.x], abase = b.part_aoff[blockIdx.x];
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
    s_old[threadIdx.x] = (in && !dirty) ? b.tstart[cur][t] : 0xffffffffu;
    if (threadIdx.x == 0)
        s_ndl = 0;
    __syncthreads();
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
    // dirty tiles of this block's round-robin share are re-emitted from the labels
    const unsigned G = gridDim.x;
    const unsigned td = blockIdx.x + threadIdx.x * G;
    if (td < (unsigned)g.ntiles && b.tcnt[td] && tile_dirty(b, td, epoch, all_dirty))
        s_dl[atomicAdd(&s_ndl, 1u)] = td;
    __syncthreads();
    const unsigned ndl = s_ndl;
    for (unsigned i = 0; i < ndl; ++i) {
        const unsigned tt = s_dl[i];
        const int r0 = (int)(tt >> g.lgRe) << g.lgRe;
        // offset of tile tt: its range's base plus the counts before it in the range
        unsigned part = (r0 + (int)threadIdx.x < (int)tt) ? b.tcnt[r0 + threadIdx.x] : 0u;
        unsigned o = b.part_off[tt >> g.lgRe] + block_sum_u(part, L.red);
        emit_tile<true>(g, b.lab, tt, L, rec, o);
    }
}

// --------------------------------------------------- L2 gradient per particle
//
// Energy change of one move a -> b at pixel x with value v (Eqs. (10)-(11)):
//   PC: n_b/(n_b+1) (v - mu_b)^2 - n_a/(n_a-1) (v - mu_a)^2   (means re-estimated)
//   PS: (v - m_b(x))^2 - (v - m_a(x))^2, m_l = mean of label l in the ball |y-x| <= R
//   + lambda (c_a - c_b), c_l = face neighbours with label l (contour length).
__global__ __launch_bounds__(kBlock) void k_l2diff(Geom g, Bufs b, const void* img, int cur, float* __restrict__ out,
                                                  int gated)
{
    DevState* ds = b.ds;
    if (gated && blockIdx.x == 0 && threadIdx.x == 0) {
        ds->go = 0;
        ds->undo = 0;
        ds->epoch = ds->epoch + 1;
    }
    if (gated && stopped(ds))
        return;
    unsigned n = ds->n[cur];
    const uint2* rec = b.rec[cur];
    long long nxy = (long long)g.nx * g.ny;
    for (unsigned p = blockIdx.x * kBlock + threadIdx.x; p < n; p += gridDim.x * kBlock) {
        uint2 r = rec[p];
        int x, y, z;
        unpack(g, r.x, x, y, z);
        int a = (int)(r.y & 0xffffu), bl = (int)(r.y >> 16);
        long long i = lin_of(g, x, y, z);
        float v = img_at(g, img, i);
        int ca = 0, cb = 0;
#define SOBRC_FACE(cond, j)                    \
    if (cond) {                                \
        int l = b.lab[j];                      \
        ca += l == a;                          \
        cb += l == bl;                         \
    }
        SOBRC_FACE(x > 0, i - 1)
        SOBRC_FACE(x + 1 < g.nx, i + 1)
        SOBRC_FACE(y > 0, i - g.nx)
        SOBRC_FACE(y + 1 < g.ny, i + g.nx)
        SOBRC_FACE(z > 0, i - nxy)
        SOBRC_FACE(z + 1 < g.nz, i + nxy)
#undef SOBRC_FACE
        float dext;
        if (g.model == 0) {
            float4 sa = b.lstat[a], sb = b.lstat[bl];
            float da = v - sa.x, db = v - sb.x;
            dext = sb.z * db * db - sa.y * da * da;
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
            dext = (v - mb) * (v - mb) - (v - ma) * (v - ma);
        }
        out[p] = dext + g.lambda * (float)(ca - cb);
    }
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

// Tiles [a0, a1) of the non-empty list for this block: contiguous chunks,
// consecutive chunks on the same XCD (blocks are dealt to the 8 XCDs
// round-robin).
__device__ __forceinline__ void xcd_chunk(unsigned na, unsigned& a0, unsigned& a1)
{
    const unsigned G = gridDim.x, L = (blockIdx.x & 7u) * (G >> 3) + (blockIdx.x >> 3);
    a0 = (unsigned)((unsigned long long)L * na / G);
    a1 = (unsigned)((unsigned long long)(L + 1) * na / G);
}

__global__ __launch_bounds__(kSobBlock) void k_sobolev_generic(Geom g, Bufs b, int cur,
                                                              const float* __restrict__ in,
                                                              float* __restrict__ out, int gated)
{
    extern __shared__ __align__(16) char lds[];
    if (gated && stopped(b.ds))
        return;
    unsigned a0, a1;
    xcd_chunk(b.ds->n_active[cur], a0, a1);
    for (unsigned ai = a0; ai < a1; ++ai)
        sob_generic_tile(g, b, cur, in, out, b.active[cur][ai], lds);
}

template <int ND, int H>
struct BrickShape {
    static constexpr int TX = ND == 3 ? 8 : 16, TY = TX, TZ = ND == 3 ? 8 : 1;
    static constexpr int HZ = ND == 3 ? H : 0;
    static constexpr int BX = TX + 2 * H, BY = TY + 2 * H, BZ = TZ + 2 * HZ;
    static constexpr int NCELL = BX * BY * BZ;
    static constexpr int LIM = (H + 1) * (H + 1);
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

template <int ND, int H>
constexpr TapList<BrickShape<ND, H>::NT> make_taps()
{
    using S = BrickShape<ND, H>;
    TapList<S::NT> t{};
    int k = 0;
    for (int dz = -S::HZ; dz <= S::HZ; ++dz)
        for (int dy = -H; dy <= H; ++dy)
            for (int dx = -H; dx <= H; ++dx) {
                int d2 = dx * dx + dy * dy + dz * dz;
                if (d2 < S::LIM) {
                    t.off[k] = (dx + H) + S::BX * ((dy + H) + S::BY * (dz + S::HZ));
                    t.d2[k] = d2;
                    ++k;
                }
            }
    return t;
}

template <int ND, int H, bool FULL>
__global__ __launch_bounds__(kSobBlock) void k_sobolev_brick(Geom g, Bufs b, SobW sw, int cur,
                                                            const float* __restrict__ in,
                                                            float* __restrict__ out, int gated)
{
    using S = BrickShape<ND, H>;
    constexpr TapList<S::NT> taps = make_taps<ND, H>();
    __shared__ __align__(16) char lds[brick_lds_bytes(ND, H)];
    __shared__ unsigned s_flag;
    __shared__ unsigned s_beg[32];
    __shared__ unsigned s_pre[33];
    float2* s_v = (float2*)lds;                      // (value of lo->hi, value of hi->lo)
    unsigned* s_n = (unsigned*)(s_v + S::NCELL);     // count of lo->hi | count of hi->lo << 16
    DevState* ds = b.ds;
    if (gated && stopped(ds))
        return;
    unsigned a0, a1;
    xcd_chunk(ds->n_active[cur], a0, a1);
    const unsigned* ts = b.tstart[cur];
    const uint2* rec = b.rec[cur];
    for (unsigned ai = a0; ai < a1; ++ai) {
        const unsigned t = b.active[cur][ai];
        const int tx = (int)(t % (unsigned)g.ntx), ty = (int)((t / (unsigned)g.ntx) % (unsigned)g.nty);
        const int tz = (int)(t / ((unsigned)g.ntx * (unsigned)g.nty));
        const int ox = tx * S::TX - H, oy = ty * S::TY - H, oz = tz * S::TZ - S::HZ;
        const int bx0 = max(ox, 0), bx1 = min(ox + S::BX, g.nx);
        const int by0 = max(oy, 0), by1 = min(oy + S::BY, g.ny);
        const int bz0 = max(oz, 0), bz1 = min(oz + S::BZ, g.nz);
        const int kx0 = bx0 >> g.tsx, nkx = ((bx1 - 1) >> g.tsx) - kx0 + 1;
        const int ky0 = by0 >> g.tsy, nky = ((by1 - 1) >> g.tsy) - ky0 + 1;
        const int kz0 = bz0 >> g.tsz, nkz = ((bz1 - 1) >> g.tsz) - kz0 + 1;
        const int nnt = nkx * nky * nkz;
        const unsigned cs = ts[t], ce = ts[t + 1];
        const unsigned code0 = rec[cs].y;
        const unsigned lo = min(code0 & 0xffffu, code0 >> 16), hi = max(code0 & 0xffffu, code0 >> 16);
        const unsigned codeA = lo | (hi << 16), codeB = hi | (lo << 16);
        __syncthreads();  // the previous tile is done with LDS
        for (int k = threadIdx.x; k < S::NCELL; k += kSobBlock) {
            s_v[k] = make_float2(0.f, 0.f);
            s_n[k] = 0u;
        }
        if (threadIdx.x == 0)
            s_flag = 0;
        if ((int)threadIdx.x < nnt) {
            int k = threadIdx.x;
            int kx = kx0 + k % nkx, ky = ky0 + (k / nkx) % nky, kz = kz0 + k / (nkx * nky);
            unsigned nt = (unsigned)(kx + g.ntx * (ky + g.nty * kz));
            s_beg[k] = ts[nt];
            s_pre[k + 1] = ts[nt + 1] - ts[nt];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            s_pre[0] = 0;
            for (int k = 0; k < nnt; ++k)
                s_pre[k + 1] += s_pre[k];
        }
        __syncthreads();
        // scatter the box's particles into the brick, 8 loads in flight per thread
        const unsigned total = s_pre[nnt];
        int j = 0;  // neighbour tile of this thread's flat index (monotone)
        for (unsigned k0 = 0; k0 < total; k0 += 8 * kSobBlock) {
            uint2 r[8];
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                unsigned k = k0 + u * kSobBlock + threadIdx.x;
                r[u] = make_uint2(0xffffffffu, 0u);
                v[u] = 0.f;
                if (k < total) {
                    while (s_pre[j + 1] <= k)
                        ++j;
                    unsigned q = s_beg[j] + (k - s_pre[j]);
                    r[u] = rec[q];
                    v[u] = in[q];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (r[u].x == 0xffffffffu)
                    continue;
                int x, y, z;
                unpack(g, r[u].x, x, y, z);
                if (x < bx0 || x >= bx1 || y < by0 || y >= by1 || z < bz0 || z >= bz1)
                    continue;
                int c = (x - ox) + S::BX * ((y - oy) + S::BY * (z - oz));
                if (r[u].y == codeA) {
                    s_v[c] = make_float2(v[u], 0.f);
                    s_n[c] = 1u;
                } else if (r[u].y == codeB) {
                    s_v[c] = make_float2(0.f, v[u]);
                    s_n[c] = 1u << 16;
                } else {
                    s_flag = 1;
                }
            }
        }
        __syncthreads();
        if (s_flag) {
            sob_generic_tile(g, b, cur, in, out, t, lds);
            continue;
        }
        // stencil: uniform trip count, idle lanes work on the tile's first particle
        for (unsigned base = cs; base < ce; base += kSobBlock) {
            const unsigned p = base + threadIdx.x;
            const bool act = p < ce;
            const uint2 r = rec[act ? p : cs];
            int x, y, z;
            unpack(g, r.x, x, y, z);
            const int c0 = (x - ox - H) + S::BX * ((y - oy - H) + S::BY * (z - oz - S::HZ));
            const float2* vb = s_v + c0;
            const unsigned* nb = s_n + c0;
            float sA = 0.f, sB = 0.f;
            unsigned cnt = 0;
#pragma unroll
            for (int k = 0; k < S::NT; ++k) {
                const float2 cv = vb[taps.off[k]];
                const float wk = sw.w[taps.d2[k]];
                sA = fmaf(wk, cv.x, sA);
                sB = fmaf(wk, cv.y, sB);
                if (FULL)
                    cnt += nb[taps.off[k]];
                else
                    cnt += nb[taps.off[k]] * sw.m[taps.d2[k]];
            }
            const bool sideA = r.y == codeA;
            const float same = sideA ? sA : sB, other = sideA ? sB : sA;
            const unsigned nS = sideA ? (cnt & 0xffffu) : (cnt >> 16), nO = sideA ? (cnt >> 16) : (cnt & 0xffffu);
            float res = same / (float)nS;
            if (nO)
                res -= other / (float)nO;
            if (act)
                out[p] = res;
        }
    }
}

// ------------------------------------------------------- acceptance of moves
//
// Every particle with gradient < 0 is a candidate; per pixel the smallest
// gradient wins (ties: first in order, i.e. smaller b).  Decisions read only
// gradients and records of state t, so the label field is updated in place.
// Region statistics follow exactly (integer deltas): per-block partials for
// few labels, wave-merged atomics otherwise.  Tiles within one pixel of a
// flip are marked dirty for the particle-set update.
__global__ __launch_bounds__(kBlock) void k_flip(Geom g, Bufs b, const void* img, int cur,
                                                const float* __restrict__ grad)
{
    __shared__ long long s_dn[kSmallM], s_dq[kSmallM];
    __shared__ unsigned s_f;
    DevState* ds = b.ds;
    if (stopped(ds))
        return;
    if (threadIdx.x < kSmallM) {
        s_dn[threadIdx.x] = 0;
        s_dq[threadIdx.x] = 0;
    }
    if (threadIdx.x == 0)
        s_f = 0;
    __syncthreads();
    const unsigned n = ds->n[cur];
    const unsigned epoch = ds->epoch;
    const uint2* rec = b.rec[cur];
    const int lane = lane_id();
    const int TX = 1 << g.tsx, TY = 1 << g.tsy, TZ = 1 << g.tsz;
    for (unsigned base = blockIdx.x * kBlock; base < n; base += gridDim.x * kBlock) {
        unsigned p = base + threadIdx.x;
        bool f = false;
        unsigned lin = 0;
        int a = 0, bb = 0;
        if (p < n) {
            uint2 r;
            if (decide_move(rec, grad, n, p, r, bb)) {
                f = true;
                int x, y, z;
                unpack(g, r.x, x, y, z);
                lin = (unsigned)lin_of(g, x, y, z);
                a = (int)(r.y & 0xffffu);
                b.lab[lin] = (unsigned short)bb;
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
        if (lane == leader)
            atomicAdd(&s_f, (unsigned)__popcll(m));
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
    if (threadIdx.x == 0)
        b.part_f[blockIdx.x] = s_f;
    if (g.small_m && (int)threadIdx.x < g.max_labels) {
        b.part_n[(long long)threadIdx.x * gridDim.x + blockIdx.x] = s_dn[threadIdx.x];
        b.part_q[(long long)threadIdx.x * gridDim.x + blockIdx.x] = s_dq[threadIdx.x];
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

hipError_t launch_l2diff(const Geom& g, const Bufs& b, const void* img, int cur, float* out, int gated,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_l2diff, dim3(g.gp), dim3(kBlock), 0, s, g, b, img, cur, out, gated);
    return hipGetLastError();
}

hipError_t launch_sobolev(const Geom& g, const Bufs& b, const SobW& sw, int cur, const float* in, float* out,
                          int gated, hipStream_t s)
{
    dim3 gd(g.sob_grid), bd(kSobBlock);
    if (!g.brick) {
        hipLaunchKernelGGL(k_sobolev_generic, gd, bd, g.sob_lds, s, g, b, cur, in, out, gated);
        return hipGetLastError();
    }
#define SOBRC_BRICK(ND, H)                                                                         \
    if (g.ndim == ND && g.h == H) {                                                                \
        if (g.full)                                                                                \
            hipLaunchKernelGGL((k_sobolev_brick<ND, H, true>), gd, bd, 0, s, g, b, sw, cur, in, out, gated); \
        else                                                                                       \
            hipLaunchKernelGGL((k_sobolev_brick<ND, H, false>), gd, bd, 0, s, g, b, sw, cur, in, out, gated); \
        return hipGetLastError();                                                                  \
    }
    SOBRC_BRICK(3, 1) SOBRC_BRICK(3, 2) SOBRC_BRICK(3, 3) SOBRC_BRICK(3, 4)
    SOBRC_BRICK(2, 1) SOBRC_BRICK(2, 2) SOBRC_BRICK(2, 3) SOBRC_BRICK(2, 4)
    SOBRC_BRICK(2, 5) SOBRC_BRICK(2, 6) SOBRC_BRICK(2, 7) SOBRC_BRICK(2, 8)
#undef SOBRC_BRICK
    return hipErrorInvalidValue;
}

hipError_t launch_flip(const Geom& g, const Bufs& b, const void* img, int cur, const float* grad, hipStream_t s)
{
    hipLaunchKernelGGL(k_flip, dim3(g.gp), dim3(kBlock), 0, s, g, b, img, cur, grad);
    return hipGetLastError();
}

hipError_t launch_count(const Geom& g, const Bufs& b, int cur, int gated, int all_dirty, hipStream_t s)
{
    hipLaunchKernelGGL(k_count, dim3(g.ge), dim3(kBlock), 0, s, g, b, cur, gated, all_dirty);
    return hipGetLastError();
}

hipError_t launch_scan(const Geom& g, const Bufs& b, int cur, int nxt, int is_init, float tol, int32_t* d_nflips,
                       int gated, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, g, b, cur, nxt, is_init, tol, d_nflips, gated);
    return hipGetLastError();
}

hipError_t launch_write(const Geom& g, const Bufs& b, const void* img, int cur, int nxt, const float* grad,
                        int all_dirty, hipStream_t s)
{
    hipLaunchKernelGGL(k_write, dim3(g.ge), dim3(kBlock), 0, s, g, b, img, cur, nxt, grad, all_dirty);
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

}  // namespace sobrc
