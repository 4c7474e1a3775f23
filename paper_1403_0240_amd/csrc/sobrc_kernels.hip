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
                atomicAdd((unsigned long long*)&b.st_n[key], (unsigned long long)c);
                atomicAdd((unsigned long long*)&b.st_s1[key], (unsigned long long)s);
            }
            pend = pend && !match;
        }
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

// Count the particles of every candidate tile of the next state.
__global__ __launch_bounds__(kBlock) void k_count(Geom g, Bufs b, int gated)
{
    __shared__ unsigned short s_box[kBoxMax];
    __shared__ unsigned s_red[kBlock / 64];
    if (gated && stopped(b.ds))
        return;
    for (unsigned t = blockIdx.x; t < (unsigned)g.ntiles; t += gridDim.x) {
        int flag = b.cand[t];
        __syncthreads();
        if (!flag) {
            if (threadIdx.x == 0)
                b.tcnt[t] = 0;
            continue;
        }
        if (threadIdx.x == 0)
            b.cand[t] = 0;
        TileInfo ti = tile_info(g, t);
        load_label_box(g, b.lab, s_box, ti);
        __syncthreads();
        int BXY = ti.BX * ti.BY, zr = ti.hz;
        unsigned c = 0;
        int nv = ti.TX * ti.TY * ti.TZ;
        for (int v = threadIdx.x; v < nv; v += kBlock) {
            int lx = v & (ti.TX - 1), ly = (v >> g.tsx) & (ti.TY - 1), lz = v >> (g.tsx + g.tsy);
            int x = ti.tx * ti.TX + lx, y = ti.ty * ti.TY + ly, z = ti.tz * ti.TZ + lz;
            if (x >= g.nx || y >= g.ny || z >= g.nz)
                continue;
            int cidx = (lx + 1) + ti.BX * ((ly + 1) + ti.BY * (lz + ti.hz));
            int lo, hi;
            c += neighbour_span(s_box, cidx, ti.BX, BXY, zr, s_box[cidx], lo, hi);
        }
        unsigned tot = block_sum_u(c, s_red);
        if (threadIdx.x == 0)
            b.tcnt[t] = tot;
    }
}

// Exclusive scan of tile counts into the next state's cell list (single block).
// Also: capacity check with roll-back request, telemetry, convergence test.
__global__ __launch_bounds__(kScanThreads) void k_scan(Geom g, Bufs b, int cur, int nxt, int is_init, float tol,
                                                      int32_t* d_nflips, int gated)
{
    __shared__ unsigned long long s_sum[kScanThreads / 64];
    __shared__ unsigned s_nz[kScanThreads / 64];
    DevState* ds = b.ds;
    if (gated && stopped(ds))
        return;
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
    bool overflow = total > (unsigned long long)b.cap;
    if (!overflow) {
        unsigned* ts = b.tstart[nxt];
        unsigned* act = b.active[nxt];
        unsigned long long run = off;
        unsigned an = offz;
        for (int t = t0; t < t1; ++t) {
            unsigned c = b.tcnt[t];
            ts[t] = (unsigned)run;
            if (c)
                act[an++] = (unsigned)t;
            run += c;
        }
        if (tid == 0)
            ts[nt] = (unsigned)total;
    } else if (!is_init) {
        for (int t = tid; t <= nt; t += kScanThreads)
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
            if (!is_init) {
                unsigned nf = ds->nflips, ncur = ds->n[cur], it = ds->iters;
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

// Write the particle records of every non-empty tile of the next state in
// canonical order and flag the tiles the following emission has to scan
// (particles move by at most one pixel per iteration, so the next particle set
// lies in this tile set dilated by one tile).  On an overflowing step, restore
// state t instead.
__global__ __launch_bounds__(kBlock) void k_write(Geom g, Bufs b, const void* img, int cur, int nxt)
{
    __shared__ unsigned short s_box[kBoxMax];
    __shared__ unsigned s_red[kBlock / 64];
    DevState* ds = b.ds;
    if (ds->undo) {
        long long stride = (long long)gridDim.x * kBlock;
        unsigned n = ds->n[cur];
        for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
            b.rec[nxt][i] = b.rec[cur][i];
        unsigned nf = ds->nflip_list;
        for (long long k = (long long)blockIdx.x * kBlock + threadIdx.x; k < nf; k += stride) {
            uint2 e = b.flist[k];
            int a = (int)(e.y & 0xffffu), bb = (int)(e.y >> 16);
            b.lab[e.x] = (unsigned short)a;
            long long q = qvalue(g, img, e.x);
            atomicAdd((unsigned long long*)&b.st_n[a], 1ull);
            atomicAdd((unsigned long long*)&b.st_n[bb], (unsigned long long)(-1ll));
            atomicAdd((unsigned long long*)&b.st_s1[a], (unsigned long long)q);
            atomicAdd((unsigned long long*)&b.st_s1[bb], (unsigned long long)(-q));
        }
        return;
    }
    if (!ds->go)
        return;
    unsigned na = ds->n_active[nxt];
    const unsigned* ts = b.tstart[nxt];
    uint2* rec = b.rec[nxt];
    for (unsigned ai = blockIdx.x; ai < na; ai += gridDim.x) {
        unsigned t = b.active[nxt][ai];
        TileInfo ti = tile_info(g, t);
        __syncthreads();
        load_label_box(g, b.lab, s_box, ti);
        __syncthreads();
        int BXY = ti.BX * ti.BY, zr = ti.hz;
        int nv = ti.TX * ti.TY * ti.TZ;
        int per = (nv + kBlock - 1) / kBlock;   // contiguous run of voxels per thread
        int v0 = threadIdx.x * per, v1 = min(v0 + per, nv);
        unsigned c = 0;
        for (int v = v0; v < v1; ++v) {
            int lx = v & (ti.TX - 1), ly = (v >> g.tsx) & (ti.TY - 1), lz = v >> (g.tsx + g.tsy);
            int x = ti.tx * ti.TX + lx, y = ti.ty * ti.TY + ly, z = ti.tz * ti.TZ + lz;
            if (x >= g.nx || y >= g.ny || z >= g.nz)
                continue;
            int cidx = (lx + 1) + ti.BX * ((ly + 1) + ti.BY * (lz + ti.hz));
            int lo, hi;
            c += neighbour_span(s_box, cidx, ti.BX, BXY, zr, s_box[cidx], lo, hi);
        }
        unsigned tot;
        unsigned o = ts[t] + block_exscan_u(c, s_red, &tot);
        for (int v = v0; v < v1; ++v) {
            int lx = v & (ti.TX - 1), ly = (v >> g.tsx) & (ti.TY - 1), lz = v >> (g.tsx + g.tsy);
            int x = ti.tx * ti.TX + lx, y = ti.ty * ti.TY + ly, z = ti.tz * ti.TZ + lz;
            if (x >= g.nx || y >= g.ny || z >= g.nz)
                continue;
            int cidx = (lx + 1) + ti.BX * ((ly + 1) + ti.BY * (lz + ti.hz));
            int own = s_box[cidx];
            unsigned pos = pack(g, x, y, z);
            int l = neighbour_next(s_box, cidx, ti.BX, BXY, zr, own, -1);
            while (l != 0x10000) {
                rec[o++] = make_uint2(pos, (unsigned)own | ((unsigned)l << 16));
                l = neighbour_next(s_box, cidx, ti.BX, BXY, zr, own, l);
            }
        }
        if (threadIdx.x < 27) {
            int dx = (int)threadIdx.x % 3 - 1, dy = ((int)threadIdx.x / 3) % 3 - 1, dz = (int)threadIdx.x / 9 - 1;
            int x = ti.tx + dx, y = ti.ty + dy, z = ti.tz + dz;
            if (x >= 0 && x < g.ntx && y >= 0 && y < g.nty && z >= 0 && z < g.ntz)
                b.cand[x + g.ntx * (y + g.nty * z)] = 1;
        }
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
        ds->nflips = 0;
        ds->nflip_list = 0;
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
            long long na = b.st_n[a], nb = b.st_n[bl];
            double mua = (double)b.st_s1[a] * g.fx_inv / (double)na;
            double mub = (double)b.st_s1[bl] * g.fx_inv / (double)nb;
            float fb = (float)((double)nb / ((double)nb + 1.0));
            float fa = na > 1 ? (float)((double)na / ((double)na - 1.0)) : 0.f;
            float da = v - (float)mua, db = v - (float)mub;
            dext = fb * db * db - fa * da * da;
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
// One block per non-empty tile (the cell of the cell list).  The particles of
// all tiles overlapping the tile's box grown by h (the largest axis offset
// inside the support) are filtered to that box and staged in LDS in rounds of
// up to kStageCap; every core particle then scans the staged set.  Membership
// is exact integer arithmetic (d^2 < T); weights come from the table
// W[d^2] = K(sqrt(d^2)) built on the host in FP64.
__global__ __launch_bounds__(kBlock) void k_sobolev(Geom g, Bufs b, int cur, const float* __restrict__ in,
                                                   float* __restrict__ out, int gated)
{
    __shared__ unsigned s_pos[kStageCap];
    __shared__ unsigned s_ab[kStageCap];
    __shared__ float s_v[kStageCap];
    __shared__ float s_W[kMaxT];
    __shared__ unsigned s_wtot[kBlock / 64];
    DevState* ds = b.ds;
    if (gated && stopped(ds))
        return;
    for (int k = threadIdx.x; k < g.T; k += kBlock)
        s_W[k] = b.W[k];
    const unsigned na = ds->n_active[cur];
    const unsigned* ts = b.tstart[cur];
    const uint2* rec = b.rec[cur];
    const int TX = 1 << g.tsx, TY = 1 << g.tsy, TZ = 1 << g.tsz;
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    for (unsigned ai = blockIdx.x; ai < na; ai += gridDim.x) {
        unsigned t = b.active[cur][ai];
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
        for (unsigned cb = cs; cb < ce; cb += kBlock) {
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
                while (k < nnt && fill <= kStageCap - kBlock) {
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
                    for (int i = 0; i < kBlock / 64; ++i) {
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
                    qs += kBlock;
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
                __syncthreads();
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
}

// ------------------------------------------------------- acceptance of moves
//
// Every particle with gradient < 0 is a candidate; per pixel the smallest
// gradient wins (ties: first in order, i.e. smaller b).  Decisions read only
// gradients and records of state t, so the label field is updated in place.
// Region statistics follow exactly (integer deltas, merged per wave).
__global__ __launch_bounds__(kBlock) void k_flip(Geom g, Bufs b, const void* img, int cur,
                                                const float* __restrict__ grad)
{
    DevState* ds = b.ds;
    if (stopped(ds))
        return;
    const unsigned n = ds->n[cur];
    const uint2* rec = b.rec[cur];
    const int lane = lane_id();
    for (unsigned base = blockIdx.x * kBlock; base < n; base += gridDim.x * kBlock) {
        unsigned p = base + threadIdx.x;
        bool f = false;
        unsigned lin = 0;
        int a = 0, bb = 0;
        if (p < n) {
            uint2 r = rec[p];
            bool first = p == 0 || rec[p - 1].x != r.x;
            if (first) {
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
                    }
                }
                if (best >= 0) {
                    f = true;
                    int x, y, z;
                    unpack(g, r.x, x, y, z);
                    lin = (unsigned)lin_of(g, x, y, z);
                    a = (int)(r.y & 0xffffu);
                    bb = (int)(rec[best].y >> 16);
                }
            }
        }
        if (f)
            b.lab[lin] = (unsigned short)bb;
        unsigned long long m = __ballot(f);
        if (m == 0)
            continue;
        int leader = __ffsll((long long)m) - 1;
        unsigned cnt = (unsigned)__popcll(m), lbase = 0;
        if (lane == leader) {
            atomicAdd(&ds->nflips, cnt);
            lbase = atomicAdd(&ds->nflip_list, cnt);
        }
        lbase = __shfl(lbase, leader);
        if (f)
            b.flist[lbase + lanes_below(m)] = make_uint2(lin, (unsigned)a | ((unsigned)bb << 16));
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
                atomicAdd((unsigned long long*)&b.st_n[hi], (unsigned long long)dn);
                atomicAdd((unsigned long long*)&b.st_n[lo], (unsigned long long)(-dn));
                atomicAdd((unsigned long long*)&b.st_s1[hi], (unsigned long long)dq);
                atomicAdd((unsigned long long*)&b.st_s1[lo], (unsigned long long)(-dq));
            }
            pend = pend && !match;
        }
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
    hipLaunchKernelGGL(k_stats_init, dim3(grid_for(nvox, 4096)), dim3(kBlock), 0, s, g, b, img, nvox);
    return hipGetLastError();
}

hipError_t launch_l2diff(const Geom& g, const Bufs& b, const void* img, int cur, float* out, int gated, int grid,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_l2diff, dim3(grid), dim3(kBlock), 0, s, g, b, img, cur, out, gated);
    return hipGetLastError();
}

hipError_t launch_sobolev(const Geom& g, const Bufs& b, int cur, const float* in, float* out, int gated, int grid,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_sobolev, dim3(grid), dim3(kBlock), 0, s, g, b, cur, in, out, gated);
    return hipGetLastError();
}

hipError_t launch_flip(const Geom& g, const Bufs& b, const void* img, int cur, const float* grad, int grid,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_flip, dim3(grid), dim3(kBlock), 0, s, g, b, img, cur, grad);
    return hipGetLastError();
}

hipError_t launch_count(const Geom& g, const Bufs& b, int grid, int gated, hipStream_t s)
{
    hipLaunchKernelGGL(k_count, dim3(grid), dim3(kBlock), 0, s, g, b, gated);
    return hipGetLastError();
}

hipError_t launch_scan(const Geom& g, const Bufs& b, int cur, int nxt, int is_init, float tol, int32_t* d_nflips,
                       int gated, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, g, b, cur, nxt, is_init, tol, d_nflips, gated);
    return hipGetLastError();
}

hipError_t launch_write(const Geom& g, const Bufs& b, const void* img, int cur, int nxt, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_write, dim3(grid), dim3(kBlock), 0, s, g, b, img, cur, nxt);
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
