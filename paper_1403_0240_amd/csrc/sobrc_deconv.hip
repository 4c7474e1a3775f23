// Deconvolving image model (Methods, Eq. (8): J = s_theta(Gamma) * K) for
// the L2 gradient: a separable Gaussian point-spread function K, the region
// intensities theta by least squares for the labels at the start of the
// iteration, and per pixel the two images a move needs.
//
// A move of pixel x from a to b changes s(x) by delta = theta_b - theta_a
// (theta held fixed), so its data term is
//   sum_y [(R(y) - delta K(y - x))^2 - R(y)^2] = delta^2 N(x) - 2 delta C(x)
// with R = I - J, C = K (*) R (the PSF is symmetric: correlation equals
// convolution) and N(x) = sum over image pixels y of K(y - x)^2.  Sums run
// over the image (s and the products vanish outside it).  Every image here is
// made by separable passes along x, y (and z): HBM-bound streaming work, no
// MFMA.
#include "sobrc_dev.h"

namespace sobrc {

namespace {

__device__ __forceinline__ bool stopped_dc(const DevState* ds) { return (ds->err | ds->converged) != 0; }

// One pass along `axis` with zero padding: dst(y) = sum_t k[t] f(y + t e_axis).
// f: src if given, else the indicator of label `lab_i` (lab_i >= 0) or of the
// image itself (lab_i < 0) -- the first pass of a convolution of an indicator.
// The line segment a block works on, with its halo of r on each side, is
// staged in LDS; along x a block takes 256 outputs of one row, along y or z
// 64 columns of x times kPsfSeg outputs along the axis (coalesced loads).
constexpr int kPsfSeg = 16;

__device__ __forceinline__ float psf_src(const Bufs& b, const float* __restrict__ src, int lab_i, long long i)
{
    if (src)
        return src[i];
    return lab_i >= 0 ? (b.lab[i] == lab_i ? 1.f : 0.f) : 1.f;
}

__global__ __launch_bounds__(kBlock) void k_psf_pass_x(Geom g, Bufs b, Psf k, const float* __restrict__ src,
                                                      int lab_i, float* __restrict__ dst, int squared)
{
    __shared__ float s[kBlock + 2 * kPsfMaxR];
    if (stopped_dc(b.ds))
        return;
    const int x0 = blockIdx.x * kBlock, y = blockIdx.y, z = blockIdx.z;
    const long long row = (long long)g.nx * (y + (long long)g.ny * z);
    const int n = kBlock + 2 * k.r;
    for (int j = threadIdx.x; j < n; j += kBlock) {
        const int x = x0 - k.r + j;
        s[j] = (x >= 0 && x < g.nx) ? psf_src(b, src, lab_i, row + x) : 0.f;
    }
    __syncthreads();
    const float* taps = squared ? k.k2 : k.k;
    const int x = x0 + threadIdx.x;
    if (x >= g.nx)
        return;
    float acc = 0.f;
    for (int t = 0; t <= 2 * k.r; ++t)
        acc += taps[t] * s[threadIdx.x + t];
    dst[row + x] = acc;
}

// axis 1 (y) or 2 (z): blockIdx.x: 64 columns of x, blockIdx.y: kPsfSeg
// positions along the axis, blockIdx.z: the remaining coordinate.  Each thread
// issues all of its staging loads before storing any, then computes four
// consecutive outputs o0 .. o0 + 3 of its column tap by tap: at tap t a window
// of registers holds s[o0 + t .. o0 + t + 3], one new value is read from LDS
// per tap, and each output still adds its taps in order 0 .. 2r.
__global__ __launch_bounds__(kBlock) void k_psf_pass_yz(Geom g, Bufs b, Psf k, const float* __restrict__ src,
                                                       int lab_i, float* __restrict__ dst, int axis, int squared)
{
    constexpr int kRows = kPsfSeg + 2 * kPsfMaxR;
    constexpr int kGroups = kBlock / 64;               // row groups
    constexpr int kPer = (kRows + kGroups - 1) / kGroups;  // staged rows per thread
    constexpr int kOut = kPsfSeg / kGroups;             // consecutive outputs per thread
    static_assert(kPsfSeg % kGroups == 0, "outputs per thread");
    __shared__ float s[kRows][64];
    if (stopped_dc(b.ds))
        return;
    const int lx = threadIdx.x & 63, lr = threadIdx.x >> 6;  // column, row group
    const int x = blockIdx.x * 64 + lx;
    const int a0 = blockIdx.y * kPsfSeg;
    const int n_axis = axis == 1 ? g.ny : g.nz;
    const long long stride = axis == 1 ? g.nx : (long long)g.nx * g.ny;
    // base index of (x, a = 0, other coordinate)
    const long long base = axis == 1 ? (long long)g.nx * g.ny * blockIdx.z + x : (long long)g.nx * blockIdx.z + x;
    const int n = kPsfSeg + 2 * k.r;
    float v[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int j = lr + kGroups * q;
        const int a = a0 - k.r + j;
        v[q] = (j < n && x < g.nx && a >= 0 && a < n_axis) ? psf_src(b, src, lab_i, base + a * stride) : 0.f;
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int j = lr + kGroups * q;
        if (j < n)
            s[j][lx] = v[q];
    }
    __syncthreads();
    if (x >= g.nx)
        return;
    const float* taps = squared ? k.k2 : k.k;
    static_assert(kOut == 4, "a window of four outputs");
    const int o0 = kOut * lr, T = 2 * k.r;
    float acc[kOut] = {0.f, 0.f, 0.f, 0.f};
    float w0 = s[o0][lx], w1 = s[o0 + 1][lx], w2 = s[o0 + 2][lx];
    for (int t = 0; t <= T; ++t) {
        const float w3 = s[o0 + t + 3][lx];  // o0 + T + 3 <= kPsfSeg - 1 + T < n
        const float c = taps[t];
        acc[0] += c * w0;
        acc[1] += c * w1;
        acc[2] += c * w2;
        acc[3] += c * w3;
        w0 = w1;
        w1 = w2;
        w2 = w3;
    }
#pragma unroll
    for (int j = 0; j < kOut; ++j) {
        const int a = a0 + o0 + j;
        if (a < n_axis)
            dst[base + a * stride] = acc[j];
    }
}

// Partial sums of the normal equations of min sum_y (I(y) - sum_l theta_l
// u_l(y))^2 with u_l = K * chi_l (u_0 = K * 1 - sum_{l>0} u_l): the upper
// triangle of A_lm = sum u_l u_m, then c_l = sum u_l I.  FP64 per block.
__global__ __launch_bounds__(kBlock) void k_deconv_normal(Geom g, Bufs b, const void* img)
{
    __shared__ double s_part[kBlock / 64][kDeconvSums];
    if (stopped_dc(b.ds))
        return;
    const int M = g.max_labels;
    const long long nvox = (long long)g.nx * g.ny * g.nz;
    double acc[kDeconvSums];
#pragma unroll
    for (int j = 0; j < kDeconvSums; ++j)
        acc[j] = 0.0;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < nvox; i += (long long)gridDim.x * kBlock) {
        float u[kDeconvM];
        float rest = b.dw[i];
#pragma unroll
        for (int l = 1; l < kDeconvM; ++l) {
            u[l] = l < M ? b.du[(long long)(l - 1) * nvox + i] : 0.f;
            rest -= u[l];
        }
        u[0] = rest;
        const double v = g.img_u16 ? (double)((const unsigned short*)img)[i] : (double)((const float*)img)[i];
        int j = 0;
#pragma unroll
        for (int l = 0; l < kDeconvM; ++l)
#pragma unroll
            for (int m = l; m < kDeconvM; ++m)
                acc[j++] += (double)u[l] * (double)u[m];
#pragma unroll
        for (int l = 0; l < kDeconvM; ++l)
            acc[j++] += (double)u[l] * v;
    }
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < kDeconvSums; ++j) {
        double v = acc[j];
        for (int o = 32; o > 0; o >>= 1)
            v += __shfl_xor(v, o);
        if (lane == 0)
            s_part[wv][j] = v;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < kDeconvSums; j += kBlock) {
        double v = 0.0;
        for (int w = 0; w < kBlock / 64; ++w)
            v += s_part[w][j];
        b.dpart[(long long)blockIdx.x * kDeconvSums + j] = v;
    }
}

// theta: the partial sums folded, the labels without pixels set to 0, the
// normal equations solved by elimination.
__global__ __launch_bounds__(kBlock) void k_deconv_solve(Geom g, Bufs b, int nblocks)
{
    __shared__ double s_part[kBlock / 64][kDeconvSums];
    __shared__ double s_sum[kDeconvSums];
    if (stopped_dc(b.ds))
        return;
    // every thread folds a strided share of the blocks, then the waves combine
    double acc[kDeconvSums];
#pragma unroll
    for (int j = 0; j < kDeconvSums; ++j)
        acc[j] = 0.0;
    for (int k = threadIdx.x; k < nblocks; k += kBlock)
#pragma unroll
        for (int j = 0; j < kDeconvSums; ++j)
            acc[j] += b.dpart[(long long)k * kDeconvSums + j];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < kDeconvSums; ++j) {
        double v = acc[j];
        for (int o = 32; o > 0; o >>= 1)
            v += __shfl_xor(v, o);
        if (lane == 0)
            s_part[wv][j] = v;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < kDeconvSums; j += kBlock) {
        double v = 0.0;
        for (int w = 0; w < kBlock / 64; ++w)
            v += s_part[w][j];
        s_sum[j] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0)
        return;
    // the kDeconvM x kDeconvM system with identity rows for absent labels
    // (theta 0 there), eliminated with every index known at compile time
    const int M = g.max_labels;
    bool present[kDeconvM];
#pragma unroll
    for (int l = 0; l < kDeconvM; ++l)
        present[l] = l < M && b.st_n[l] > 0;
    double A[kDeconvM][kDeconvM], c[kDeconvM];
    int j = 0;
#pragma unroll
    for (int l = 0; l < kDeconvM; ++l)
#pragma unroll
        for (int m = l; m < kDeconvM; ++m, ++j) {
            const double v = present[l] && present[m] ? s_sum[j] : (l == m ? 1.0 : 0.0);
            A[l][m] = v;
            A[m][l] = v;
        }
#pragma unroll
    for (int l = 0; l < kDeconvM; ++l, ++j)
        c[l] = present[l] ? s_sum[j] : 0.0;
    bool ok = false;
#pragma unroll
    for (int l = 0; l < kDeconvM; ++l)
        ok = ok || present[l];
    // symmetric positive (semi)definite: elimination in order, pivots checked
#pragma unroll
    for (int col = 0; col < kDeconvM; ++col) {
        ok = ok && A[col][col] != 0.0;
        const double inv = ok ? 1.0 / A[col][col] : 0.0;
#pragma unroll
        for (int r = col + 1; r < kDeconvM; ++r) {
            const double f = A[r][col] * inv;
#pragma unroll
            for (int q = col; q < kDeconvM; ++q)
                A[r][q] -= f * A[col][q];
            c[r] -= f * c[col];
        }
    }
    double t[kDeconvM];
#pragma unroll
    for (int r = kDeconvM - 1; r >= 0; --r) {
        double acc = c[r];
#pragma unroll
        for (int q = r + 1; q < kDeconvM; ++q)
            acc -= A[r][q] * t[q];
        t[r] = ok ? acc / A[r][r] : 0.0;
    }
    for (int l = 0; l < M; ++l)
        b.dtheta[l] = ok && present[l] ? t[l] : 0.0;
}

// R = I - J with J = sum_l theta_l u_l.
__global__ __launch_bounds__(kBlock) void k_deconv_resid(Geom g, Bufs b, const void* img, float* __restrict__ out)
{
    if (stopped_dc(b.ds))
        return;
    const int M = g.max_labels;
    const long long nvox = (long long)g.nx * g.ny * g.nz;
    float th[kDeconvM];
    for (int l = 0; l < kDeconvM; ++l)
        th[l] = l < M ? (float)b.dtheta[l] : 0.f;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < nvox; i += (long long)gridDim.x * kBlock) {
        float rest = b.dw[i], J = 0.f;
#pragma unroll
        for (int l = 1; l < kDeconvM; ++l) {
            const float u = l < M ? b.du[(long long)(l - 1) * nvox + i] : 0.f;
            rest -= u;
            J += th[l] * u;
        }
        J += th[0] * rest;
        const float v = g.img_u16 ? (float)((const unsigned short*)img)[i] : ((const float*)img)[i];
        out[i] = v - J;
    }
}

int pixel_grid(const Geom& g)
{
    const long long nvox = (long long)g.nx * g.ny * g.nz;
    long long gb = (nvox + kBlock - 1) / kBlock;
    return (int)(gb < kDeconvGrid ? (gb < 1 ? 1 : gb) : kDeconvGrid);
}

// dst = K * f along every axis; f as in the passes; uses both scratch images.
void psf_conv(const Geom& g, const Bufs& b, const Psf& k, const float* src, int lab_i, float* dst, int squared,
              hipStream_t s)
{
    const dim3 B(kBlock);
    const dim3 gx((g.nx + kBlock - 1) / kBlock, g.ny, g.nz);
    const dim3 gy((g.nx + 63) / 64, (g.ny + kPsfSeg - 1) / kPsfSeg, g.nz);
    hipLaunchKernelGGL(k_psf_pass_x, gx, B, 0, s, g, b, k, src, lab_i, b.dt[0], squared);
    if (g.ndim == 3) {
        const dim3 gz((g.nx + 63) / 64, (g.nz + kPsfSeg - 1) / kPsfSeg, g.ny);
        hipLaunchKernelGGL(k_psf_pass_yz, gy, B, 0, s, g, b, k, b.dt[0], 0, b.dt[1], 1, squared);
        hipLaunchKernelGGL(k_psf_pass_yz, gz, B, 0, s, g, b, k, b.dt[1], 0, dst, 2, squared);
    } else {
        hipLaunchKernelGGL(k_psf_pass_yz, gy, B, 0, s, g, b, k, b.dt[0], 0, dst, 1, squared);
    }
}

}  // namespace

// Images that depend only on the geometry: K * 1 and the move's own term N.
hipError_t launch_deconv_init(const Geom& g, const Bufs& b, const Psf& k, hipStream_t s)
{
    psf_conv(g, b, k, nullptr, -1, b.dw, 0, s);
    psf_conv(g, b, k, nullptr, -1, b.dN, 1, s);
    return hipGetLastError();
}

// Per iteration, before the L2 gradient: u_l, theta, and C = K * (I - J).
hipError_t launch_deconv(const Geom& g, const Bufs& b, const Psf& k, const void* img, hipStream_t s)
{
    const long long nvox = (long long)g.nx * g.ny * g.nz;
    for (int l = 1; l < g.max_labels; ++l)
        psf_conv(g, b, k, nullptr, l, b.du + (long long)(l - 1) * nvox, 0, s);
    const int G = pixel_grid(g);
    hipLaunchKernelGGL(k_deconv_normal, dim3(G), dim3(kBlock), 0, s, g, b, img);
    hipLaunchKernelGGL(k_deconv_solve, dim3(1), dim3(kBlock), 0, s, g, b, G);
    // the residual goes to dC, its convolution through the scratch images back to dC
    hipLaunchKernelGGL(k_deconv_resid, dim3(G), dim3(kBlock), 0, s, g, b, img, b.dC);
    psf_conv(g, b, k, b.dC, 0, b.dC, 0, s);
    return hipGetLastError();
}

}  // namespace sobrc
