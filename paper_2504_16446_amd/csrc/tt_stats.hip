// Reductions over the normal operator's diagonal and over training inputs:
//   - the unit isotropic field u (u_{v,0} = 1, other coefficients 0);
//   - an exact selection (radix select on the float bit patterns) of the
//     lower median of one coefficient channel over the voxels inside a ball,
//     which scales the network input (A^T I divided by the median over the
//     support of (A^T A u)_{v,0});
//   - the diagonal preconditioner 1 / max((A^T A u)_{v,0}, floor * max_v(...))
//     shared by all coefficients of a voxel;
//   - per-channel mean and inverse standard deviation of a channels-last
//     array (the network's input standardisation).
// Every reduction uses integer histograms or fixed-order float64 partial sums,
// so results do not depend on the order in which blocks run.
#include "tt_device.h"
#include "tt_internal.h"

namespace tt {

__global__ __launch_bounds__(256) void k_fill_iso(float *__restrict__ u, long long nvox, int C)
{
    const long long n = nvox * C;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256)
        u[e] = (e % C) == 0 ? 1.0f : 0.0f;
}

hipError_t launch_fill_iso(float *u, long long nvox, int C, hipStream_t st)
{
    const long long n = nvox * C;
    const int g = (int)std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_iso, dim3(std::max(g, 1)), dim3(256), 0, st, u, nvox, C);
    return hipGetLastError();
}

// Monotone map of a float's bit pattern to an unsigned key (negative values
// below positive ones, each side in numeric order), and its inverse.
__device__ __forceinline__ unsigned float_key(float f)
{
    const unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_float(unsigned k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__device__ __forceinline__ bool in_ball(long long v, int nx, int ny, int nz, double r2)
{
    const int iz = (int)(v % nz);
    const long long t = v / nz;
    const int iy = (int)(t % ny), ix = (int)(t / ny);
    const double x = ix - 0.5 * (nx - 1), y = iy - 0.5 * (ny - 1), z = iz - 0.5 * (nz - 1);
    return x * x + y * y + z * z <= r2;
}

// Radix select in three passes of 11, 11 and 10 bits (high to low).  Device
// state: sel[0] = key prefix found so far, sel[1] = rank k still to find
// within the prefix, sel[2] = number of selected voxels; bins[2048] counts.
constexpr int kSelBins = 2048;
__device__ __forceinline__ int sel_shift(int pass) { return pass == 0 ? 21 : (pass == 1 ? 10 : 0); }
__device__ __forceinline__ int sel_width(int pass) { return pass == 2 ? 10 : 11; }

__global__ __launch_bounds__(256) void k_select_hist(const float *__restrict__ g, int nx, int ny, int nz, int C,
                                                     int ch, double r2, int pass,
                                                     const unsigned long long *__restrict__ sel,
                                                     unsigned *__restrict__ bins)
{
    __shared__ unsigned h[kSelBins];
    for (int i = threadIdx.x; i < kSelBins; i += 256) h[i] = 0u;
    __syncthreads();
    const int shift = sel_shift(pass), width = sel_width(pass);
    const unsigned prefix = pass == 0 ? 0u : (unsigned)sel[0];
    const long long nvox = (long long)nx * ny * nz;
    for (long long v = blockIdx.x * 256LL + threadIdx.x; v < nvox; v += (long long)gridDim.x * 256) {
        if (!in_ball(v, nx, ny, nz, r2)) continue;
        const unsigned key = float_key(g[v * C + ch]);
        if (pass > 0 && (key >> (shift + width)) != prefix) continue;
        atomicAdd(&h[(key >> shift) & ((1u << width) - 1u)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSelBins; i += 256)
        if (h[i]) atomicAdd(&bins[i], h[i]);
}

__global__ __launch_bounds__(256) void k_zero_u32(unsigned *__restrict__ p) { p[blockIdx.x * 256 + threadIdx.x] = 0u; }

// One thread: find the bin holding rank k, extend the prefix, clear the bins.
__global__ void k_select_step(int pass, unsigned long long *sel, unsigned *bins, float *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int width = sel_width(pass);
    if (pass == 0) {
        unsigned long long n = 0;
        for (int i = 0; i < kSelBins; ++i) n += bins[i];
        sel[2] = n;
        sel[1] = n > 0 ? (n - 1) / 2 : 0;  // the lower median
        sel[0] = 0;
    }
    unsigned long long k = sel[1], below = 0;
    int b = 0;
    for (; b < (1 << width); ++b) {
        if (below + bins[b] > k) break;
        below += bins[b];
    }
    if (b == (1 << width)) b = (1 << width) - 1;  // no selected voxel: any key
    sel[0] = (sel[0] << width) | (unsigned long long)b;
    sel[1] = k - below;
    for (int i = 0; i < kSelBins; ++i) bins[i] = 0u;
    if (pass == 2) out[0] = sel[2] > 0 ? key_float((unsigned)sel[0]) : __uint_as_float(0x7fc00000u);
}

size_t ball_median_work_bytes() { return sizeof(unsigned long long) * 4 + sizeof(unsigned) * kSelBins + 256; }

hipError_t launch_ball_median(const float *g, int nx, int ny, int nz, int C, int ch, double radius, void *work,
                              float *out, hipStream_t st)
{
    auto *sel = reinterpret_cast<unsigned long long *>(work);
    auto *bins = reinterpret_cast<unsigned *>(sel + 4);
    hipLaunchKernelGGL(k_zero_u32, dim3(kSelBins / 256), dim3(256), 0, st, bins);
    const long long nvox = (long long)nx * ny * nz;
    const int grid = (int)std::max<long long>(1, std::min<long long>((nvox + 255) / 256, 2048));
    for (int pass = 0; pass < 3; ++pass) {
        hipLaunchKernelGGL(k_select_hist, dim3(grid), dim3(256), 0, st, g, nx, ny, nz, C, ch, radius * radius, pass,
                           sel, bins);
        hipLaunchKernelGGL(k_select_step, dim3(1), dim3(64), 0, st, pass, sel, bins, out);
    }
    return hipGetLastError();
}

// Preconditioner: partial maxima of channel 0, then p[v][i] = 1 / max(d_v, floor * max d).
constexpr int kMaxBlocks = 1024;
__global__ __launch_bounds__(256) void k_ch0_max(const float *__restrict__ g, long long nvox, int C,
                                                 float *__restrict__ partial)
{
    __shared__ float ws[256];
    float m = -INFINITY;
    for (long long v = blockIdx.x * 256LL + threadIdx.x; v < nvox; v += (long long)gridDim.x * 256)
        m = fmaxf(m, g[v * C]);
    ws[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) ws[threadIdx.x] = fmaxf(ws[threadIdx.x], ws[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = ws[0];
}

__global__ __launch_bounds__(256) void k_precond_fill(float *__restrict__ p, long long nvox, int C, float floor_frac,
                                                      const float *__restrict__ partial, int npart)
{
    __shared__ float dmax;
    if (threadIdx.x == 0) {
        float m = -INFINITY;
        for (int i = 0; i < npart; ++i) m = fmaxf(m, partial[i]);
        dmax = m;
    }
    __syncthreads();
    const float lo = floor_frac * dmax;
    for (long long v = blockIdx.x * 256LL + threadIdx.x; v < nvox; v += (long long)gridDim.x * 256) {
        float *pv = p + v * C;
        const float r = 1.0f / fmaxf(pv[0], lo);
        for (int i = 0; i < C; ++i) pv[i] = r;
    }
}

hipError_t launch_voxel_precond(float *p, long long nvox, int C, float floor_frac, float *partial, hipStream_t st)
{
    const int grid = (int)std::max<long long>(1, std::min<long long>((nvox + 255) / 256, kMaxBlocks));
    hipLaunchKernelGGL(k_ch0_max, dim3(grid), dim3(256), 0, st, p, nvox, C, partial);
    hipLaunchKernelGGL(k_precond_fill, dim3(grid), dim3(256), 0, st, p, nvox, C, floor_frac, partial, grid);
    return hipGetLastError();
}

// Per-channel statistics of y = pre * x over x[v][cstride] (channels c < nch <= 64):
// pass 0 sums y, pass 1 sums (y - mean)^2.  Thread t handles channel t % 64 of
// voxel slots t / 64, so every block reduces its four slots in LDS and writes
// one float64 partial per channel; the final kernel adds the partials in
// block order.
constexpr int kStatBlocks = 1024;
template <int PASS>
__global__ __launch_bounds__(256) void k_chstats(const float *__restrict__ x, long long nvox, int cstride, int nch,
                                                 float pre, const double *__restrict__ mean,
                                                 double *__restrict__ partial)
{
    __shared__ double ws[256];
    const int ch = threadIdx.x & 63, slot = threadIdx.x >> 6;
    double acc = 0.0;
    if (ch < nch) {
        const double mu = PASS ? mean[ch] : 0.0;
        for (long long v = blockIdx.x * 4LL + slot; v < nvox; v += (long long)gridDim.x * 4) {
            const double y = (double)(pre * x[v * cstride + ch]);
            acc += PASS ? (y - mu) * (y - mu) : y;
        }
    }
    ws[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < 64 && ch < nch)
        partial[(long long)blockIdx.x * 64 + ch] = ((ws[ch] + ws[64 + ch]) + ws[128 + ch]) + ws[192 + ch];
}

template <int PASS>
__global__ void k_chstats_final(const double *__restrict__ partial, int nblocks, int nch, long long nvox,
                                double *__restrict__ mean, float *__restrict__ shift, float *__restrict__ scale)
{
    const int ch = threadIdx.x;
    if (ch >= nch) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partial[(long long)b * 64 + ch];
    if (PASS == 0) {
        mean[ch] = s / (double)nvox;
        shift[ch] = (float)(s / (double)nvox);
    } else {
        const double var = nvox > 1 ? s / (double)(nvox - 1) : 0.0;  // unbiased
        scale[ch] = (float)(1.0 / fmax(sqrt(var), 1e-12));
    }
}

size_t chstats_work_doubles() { return (size_t)kStatBlocks * 64 + 64; }

hipError_t launch_channel_stats(const float *x, long long nvox, int cstride, int nch, float pre, float *shift,
                                float *scale, double *work, hipStream_t st)
{
    double *partial = work, *mean = work + (size_t)kStatBlocks * 64;
    const int grid = (int)std::max<long long>(1, std::min<long long>((nvox + 3) / 4, kStatBlocks));
    hipLaunchKernelGGL(k_chstats<0>, dim3(grid), dim3(256), 0, st, x, nvox, cstride, nch, pre, mean, partial);
    hipLaunchKernelGGL(k_chstats_final<0>, dim3(1), dim3(64), 0, st, partial, grid, nch, nvox, mean, shift, scale);
    hipLaunchKernelGGL(k_chstats<1>, dim3(grid), dim3(256), 0, st, x, nvox, cstride, nch, pre, mean, partial);
    hipLaunchKernelGGL(k_chstats_final<1>, dim3(1), dim3(64), 0, st, partial, grid, nch, nvox, mean, shift, scale);
    return hipGetLastError();
}

}  // namespace tt
