// Other objectives on the same operator (the paper's sect. 3.5, "Optimization"):
// the finite-difference Laplacian and Huber-norm regularisers of the tensor
// field and the fixed-step gradient-descent update with Nesterov momentum.
// All are HBM streams over coefficient-sized arrays.
#include "tt_device.h"
#include "tt_internal.h"

namespace tt {

// One block per (x, y) row of the coefficient volume c[x][y][z][C]: the row's
// z * C floats are contiguous, z neighbours are +-C inside the row, y and x
// neighbours are the same offsets in the adjacent rows (zero outside).
//   ACC = false: out = Lap(in), value += lam sum Lap(in)^2 (if value)
//   ACC = true:  out += scale * Lap(in)
template <bool ACC>
__global__ __launch_bounds__(256) void k_laplacian(const float *__restrict__ in, int nx, int ny, int nz, int C,
                                                   float *__restrict__ out, float scale, double lam,
                                                   double *__restrict__ value)
{
    __shared__ double ws[4];
    const int x = blockIdx.x / ny, y = blockIdx.x % ny;
    const int row = nz * C;  // < 2^31 (checked by the caller)
    const long long base = ((long long)x * ny + y) * row;
    const float *r0 = in + base;
    const float *rxm = x > 0 ? r0 - (long long)ny * row : nullptr;
    const float *rxp = x + 1 < nx ? r0 + (long long)ny * row : nullptr;
    const float *rym = y > 0 ? r0 - row : nullptr;
    const float *ryp = y + 1 < ny ? r0 + row : nullptr;
    double ss = 0.0;
    const float invC = 1.0f / (float)C;  // exact quotient: e < 2^22 and C <= 2^8 here
    for (int e = threadIdx.x; e < row; e += 256) {
        const int z = C <= 256 && row < (1 << 22) ? (int)(((float)e + 0.5f) * invC) : e / C;
        const float v = r0[e];
        float acc = -6.0f * v;
        if (z > 0) acc += r0[e - C];
        if (z + 1 < nz) acc += r0[e + C];
        if (rym) acc += rym[e];
        if (ryp) acc += ryp[e];
        if (rxm) acc += rxm[e];
        if (rxp) acc += rxp[e];
        if (ACC) {
            out[base + e] = fmaf(scale, acc, out[base + e]);
        } else {
            out[base + e] = acc;
            ss += (double)acc * (double)acc;
        }
    }
    if (!ACC && value) {
        const double t = block_sum(ss, ws);
        if (threadIdx.x == 0) atomicAdd(value, lam * t);
    }
}

hipError_t launch_laplacian_reg(const float *c, int nx, int ny, int nz, int C, double lam, float *work, float *grad,
                                double *value, hipStream_t st)
{
    const long long rows = (long long)nx * ny;
    if (rows > 0x7fffffffLL || (long long)nz * C > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_laplacian<false>, dim3((unsigned)rows), dim3(256), 0, st, c, nx, ny, nz, C, work, 0.0f, lam,
                       value);
    hipLaunchKernelGGL(k_laplacian<true>, dim3((unsigned)rows), dim3(256), 0, st, work, nx, ny, nz, C, grad,
                       (float)(2.0 * lam), 0.0, nullptr);
    return hipGetLastError();
}

// value += lam sum h(c), grad += lam h'(c); h(x) = x^2/(2 delta) for |x| <= delta, else |x| - delta/2.
__global__ __launch_bounds__(256) void k_huber(const float *__restrict__ c, long long n, float delta, float lam,
                                               float *__restrict__ grad, double *__restrict__ value)
{
    __shared__ double ws[4];
    const float inv = 1.0f / delta;
    double hs = 0.0;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const float x = c[e], a = fabsf(x);
        hs += a <= delta ? 0.5 * (double)x * (double)x / (double)delta : (double)a - 0.5 * (double)delta;
        grad[e] = fmaf(lam, fminf(1.0f, fmaxf(-1.0f, x * inv)), grad[e]);
    }
    if (value) {
        const double t = block_sum(hs, ws);
        if (threadIdx.x == 0) atomicAdd(value, (double)lam * t);
    }
}

hipError_t launch_huber_reg(const float *c, long long n, double delta, double lam, float *grad, double *value,
                            hipStream_t st)
{
    const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_huber, dim3(std::max(blocks, 1)), dim3(256), 0, st, c, n, (float)delta, (float)lam, grad,
                       value);
    return hipGetLastError();
}

// Huber loss on the residual r = I - data: y = w h'(r) (so that A^T y is the
// gradient), value += sum w h(r).
__global__ __launch_bounds__(256) void k_huber_loss(const float *__restrict__ I, const float *__restrict__ data,
                                                    const float *__restrict__ w, long long n, float delta,
                                                    float *__restrict__ y, double *__restrict__ value)
{
    __shared__ double ws[4];
    const float inv = 1.0f / delta;
    double hs = 0.0;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const float r = I[e] - data[e], a = fabsf(r), wt = w ? w[e] : 1.0f;
        hs += (double)wt * (a <= delta ? 0.5 * (double)r * (double)r / (double)delta : (double)a - 0.5 * (double)delta);
        y[e] = wt * fminf(1.0f, fmaxf(-1.0f, r * inv));
    }
    if (value) {
        const double t = block_sum(hs, ws);
        if (threadIdx.x == 0) atomicAdd(value, t);
    }
}

hipError_t launch_huber_loss(const float *I, const float *data, const float *w, long long n, double delta, float *y,
                             double *value, hipStream_t st)
{
    const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_huber_loss, dim3(std::max(blocks, 1)), dim3(256), 0, st, I, data, w, n, (float)delta, y, value);
    return hipGetLastError();
}

// value += scale * sum x^2 (float64)
__global__ __launch_bounds__(256) void k_sumsq(const float *__restrict__ x, long long n, double scale,
                                               double *__restrict__ value)
{
    __shared__ double ws[4];
    double ss = 0.0;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const double v = x[e];
        ss += v * v;
    }
    const double t = block_sum(ss, ws);
    if (threadIdx.x == 0) atomicAdd(value, scale * t);
}

hipError_t launch_sumsq(const float *x, long long n, double scale, double *value, hipStream_t st)
{
    const int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_sumsq, dim3(std::max(blocks, 1)), dim3(256), 0, st, x, n, scale, value);
    return hipGetLastError();
}

// c_new = y - step g; y = c_new + m (c_new - c); c = c_new.
__global__ __launch_bounds__(256) void k_nesterov(float *__restrict__ c, float *__restrict__ y,
                                                  const float *__restrict__ g, long long n, float step, float m)
{
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const float cn = fmaf(-step, g[e], y[e]);
        y[e] = fmaf(m, cn - c[e], cn);
        c[e] = cn;
    }
}

hipError_t launch_nesterov(float *c, float *y, const float *g, long long n, float step, float m, hipStream_t st)
{
    const int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_nesterov, dim3(std::max(blocks, 1)), dim3(256), 0, st, c, y, g, n, step, m);
    return hipGetLastError();
}

}  // namespace tt
