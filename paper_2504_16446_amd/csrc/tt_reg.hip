// Other objectives on the same operator (the paper's sect. 3.5, "Optimization"):
// the finite-difference Laplacian and Huber-norm regularisers of the tensor
// field and the fixed-step gradient-descent update with Nesterov momentum.
// All are HBM streams over coefficient-sized arrays.  Objective values are
// reduced without atomics: every block writes one float64 partial sum and a
// single-block pass adds them in block order, so values repeat bit for bit.
#include "tt_device.h"
#include "tt_internal.h"

namespace tt {

// One block per z-chunk of an (x, y) row of the coefficient volume
// c[x][y][z][C]: the chunk's zc * C floats are contiguous; the block stages
// them with one halo voxel on each side in LDS (for the +-C z neighbours,
// zero outside the volume) and reads the four adjacent rows' same chunk
// (x +- 1, y +- 1, zero outside) as float4 streams when rows are 16-byte
// aligned.  A ~12 KiB chunk instead of a whole staged row lets eight blocks
// share a CU.
//   ACC = false: out = Lap(in), value += lam sum Lap(in)^2 (if value)
//   ACC = true:  out += scale * Lap(in)
constexpr int kLapChunkFloats = 3072;  // target zc * C per block

typedef float f4r __attribute__((ext_vector_type(4)));

template <bool ACC>
__global__ __launch_bounds__(256) void k_laplacian(const float *__restrict__ in, int nx, int ny, int nz, int C,
                                                   int zc, float *__restrict__ out, float scale,
                                                   double *__restrict__ partials, int aligned)
{
    __shared__ double ws[4];
    extern __shared__ float rowc[];  // (zc + 2) C floats: voxels z0 - 1 .. z0 + zc
    const int nzc = (nz + zc - 1) / zc;
    const long long nchunks = (long long)nx * ny * nzc;
    double ss = 0.0;
    for (long long bi = blockIdx.x; bi < nchunks; bi += gridDim.x) {
        __syncthreads();  // the previous chunk's LDS reads are done
        const int chunk = (int)(bi % nzc);
        const long long rowi = bi / nzc;
        const int x = (int)(rowi / ny), y = (int)(rowi % ny);
        const int z0 = chunk * zc, z1 = min(nz, z0 + zc);
        const int len = (z1 - z0) * C;  // output floats of this block
        const long long rowlen = (long long)nz * C;
        const long long base = ((long long)x * ny + y) * rowlen + (long long)z0 * C;
        const float *r0 = in + base;
        const long long sx = (long long)ny * rowlen;
        const float *nb[4] = {x > 0 ? r0 - sx : nullptr, x + 1 < nx ? r0 + sx : nullptr, y > 0 ? r0 - rowlen : nullptr,
                              y + 1 < ny ? r0 + rowlen : nullptr};
        // rowc[C + e] = r0[e] for e in [-C, len + C), zero beyond the volume
        const int lo = z0 > 0 ? -C : 0, hi = z1 < nz ? len + C : len;
        for (int e = threadIdx.x - C; e < len + C; e += 256) rowc[C + e] = (e >= lo && e < hi) ? r0[e] : 0.0f;
        __syncthreads();
        // z0 C is a multiple of 4 (zc is), so with 4 | nz C every chunk starts 16-byte aligned
        const bool vec = aligned && (rowlen & 3) == 0;
        const int n4 = vec ? len / 4 : 0;
        for (int e4 = threadIdx.x; e4 < n4; e4 += 256) {
            f4r acc;
    #pragma unroll
            for (int l = 0; l < 4; ++l) acc[l] = rowc[C + 4 * e4 + l - C] + rowc[C + 4 * e4 + l + C] - 6.0f * rowc[C + 4 * e4 + l];
    #pragma unroll
            for (int q = 0; q < 4; ++q)
                if (nb[q]) acc += reinterpret_cast<const f4r *>(nb[q])[e4];
            f4r *o = reinterpret_cast<f4r *>(out + base) + e4;
            if (ACC) {
                *o = scale * acc + *o;
            } else {
                *o = acc;
    #pragma unroll
                for (int l = 0; l < 4; ++l) ss += (double)acc[l] * (double)acc[l];
            }
        }
        for (int e = 4 * n4 + threadIdx.x; e < len; e += 256) {
            float acc = rowc[e] + rowc[e + 2 * C] - 6.0f * rowc[C + e];
    #pragma unroll
            for (int q = 0; q < 4; ++q)
                if (nb[q]) acc += nb[q][e];
            if (ACC) {
                out[base + e] = fmaf(scale, acc, out[base + e]);
            } else {
                out[base + e] = acc;
                ss += (double)acc * (double)acc;
            }
        }
    }
    if (!ACC && partials) {
        const double t = block_sum(ss, ws);
        if (threadIdx.x == 0) partials[blockIdx.x] = t;
    }
}

// Sliding-window form for 16-byte aligned rows (nz C a multiple of 4): a
// block owns LY rows (y) x LZ floats (a float4-aligned segment of the
// contiguous z-C row) and marches along x through a range of planes.  The
// planes x - 1, x, x + 1 of its own elements stay in registers (each element
// is read from memory once per range, plus one plane at each end); plane x
// is staged in LDS with its y-halo rows (y0 - 1, y0 + LY) and z-halo (C
// floats on either side of the segment) for the four in-plane neighbours,
// zero outside the volume.  The next plane's loads are issued before the
// current plane is staged.
constexpr int kLY = 8, kLZ = 512;            // tile: 8 rows x 512 floats = 1024 float4
constexpr int kLF4 = kLY * kLZ / 4 / 256;    // float4 per thread

template <bool ACC>
__global__ __launch_bounds__(256) void k_laplacian_x(const float *__restrict__ in, int nx, int ny, int nz, int C,
                                                     int xr, float *__restrict__ out, float scale,
                                                     double *__restrict__ partials)
{
    __shared__ double ws[4];
    extern __shared__ float pl[];  // (kLY + 2) rows of kLZ + 2 CP floats, interior at column CP
    const long long R = (long long)nz * C;  // row length (floats), a multiple of 4
    const int nzs = (int)((R + kLZ - 1) / kLZ), nyt = (ny + kLY - 1) / kLY;
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int zs = lb % nzs, yt = (lb / nzs) % nyt, xg = lb / (nzs * nyt);
    const int y0 = yt * kLY;
    const long long e0 = (long long)zs * kLZ;
    const int x0 = xg * xr, x1 = min(nx, x0 + xr);
    const int CP = (C + 3) & ~3;  // halo width rounded to float4: every row and the interior 16-byte aligned
    const int L = kLZ + 2 * CP;
    const long long sx = (long long)ny * R;
    // this thread's float4s: element q -> (row, column) of the tile
    int rr[kLF4], cc[kLF4];
    bool ok[kLF4];
#pragma unroll
    for (int q = 0; q < kLF4; ++q) {
        const int f = threadIdx.x + 256 * q;
        rr[q] = f / (kLZ / 4);
        cc[q] = 4 * (f % (kLZ / 4));
        ok[q] = y0 + rr[q] < ny && e0 + cc[q] < R;
    }
    auto load_plane = [&](int x, f4r v[kLF4]) {
#pragma unroll
        for (int q = 0; q < kLF4; ++q) {
            v[q] = f4r{0.f, 0.f, 0.f, 0.f};
            if (x >= 0 && x < nx && ok[q])
                v[q] = *reinterpret_cast<const f4r *>(in + x * sx + (long long)(y0 + rr[q]) * R + e0 + cc[q]);
        }
    };
    f4r vp[kLF4], vc[kLF4], vn[kLF4];
    load_plane(x0 - 1, vp);
    load_plane(x0, vc);
    double ss = 0.0;
    for (int x = x0; x < x1; ++x) {
        load_plane(x + 1, vn);
        __syncthreads();  // the previous plane's LDS reads are done
        // interior
#pragma unroll
        for (int q = 0; q < kLF4; ++q) *reinterpret_cast<f4r *>(pl + (rr[q] + 1) * L + CP + cc[q]) = vc[q];
        // y-halo rows: columns [0, kLZ) of rows y0 - 1 and y0 + kLY
        const float *px = in + x * sx;
        for (int i = threadIdx.x; i < 2 * (kLZ / 4); i += 256) {
            const int side = i / (kLZ / 4), col = 4 * (i % (kLZ / 4));
            const int y = side ? y0 + kLY : y0 - 1;
            f4r v = f4r{0.f, 0.f, 0.f, 0.f};
            if (y >= 0 && y < ny && e0 + col < R) v = *reinterpret_cast<const f4r *>(px + (long long)y * R + e0 + col);
            *reinterpret_cast<f4r *>(pl + (side ? kLY + 1 : 0) * L + CP + col) = v;
        }
        // z-halo: C floats on either side of the segment, interior rows
        for (int i = threadIdx.x; i < 2 * kLY * C; i += 256) {
            const int row = i / (2 * C), j = i % (2 * C);
            const long long e = j < C ? e0 - C + j : e0 + kLZ + (j - C);
            const int y = y0 + row;
            float v = 0.0f;
            if (y < ny && e >= 0 && e < R) v = px[(long long)y * R + e];
            pl[(row + 1) * L + (j < C ? CP - C + j : CP + kLZ + (j - C))] = v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kLF4; ++q) {
            if (!ok[q]) continue;
            const float *p = pl + (rr[q] + 1) * L + CP + cc[q];
            f4r a = vp[q] + vn[q] - 6.0f * vc[q] + *reinterpret_cast<const f4r *>(p - L) +
                    *reinterpret_cast<const f4r *>(p + L);
#pragma unroll
            for (int l = 0; l < 4; ++l) a[l] += p[l - C] + p[l + C];
            f4r *o = reinterpret_cast<f4r *>(out + x * sx + (long long)(y0 + rr[q]) * R + e0 + cc[q]);
            if (ACC) {
                *o = scale * a + *o;
            } else {
                *o = a;
#pragma unroll
                for (int l = 0; l < 4; ++l) ss += (double)a[l] * (double)a[l];
            }
        }
#pragma unroll
        for (int q = 0; q < kLF4; ++q) {
            vp[q] = vc[q];
            vc[q] = vn[q];
        }
    }
    if (!ACC && partials) {
        const double t = block_sum(ss, ws);
        if (threadIdx.x == 0) partials[blockIdx.x] = t;
    }
}

hipError_t launch_laplacian_reg(const float *c, int nx, int ny, int nz, int C, double lam, float *work, float *grad,
                                double *value, double *partials, hipStream_t st)
{
    const long long R = (long long)nz * C;
    const bool aligned16 = ((reinterpret_cast<uintptr_t>(c) | reinterpret_cast<uintptr_t>(work) |
                             reinterpret_cast<uintptr_t>(grad)) & 15) == 0;
    if (aligned16 && (R & 3) == 0 && C <= kLapMaxC) {
        // x ranges: enough blocks to fill the chip (>= 2048), at most kReduceBlocks
        const long long cols = ((R + kLZ - 1) / kLZ) * ((ny + kLY - 1) / kLY);
        if (cols <= kReduceBlocks) {
            int nxg = (int)std::max(1LL, std::min<long long>(nx, (2048 + cols - 1) / cols));
            nxg = (int)std::min<long long>(nxg, kReduceBlocks / cols);
            const int xr = (nx + nxg - 1) / nxg;
            nxg = (nx + xr - 1) / xr;
            const int blocks = (int)(cols * nxg);
            const size_t lds = sizeof(float) * (size_t)(kLY + 2) * (kLZ + 2 * ((C + 3) & ~3));
            hipLaunchKernelGGL(k_laplacian_x<false>, dim3(blocks), dim3(256), lds, st, c, nx, ny, nz, C, xr, work,
                               0.0f, value ? partials : nullptr);
            if (value) {
                hipError_t e = launch_sum_partials(partials, blocks, value, lam, 1, st);
                if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL(k_laplacian_x<true>, dim3(blocks), dim3(256), lds, st, work, nx, ny, nz, C, xr, grad,
                               (float)(2.0 * lam), nullptr);
            return hipGetLastError();
        }
    }
    const int zc = std::max(4, (kLapChunkFloats / C) & ~3);  // multiple of 4
    const long long chunks = (long long)nx * ny * ((nz + zc - 1) / zc);
    if (C > kLapMaxC) return hipErrorNotSupported;
    const int blocks = (int)std::min<long long>(chunks, kReduceBlocks);
    const size_t lds = sizeof(float) * (size_t)(zc + 2) * C;
    const int aligned = ((reinterpret_cast<uintptr_t>(c) | reinterpret_cast<uintptr_t>(work) |
                          reinterpret_cast<uintptr_t>(grad)) & 15) == 0;
    hipLaunchKernelGGL(k_laplacian<false>, dim3(blocks), dim3(256), lds, st, c, nx, ny, nz, C, zc, work, 0.0f,
                       value ? partials : nullptr, aligned);
    if (value) {
        hipError_t e = launch_sum_partials(partials, blocks, value, lam, 1, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_laplacian<true>, dim3(blocks), dim3(256), lds, st, work, nx, ny, nz, C, zc, grad,
                       (float)(2.0 * lam), nullptr, aligned);
    return hipGetLastError();
}

// value += lam sum h(c), grad += lam h'(c); h(x) = x^2/(2 delta) for |x| <= delta, else |x| - delta/2.
// Float4 streams over the first 4 * (n / 4) elements when both arrays are
// 16-byte aligned, scalar for the rest.
__device__ __forceinline__ double huber_h(float x, float delta)
{
    const float a = fabsf(x);
    return a <= delta ? 0.5 * (double)x * (double)x / (double)delta : (double)a - 0.5 * (double)delta;
}

__global__ __launch_bounds__(256) void k_huber(const float *__restrict__ c, long long n, float delta, float lam,
                                               float *__restrict__ grad, double *__restrict__ partials, int aligned)
{
    __shared__ double ws[4];
    const float inv = 1.0f / delta;
    double hs = 0.0;
    const long long stride = (long long)gridDim.x * 256;
    long long n4 = aligned ? n / 4 : 0;
    for (long long e4 = blockIdx.x * 256LL + threadIdx.x; e4 < n4; e4 += stride) {
        const f4r x = reinterpret_cast<const f4r *>(c)[e4];
        f4r g = reinterpret_cast<const f4r *>(grad)[e4];
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            hs += huber_h(x[l], delta);
            g[l] = fmaf(lam, fminf(1.0f, fmaxf(-1.0f, x[l] * inv)), g[l]);
        }
        reinterpret_cast<f4r *>(grad)[e4] = g;
    }
    for (long long e = 4 * n4 + blockIdx.x * 256LL + threadIdx.x; e < n; e += stride) {
        const float x = c[e];
        hs += huber_h(x, delta);
        grad[e] = fmaf(lam, fminf(1.0f, fmaxf(-1.0f, x * inv)), grad[e]);
    }
    if (partials) {
        const double t = block_sum(hs, ws);
        if (threadIdx.x == 0) partials[blockIdx.x] = t;
    }
}

hipError_t launch_huber_reg(const float *c, long long n, double delta, double lam, float *grad, double *value,
                            double *partials, hipStream_t st)
{
    const int aligned = ((reinterpret_cast<uintptr_t>(c) | reinterpret_cast<uintptr_t>(grad)) & 15) == 0;
    const int blocks = std::max(1, (int)std::min<long long>((n / 4 + 255) / 256, kReduceBlocks));
    hipLaunchKernelGGL(k_huber, dim3(blocks), dim3(256), 0, st, c, n, (float)delta, (float)lam, grad,
                       value ? partials : nullptr, aligned);
    if (value) return launch_sum_partials(partials, blocks, value, (double)(float)lam, 1, st);
    return hipGetLastError();
}

// Huber loss on the residual r = I - data: y = w h'(r) (so that A^T y is the
// gradient), value += sum w h(r).
__global__ __launch_bounds__(256) void k_huber_loss(const float *__restrict__ I, const float *__restrict__ data,
                                                    const float *__restrict__ w, long long n, float delta,
                                                    float *__restrict__ y, double *__restrict__ partials)
{
    __shared__ double ws[4];
    const float inv = 1.0f / delta;
    double hs = 0.0;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const float r = I[e] - data[e], a = fabsf(r), wt = w ? w[e] : 1.0f;
        hs += (double)wt * (a <= delta ? 0.5 * (double)r * (double)r / (double)delta : (double)a - 0.5 * (double)delta);
        y[e] = wt * fminf(1.0f, fmaxf(-1.0f, r * inv));
    }
    if (partials) {
        const double t = block_sum(hs, ws);
        if (threadIdx.x == 0) partials[blockIdx.x] = t;
    }
}

hipError_t launch_huber_loss(const float *I, const float *data, const float *w, long long n, double delta, float *y,
                             double *value, double *partials, hipStream_t st)
{
    const int blocks = std::max(1, (int)std::min<long long>((n + 255) / 256, kReduceBlocks));
    hipLaunchKernelGGL(k_huber_loss, dim3(blocks), dim3(256), 0, st, I, data, w, n, (float)delta, y,
                       value ? partials : nullptr);
    if (value) return launch_sum_partials(partials, blocks, value, 1.0, 1, st);
    return hipGetLastError();
}

// value += scale * sum x^2 (float64)
__global__ __launch_bounds__(256) void k_sumsq(const float *__restrict__ x, long long n,
                                               double *__restrict__ partials)
{
    __shared__ double ws[4];
    double ss = 0.0;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const double v = x[e];
        ss += v * v;
    }
    const double t = block_sum(ss, ws);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

hipError_t launch_sumsq(const float *x, long long n, double scale, double *value, double *partials, hipStream_t st)
{
    const int blocks = std::max(1, (int)std::min<long long>((n + 255) / 256, kReduceBlocks));
    hipLaunchKernelGGL(k_sumsq, dim3(blocks), dim3(256), 0, st, x, n, partials);
    return launch_sum_partials(partials, blocks, value, scale, 1, st);
}

// c_new = y - step p g; y = c_new + m (c_new - c); c = c_new, with p a
// diagonal preconditioner (1 when null); float4 streams when aligned.
__global__ __launch_bounds__(256) void k_nesterov(float *__restrict__ c, float *__restrict__ y,
                                                  const float *__restrict__ g, const float *__restrict__ p,
                                                  long long n, float step, float m, int aligned)
{
    const long long stride = (long long)gridDim.x * 256;
    const long long n4 = aligned ? n / 4 : 0;
    for (long long e4 = blockIdx.x * 256LL + threadIdx.x; e4 < n4; e4 += stride) {
        const f4r yv = reinterpret_cast<const f4r *>(y)[e4];
        f4r gv = reinterpret_cast<const f4r *>(g)[e4];
        if (p) gv *= reinterpret_cast<const f4r *>(p)[e4];
        const f4r cv = reinterpret_cast<const f4r *>(c)[e4];
        const f4r cn = yv - step * gv;
        reinterpret_cast<f4r *>(y)[e4] = cn + m * (cn - cv);
        reinterpret_cast<f4r *>(c)[e4] = cn;
    }
    for (long long e = 4 * n4 + blockIdx.x * 256LL + threadIdx.x; e < n; e += stride) {
        const float gp = p ? g[e] * p[e] : g[e];
        const float cn = fmaf(-step, gp, y[e]);
        y[e] = fmaf(m, cn - c[e], cn);
        c[e] = cn;
    }
}

hipError_t launch_nesterov(float *c, float *y, const float *g, const float *p, long long n, float step, float m,
                           hipStream_t st)
{
    const int aligned = ((reinterpret_cast<uintptr_t>(c) | reinterpret_cast<uintptr_t>(y) |
                          reinterpret_cast<uintptr_t>(g) | reinterpret_cast<uintptr_t>(p)) & 15) == 0;
    const int blocks = (int)std::min<long long>((n / 4 + 255) / 256, 8192);
    hipLaunchKernelGGL(k_nesterov, dim3(std::max(blocks, 1)), dim3(256), 0, st, c, y, g, p, n, step, m, aligned);
    return hipGetLastError();
}

}  // namespace tt
