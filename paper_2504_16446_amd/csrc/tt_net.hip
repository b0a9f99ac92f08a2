// Warm-start network layers on gfx950: 3x3x3 convolutions (stride 1, zero
// padding 1) in channels-last layout as implicit GEMMs on bf16 MFMA with fp32
// accumulation, their gradients, Adam, the MSE loss and layout packing.
//
//   forward  y[v, co] = b[co] + sum_d sum_ci x[v + d - 1, ci] w[d, ci, co]
//   dgrad    gx[v, ci] = sum_d sum_co gy[v - d + 1, co] w[d, ci, co]
//            = the forward with w'[d][co][ci] = w[2 - d][ci][co]
//   wgrad    gw[d, ci, co] = sum_v x[v + d - 1, ci] gy[v, co]
//
// Channel counts are 32 or 64 (the network pads 28 to 32).  Tap index
// d = (dx * 3 + dy) * 3 + dz.  Activations are bf16, weights fp32 masters
// with bf16 MFMA-ordered copies.
#include "tt_device.h"
#include "tt_internal.h"

namespace tt {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));    // eight bf16 bit patterns
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;

// gfx950 v_mfma_f32_16x16x32_bf16: D[16x16] += A[16x32] B[32x16].  Lane l
// supplies row (A) / column (B) l % 16 and eight consecutive k of the group
// l / 16; D as for the 16x16x16 forms (lane holds rows 4 (l / 16) + r of
// column l % 16).  A and B take the same k order, so the per-lane k
// assignment inside a group does not change the sum.
__device__ __forceinline__ f4 mfma_bf16(s8 a, s8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0,
                                                   0);
}

__device__ __forceinline__ u16 f2bf(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}

__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float((unsigned)h << 16); }

// Spatial tile of one block: 4 (x) x 4 (y) x 8 (z) = 128 voxels, z fastest.
constexpr int TX = 4, TY = 4, TZ = 8, TV = TX * TY * TZ;
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2, HV = HX * HY * HZ;

enum { EPI_RELU_BF16 = 0, EPI_BIAS_F32 = 1, EPI_MASK_BF16 = 2 };

// ---------------------------------------------------------------------------
// Convolution as implicit GEMM: rows = the block's 128 voxels, columns = CO,
// K = 27 taps x CI.  The (tile + 1)-halo of the input is staged in LDS once;
// each tap reads it at a shifted position.  Wave w owns voxels 32w..32w+31
// (two 16-row tiles) and all CO/16 column tiles.
// ---------------------------------------------------------------------------
template <int CI, int CO, int EPI>
__global__ __launch_bounds__(256) void k_conv(const u16 *__restrict__ x, const s8 *__restrict__ wsw,
                                              const float *__restrict__ bias, const u16 *__restrict__ mask,
                                              void *__restrict__ y, int X, int Y, int Z)
{
    constexpr int LD = CI + 8;  // padded channel stride of the halo (bf16)
    __shared__ u16 halo[HV * LD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nbz = (Z + TZ - 1) / TZ, nby = (Y + TY - 1) / TY, nbx = (X + TX - 1) / TX;
    int b = blockIdx.x;
    const int bz = b % nbz;
    b /= nbz;
    const int by = b % nby;
    b /= nby;
    const int bx = b % nbx;
    const int n = b / nbx;
    const int x0 = bx * TX - 1, y0 = by * TY - 1, z0 = bz * TZ - 1;
    const long long vol = (long long)X * Y * Z;
    const u16 *xn = x + (long long)n * vol * CI;
    // stage the halo: 16-byte chunks of 8 channels
    constexpr int CH = CI / 8;
    for (int e = tid; e < HV * CH; e += 256) {
        const int p = e / CH, ch = e % CH;
        const int hz = p % HZ, hy = (p / HZ) % HY, hx = p / (HZ * HY);
        const int gx = x0 + hx, gy = y0 + hy, gz = z0 + hz;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (gx >= 0 && gx < X && gy >= 0 && gy < Y && gz >= 0 && gz < Z)
            val = *reinterpret_cast<const uint4 *>(xn + (((long long)gx * Y + gy) * Z + gz) * CI + ch * 8);
        *reinterpret_cast<uint4 *>(halo + p * LD + ch * 8) = val;
    }
    __syncthreads();

    constexpr int NT = CO / 16, CB = CI / 32;
    f4 acc[2][NT];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
    // the two voxel rows this lane supplies to the A operand
    int hp[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        const int vt = wave * 32 + mt * 16 + (lane & 15);
        const int tz = vt % TZ, ty = (vt / TZ) % TY, tx = vt / (TZ * TY);
        hp[mt] = (tx * HY + ty) * HZ + tz;
    }
    const int kq = lane >> 4;
    for (int tap = 0; tap < 27; ++tap) {
        const int dx = tap / 9, dy = (tap / 3) % 3, dz = tap % 3;
        const int toff = (dx * HY + dy) * HZ + dz;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            s8 bv[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) bv[nt] = wsw[((tap * CB + cb) * NT + nt) * 64 + lane];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                const s8 av = *reinterpret_cast<const s8 *>(halo + (hp[mt] + toff) * LD + cb * 32 + 8 * kq);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma_bf16(av, bv[nt], acc[mt][nt]);
            }
        }
    }
    // epilogue: lane holds rows (voxels) 16 mt + 4 kq + r of column (channel) 16 nt + lane % 16
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int vt = wave * 32 + mt * 16 + 4 * kq + r;
            const int tz = vt % TZ, ty = (vt / TZ) % TY, tx = vt / (TZ * TY);
            const int gx = x0 + 1 + tx, gy = y0 + 1 + ty, gz = z0 + 1 + tz;
            if (gx >= X || gy >= Y || gz >= Z) continue;
            const long long vi = (long long)n * vol + ((long long)gx * Y + gy) * Z + gz;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int co = nt * 16 + (lane & 15);
                float v = acc[mt][nt][r];
                if (EPI == EPI_RELU_BF16) {
                    v = fmaxf(v + bias[co], 0.0f);
                    reinterpret_cast<u16 *>(y)[vi * CO + co] = f2bf(v);
                } else if (EPI == EPI_BIAS_F32) {
                    reinterpret_cast<float *>(y)[vi * CO + co] = v + bias[co];
                } else {
                    v = bf2f(mask[vi * CO + co]) > 0.0f ? v : 0.0f;
                    reinterpret_cast<u16 *>(y)[vi * CO + co] = f2bf(v);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradient, split over K (voxels): block (tap, chunk) accumulates
// gw[tap] over the voxel tiles t = chunk, chunk + nchunks, ... and writes its
// CI x CO partial; a second kernel sums the partials in chunk order.
// Tiles are staged channel-major in LDS so both MFMA operands read 8
// consecutive voxels of one channel.  Staging item (row, octet): the 8
// voxels of one z-row of the tile (contiguous in the tile's voxel order) and
// 8 channels; the thread loads the 8 voxels' 16-byte channel octets,
// transposes the 8 x 8 block in registers and writes 8 rows of 16 bytes.
// The next tile's loads are issued before the current tile's MFMAs.
// ---------------------------------------------------------------------------
struct Oct8 {
    uint4 v[8];
};

// w[q] = the q-th channel of the 8 voxels in r.v[0..7], as 8 packed bf16
__device__ __forceinline__ uint4 oct_column(const Oct8 &r, int q)
{
    unsigned h[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const unsigned word = (q >> 1) == 0 ? r.v[i].x : (q >> 1) == 1 ? r.v[i].y : (q >> 1) == 2 ? r.v[i].z : r.v[i].w;
        h[i] = (q & 1) ? (word >> 16) : (word & 0xffffu);
    }
    return make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
}

template <int CI, int CO>
__global__ __launch_bounds__(256) void k_wgrad(const u16 *__restrict__ x, const u16 *__restrict__ gy, int N, int X,
                                               int Y, int Z, int nchunks, float *__restrict__ part)
{
    constexpr int LDV = TV + 8;  // padded voxel stride (bf16; 16-byte rows)
    __shared__ __attribute__((aligned(16))) u16 xs[CI * LDV];
    __shared__ __attribute__((aligned(16))) u16 gs[CO * LDV];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tap = blockIdx.x / nchunks, chunk = blockIdx.x % nchunks;
    const int dx = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dz = tap % 3 - 1;
    const int nbz = (Z + TZ - 1) / TZ, nby = (Y + TY - 1) / TY, nbx = (X + TX - 1) / TX;
    const int ntiles = N * nbx * nby * nbz;
    const long long vol = (long long)X * Y * Z;
    constexpr int MT = CI / 16, NT = CO / 16;
    constexpr int TPW = MT * NT / 4;  // output tiles per wave
    constexpr int ROWS = TX * TY;     // z-rows of TZ = 8 voxels per tile
    constexpr int XI = ROWS * (CI / 8), GI = ROWS * (CO / 8);  // staging items of x and gy
    static_assert(TZ == 8 && XI + GI <= 256, "one staging item per thread");
    // this thread's staging item: x rows first, then gy rows
    const bool is_x = tid < XI, has_item = tid < XI + GI;
    const int it = is_x ? tid : tid - XI;
    const int row = it % ROWS, oct = it / ROWS;
    const int rtx = row / TY, rty = row % TY;
    const int cstride = is_x ? CI : CO;
    const u16 *src = is_x ? x : gy;
    const int sx = is_x ? dx : 0, sy = is_x ? dy : 0, sz = is_x ? dz : 0;
    u16 *dst = (is_x ? xs : gs) + oct * 8 * LDV + row * TZ;

    auto load = [&](int t, Oct8 &r) {
#pragma unroll
        for (int i = 0; i < 8; ++i) r.v[i] = make_uint4(0, 0, 0, 0);
        if (!has_item || t >= ntiles) return;
        int b = t;
        const int bz = b % nbz;
        b /= nbz;
        const int by = b % nby;
        b /= nby;
        const int bx = b % nbx;
        const int n = b / nbx;
        const int ox = bx * TX + rtx, oy = by * TY + rty;
        const int gx = ox + sx, gyy = oy + sy;
        if (ox >= X || oy >= Y || gx < 0 || gx >= X || gyy < 0 || gyy >= Y) return;
        const u16 *p = src + ((long long)n * vol + ((long long)gx * Y + gyy) * Z) * cstride + oct * 8;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int oz = bz * TZ + i, gz = oz + sz;
            if (oz < Z && gz >= 0 && gz < Z) r.v[i] = *reinterpret_cast<const uint4 *>(p + (long long)gz * cstride);
        }
    };

    f4 acc[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i) acc[i] = f4{0.f, 0.f, 0.f, 0.f};
    const int kq = lane >> 4;
    Oct8 cur;
    load(chunk, cur);
    for (int t = chunk; t < ntiles; t += nchunks) {
        __syncthreads();  // the previous tile's MFMA reads are done
        if (has_item) {
#pragma unroll
            for (int q = 0; q < 8; ++q) *reinterpret_cast<uint4 *>(dst + q * LDV) = oct_column(cur, q);
        }
        __syncthreads();
        load(t + nchunks, cur);  // next tile in flight during the MFMAs
        // gw[ci][co] += sum_v xs[ci][v] gs[co][v]: M = CI, N = CO, K = 128 voxels
#pragma unroll
        for (int ks = 0; ks < TV / 32; ++ks) {
#pragma unroll
            for (int i = 0; i < TPW; ++i) {
                const int tile = wave * TPW + i;
                const int mt = tile / NT, nt = tile % NT;
                const s8 av = *reinterpret_cast<const s8 *>(xs + (mt * 16 + (lane & 15)) * LDV + ks * 32 + 8 * kq);
                const s8 bv = *reinterpret_cast<const s8 *>(gs + (nt * 16 + (lane & 15)) * LDV + ks * 32 + 8 * kq);
                acc[i] = mfma_bf16(av, bv, acc[i]);
            }
        }
    }
    // partial[tap][chunk][ci][co]; lane holds rows ci = 16 mt + 4 kq + r, column co = 16 nt + lane % 16
    float *pp = part + ((long long)tap * nchunks + chunk) * CI * CO;
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
        const int tile = wave * TPW + i;
        const int mt = tile / NT, nt = tile % NT;
#pragma unroll
        for (int r = 0; r < 4; ++r) pp[(mt * 16 + 4 * kq + r) * CO + nt * 16 + (lane & 15)] = acc[i][r];
    }
}

__global__ __launch_bounds__(256) void k_wgrad_reduce(const float *__restrict__ part, int nchunks, int per_tap,
                                                      float *__restrict__ gw)
{
    const int tap = blockIdx.y;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < per_tap; e += gridDim.x * 256) {
        float s = 0.0f;
        for (int c = 0; c < nchunks; ++c) s += part[((long long)tap * nchunks + c) * per_tap + e];
        gw[(long long)tap * per_tap + e] = s;
    }
}

// bias gradient, stage 1: partial[blk][co] = sum over this block's voxels of gy[v][co]
__global__ __launch_bounds__(256) void k_bias_partial(const u16 *__restrict__ gy, long long nvox, int CO,
                                                      float *__restrict__ partial)
{
    __shared__ float sh[256];
    const int per = 256 / CO;  // voxels handled side by side
    const int c = threadIdx.x % CO, vo = threadIdx.x / CO;
    float s = 0.0f;
    for (long long v = (long long)blockIdx.x * per + vo; v < nvox; v += (long long)gridDim.x * per)
        s += bf2f(gy[v * CO + c]);
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < CO) {
        float t = 0.0f;
        for (int i = 0; i < per; ++i) t += sh[i * CO + threadIdx.x];
        partial[(long long)blockIdx.x * CO + threadIdx.x] = t;
    }
}

// bias gradient, stage 2: gb[co] = sum over blocks, one block per channel: thread t
// adds partials t, t + 256, ... in order, then a fixed-shape tree in LDS
__global__ __launch_bounds__(256) void k_bias_reduce(const float *__restrict__ partial, int nblk, int CO, float *gb)
{
    __shared__ float sh[256];
    const int c = blockIdx.x, t = threadIdx.x;
    float s = 0.0f;
    for (int b = t; b < nblk; b += 256) s += partial[(long long)b * CO + c];
    sh[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) gb[c] = sh[0];
}

// MFMA-ordered bf16 copies of w[27][ci][co]: forward (B[k = ci][n = co]) and
// dgrad (w'[d][co][ci] = w[26 - d][ci][co], B[k = co][n = ci]), eight k per lane.
__global__ __launch_bounds__(256) void k_swizzle(const float *__restrict__ w, int CI, int CO, s8 *__restrict__ wf,
                                                 s8 *__restrict__ wd)
{
    const int total = 27 * (CI / 32) * (CO / 16) * 64;  // = 27 (CO / 32) (CI / 16) 64
    for (int e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256) {
        const int l = e % 64;
        int r = e / 64;
        // forward: e = ((tap * CB + cb) * NT + nt) * 64 + l with CB = CI/32, NT = CO/16
        {
            const int nt = r % (CO / 16), cb = (r / (CO / 16)) % (CI / 32), tap = r / ((CO / 16) * (CI / 32));
            const int co = nt * 16 + l % 16, ci0 = cb * 32 + 8 * (l / 16);
            s8 v;
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = (short)f2bf(w[((long long)tap * CI + ci0 + q) * CO + co]);
            wf[e] = v;
        }
        // dgrad: input channels CO, output channels CI: e = ((tap * (CO/32) + cb) * (CI/16) + nt) * 64 + l
        {
            const int nt = r % (CI / 16), cb = (r / (CI / 16)) % (CO / 32), tap = r / ((CI / 16) * (CO / 32));
            const int src = 26 - tap;
            const int ci = nt * 16 + l % 16, co0 = cb * 32 + 8 * (l / 16);
            s8 v;
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = (short)f2bf(w[((long long)src * CI + ci) * CO + co0 + q]);
            wd[e] = v;
        }
    }
}

__global__ __launch_bounds__(256) void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                                              float *__restrict__ v, long long n, float lr, float b1, float b2,
                                              float eps, float c1, float c2)
{
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const float ge = g[e];
        const float me = b1 * m[e] + (1.0f - b1) * ge;
        const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
        m[e] = me;
        v[e] = ve;
        w[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
    }
}

// gy = scale (y - t) on the first creal of cpad channels (0 elsewhere), in bf16;
// partials of sum (y - t)^2 in float64.
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ y, const float *__restrict__ t, long long nvox,
                                             int cpad, int creal, float scale, u16 *__restrict__ gy,
                                             double *__restrict__ partials)
{
    __shared__ double ws[4];
    double s = 0.0;
    const long long n = nvox * cpad;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const long long v = e / cpad;
        const int c = (int)(e % cpad);
        float d = 0.0f;
        if (c < creal) {
            d = y[e] - t[v * creal + c];
            s += (double)d * d;
        }
        if (gy) gy[e] = f2bf(scale * d);
    }
    s = block_sum(s, ws);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// out[v][c] = bf16(scale[c] * (x[v][c] - shift[c])) for c < cin, 0 for cin <= c < cpad
__global__ __launch_bounds__(256) void k_pack(const float *__restrict__ x, long long nvox, int cin, int cpad,
                                              float pre, const float *__restrict__ shift,
                                              const float *__restrict__ scale, u16 *__restrict__ out)
{
    const long long n = nvox * cpad;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const long long v = e / cpad;
        const int c = (int)(e % cpad);
        float val = 0.0f;
        if (c < cin) {
            val = pre * x[v * cin + c];
            if (shift) val -= shift[c];
            if (scale) val *= scale[c];
        }
        out[e] = f2bf(val);
    }
}

// Patchwise inference.  Tiles of T^3 voxels at per-axis origins ox[], oy[], oz[]
// (tile t = (i nx_t + j) ny_t... in x-major order).
// gather: out[t][T^3][cpad] = bf16(scale[c] (pre vol[o_t + u][c] - shift[c])) for c < cin.
__global__ __launch_bounds__(256) void k_tile_gather(const float *__restrict__ vol, int X, int Y, int Z, int cv, int cin,
                                                     int cpad, const int *__restrict__ ox, int ntx,
                                                     const int *__restrict__ oy, int nty, const int *__restrict__ oz,
                                                     int ntz, int T, float pre, const float *__restrict__ shift,
                                                     const float *__restrict__ scale, int t0, int nt,
                                                     u16 *__restrict__ out)
{
    const long long per = (long long)T * T * T * cpad;
    const long long n = per * nt;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const int t = t0 + (int)(e / per);
        long long r = e % per;
        const int c = (int)(r % cpad);
        r /= cpad;
        const int uz = (int)(r % T), uy = (int)((r / T) % T), ux = (int)(r / ((long long)T * T));
        const int iz = t % ntz, iy = (t / ntz) % nty, ix = t / (ntz * nty);
        const int gx = ox[ix] + ux, gy = oy[iy] + uy, gz = oz[iz] + uz;
        float v = 0.0f;
        if (c < cin && gx < X && gy < Y && gz < Z) {
            v = pre * vol[(((long long)gx * Y + gy) * Z + gz) * cv + c];
            if (shift) v -= shift[c];
            if (scale) v *= scale[c];
        }
        out[e] = f2bf(v);
    }
}

// Separable blending weight of position u in a tile starting at o along an
// axis of length n: a linear ramp over `ramp` voxels on sides that overlap
// another tile, 1 on sides at the volume boundary.
__device__ __forceinline__ float ramp_w(int u, int o, int T, int n, int ramp)
{
    float w = 1.0f;
    if (o > 0) w = fminf(w, (u + 0.5f) / ramp);
    if (o + T < n) w = fminf(w, (T - u - 0.5f) / ramp);
    return w;
}

// blend: out[v][c] = sum_t w_t(v) y_t[v - o_t][c] / sum_t w_t(v) for c < creal,
// 0 for creal <= c < cout.  One thread per (voxel, channel); fixed tile order.
__global__ __launch_bounds__(256) void k_tile_blend(const float *__restrict__ y, int cy, int creal, int X, int Y, int Z,
                                                    const int *__restrict__ ox, int ntx, const int *__restrict__ oy,
                                                    int nty, const int *__restrict__ oz, int ntz, int T, int ramp,
                                                    int cout, float *__restrict__ out)
{
    const long long n = (long long)X * Y * Z * cout;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        const int c = (int)(e % cout);
        const long long v = e / cout;
        const int gz = (int)(v % Z), gy = (int)((v / Z) % Y), gx = (int)(v / ((long long)Y * Z));
        float num = 0.0f, den = 0.0f;
        if (c < creal) {
            for (int ix = 0; ix < ntx; ++ix) {
                const int ux = gx - ox[ix];
                if (ux < 0 || ux >= T) continue;
                const float wx = ramp_w(ux, ox[ix], T, X, ramp);
                for (int iy = 0; iy < nty; ++iy) {
                    const int uy = gy - oy[iy];
                    if (uy < 0 || uy >= T) continue;
                    const float wy = ramp_w(uy, oy[iy], T, Y, ramp);
                    for (int iz = 0; iz < ntz; ++iz) {
                        const int uz = gz - oz[iz];
                        if (uz < 0 || uz >= T) continue;
                        const float w = wx * wy * ramp_w(uz, oz[iz], T, Z, ramp);
                        const long long t = ((long long)ix * nty + iy) * ntz + iz;
                        num += w * y[((t * T + ux) * T + uy) * (long long)T * cy + (long long)uz * cy + c];
                        den += w;
                    }
                }
            }
        }
        out[e] = den > 0.0f ? num / den : 0.0f;
    }
}

int grid_for(long long n) { return (int)min((n + 255) / 256, 8192LL); }

template <int CI, int CO, int EPI>
hipError_t conv_t(const u16 *x, const void *wsw, const float *bias, const u16 *mask, void *y, int N, int X, int Y, int Z,
                  hipStream_t st)
{
    const int nb = N * ((X + TX - 1) / TX) * ((Y + TY - 1) / TY) * ((Z + TZ - 1) / TZ);
    hipLaunchKernelGGL((k_conv<CI, CO, EPI>), dim3(nb), dim3(256), 0, st, x, reinterpret_cast<const s8 *>(wsw), bias,
                       mask, y, X, Y, Z);
    return hipGetLastError();
}

template <int EPI>
hipError_t conv_dispatch(int ci, int co, const u16 *x, const void *wsw, const float *bias, const u16 *mask, void *y,
                         int N, int X, int Y, int Z, hipStream_t st)
{
    if (ci == 32 && co == 32) return conv_t<32, 32, EPI>(x, wsw, bias, mask, y, N, X, Y, Z, st);
    if (ci == 32 && co == 64) return conv_t<32, 64, EPI>(x, wsw, bias, mask, y, N, X, Y, Z, st);
    if (ci == 64 && co == 32) return conv_t<64, 32, EPI>(x, wsw, bias, mask, y, N, X, Y, Z, st);
    if (ci == 64 && co == 64) return conv_t<64, 64, EPI>(x, wsw, bias, mask, y, N, X, Y, Z, st);
    return hipErrorInvalidValue;
}

template <int CI, int CO>
hipError_t wgrad_t(const u16 *x, const u16 *gy, int N, int X, int Y, int Z, int nchunks, float *part, float *gw,
                   hipStream_t st)
{
    hipLaunchKernelGGL((k_wgrad<CI, CO>), dim3(27 * nchunks), dim3(256), 0, st, x, gy, N, X, Y, Z, nchunks, part);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((CI * CO + 255) / 256, 27), dim3(256), 0, st, part, nchunks, CI * CO, gw);
    return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers used by the C ABI
// ---------------------------------------------------------------------------
hipError_t net_conv(int epi, int ci, int co, const uint16_t *x, const void *wsw, const float *bias,
                    const uint16_t *mask, void *y, int N, int X, int Y, int Z, hipStream_t st)
{
    switch (epi) {
    case EPI_RELU_BF16: return conv_dispatch<EPI_RELU_BF16>(ci, co, x, wsw, bias, mask, y, N, X, Y, Z, st);
    case EPI_BIAS_F32: return conv_dispatch<EPI_BIAS_F32>(ci, co, x, wsw, bias, mask, y, N, X, Y, Z, st);
    case EPI_MASK_BF16: return conv_dispatch<EPI_MASK_BF16>(ci, co, x, wsw, bias, mask, y, N, X, Y, Z, st);
    default: return hipErrorInvalidValue;
    }
}

int net_wgrad_chunks(int N, int X, int Y, int Z)
{
    const long long ntiles = (long long)N * ((X + TX - 1) / TX) * ((Y + TY - 1) / TY) * ((Z + TZ - 1) / TZ);
    return (int)std::max(1LL, std::min(64LL, ntiles));
}

constexpr int kBiasBlocks = 512;

size_t net_wgrad_work_bytes(int ci, int co, int N, int X, int Y, int Z)
{
    return ((size_t)27 * net_wgrad_chunks(N, X, Y, Z) * ci * co + (size_t)kBiasBlocks * co) * sizeof(float);
}

hipError_t net_wgrad(int ci, int co, const uint16_t *x, const uint16_t *gy, int N, int X, int Y, int Z, float *work,
                     float *gw, float *gb, hipStream_t st)
{
    const int nch = net_wgrad_chunks(N, X, Y, Z);
    hipError_t e;
    if (ci == 32 && co == 32) e = wgrad_t<32, 32>(x, gy, N, X, Y, Z, nch, work, gw, st);
    else if (ci == 32 && co == 64) e = wgrad_t<32, 64>(x, gy, N, X, Y, Z, nch, work, gw, st);
    else if (ci == 64 && co == 32) e = wgrad_t<64, 32>(x, gy, N, X, Y, Z, nch, work, gw, st);
    else if (ci == 64 && co == 64) e = wgrad_t<64, 64>(x, gy, N, X, Y, Z, nch, work, gw, st);
    else return hipErrorInvalidValue;
    if (e != hipSuccess || !gb) return e;
    float *bp = work + (size_t)27 * nch * ci * co;
    hipLaunchKernelGGL(k_bias_partial, dim3(kBiasBlocks), dim3(256), 0, st, gy, (long long)N * X * Y * Z, co, bp);
    hipLaunchKernelGGL(k_bias_reduce, dim3(co), dim3(256), 0, st, bp, kBiasBlocks, co, gb);
    return hipGetLastError();
}

hipError_t net_swizzle(const float *w, int ci, int co, void *wf, void *wd, hipStream_t st)
{
    const int total = 27 * (ci / 32) * (co / 16) * 64;
    hipLaunchKernelGGL(k_swizzle, dim3((total + 255) / 256), dim3(256), 0, st, w, ci, co, reinterpret_cast<s8 *>(wf),
                       reinterpret_cast<s8 *>(wd));
    return hipGetLastError();
}

hipError_t net_adam(float *w, const float *g, float *m, float *v, long long n, int t, float lr, float b1, float b2,
                    float eps, hipStream_t st)
{
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, st, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t net_mse(const float *y, const float *t, long long nvox, int cpad, int creal, float scale, uint16_t *gy,
                   double *partials, int nblocks, double *loss, hipStream_t st)
{
    hipLaunchKernelGGL(k_mse, dim3(nblocks), dim3(256), 0, st, y, t, nvox, cpad, creal, scale, gy, partials);
    return launch_sum_partials(partials, nblocks, loss, 1.0, 0, st);
}

hipError_t net_tile_gather(const float *vol, int X, int Y, int Z, int cv, int cin, int cpad, const int *ox, int ntx,
                           const int *oy, int nty, const int *oz, int ntz, int T, float pre, const float *shift,
                           const float *scale, int t0, int nt, uint16_t *out, hipStream_t st)
{
    const long long n = (long long)T * T * T * cpad * nt;
    hipLaunchKernelGGL(k_tile_gather, dim3(grid_for(n)), dim3(256), 0, st, vol, X, Y, Z, cv, cin, cpad, ox, ntx, oy, nty,
                       oz, ntz, T, pre, shift, scale, t0, nt, out);
    return hipGetLastError();
}

hipError_t net_tile_blend(const float *y, int cy, int creal, int X, int Y, int Z, const int *ox, int ntx, const int *oy,
                          int nty, const int *oz, int ntz, int T, int ramp, int cout, float *out, hipStream_t st)
{
    const long long n = (long long)X * Y * Z * cout;
    hipLaunchKernelGGL(k_tile_blend, dim3(grid_for(n)), dim3(256), 0, st, y, cy, creal, X, Y, Z, ox, ntx, oy, nty, oz,
                       ntz, T, ramp, cout, out);
    return hipGetLastError();
}

hipError_t net_pack(const float *x, long long nvox, int cin, int cpad, float pre, const float *shift,
                    const float *scale, uint16_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack, dim3(grid_for(nvox * cpad)), dim3(256), 0, st, x, nvox, cin, cpad, pre, shift, scale,
                       out);
    return hipGetLastError();
}

}  // namespace tt
