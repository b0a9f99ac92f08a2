// Forward model and adjoint kernels for gfx950.
//
// Forward (Eq. forward_model, evaluated in the order the paper writes it):
//   1. map:    M_s[v][u] = sum_i B_{s,u,i} c_{v,i}       (MFMA, one pass over c
//              serves a batch of projections; u runs over the unique segments
//              only -- for even orders segments c and c + n_seg/2 coincide)
//   2. march:  I_{s,j,k,c} = step * sum_n sum_{8 corners} T(x_n - x_v) M_s[v][c mod U]
//              (one thread per ray, float64 sample positions, float32 sums)
// Adjoint (transpose, voxel-driven so no atomics are needed):
//   yf[s][j][k][u] = step * sum_{c mod U = u} y[s][j][k][c]
//   g_v = sum_s B_s^T Q_s(v),  Q_s(v)[u] = sum_{(j,k,n)} T(x_n - x_v) yf[s][j][k][u]
//   Each thread owns one voxel and enumerates the rays within the L1 radius of
//   its detector position and the samples of each ray inside its tent support;
//   each wave then contracts its 64 voxels' Q_s with B_s on MFMA, accumulating
//   g in registers over all projections.
#include "tt_device.h"
#include "tt_internal.h"

namespace tt {

typedef float f4 __attribute__((ext_vector_type(4)));

// MFMA 16x16x4 fp32 operand layout (one wave):
//   A[16][4]: lane l supplies A[l % 16][l / 16]
//   B[4][16]: lane l supplies B[l / 16][l % 16]
//   D[16][16]: lane l holds D[4 (l / 16) + r][l % 16], r = 0..3
__device__ __forceinline__ f4 mfma16x16x4(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

typedef short s4 __attribute__((ext_vector_type(4)));  // four bf16 bit patterns

// bf16 MFMA 16x16x16 (fp32 accumulate) operand layout (one wave):
//   A[16][16]: lane l supplies A[l % 16][4 (l / 16) + q], q = 0..3
//   B[16][16]: lane l supplies B[4 (l / 16) + q][l % 16]
//   D as for the fp32 16x16x4 instruction.
__device__ __forceinline__ f4 mfma16x16x16bf16(s4 a, s4 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// gfx950 bf16 MFMA 16x16x32: lane l supplies A[l % 16][8 (l / 16) + q] and
// B[8 (l / 16) + q][l % 16], q = 0..7; D as above.
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ f4 mfma16x16x32bf16(s8 a, s8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0,
                                                   0);
}

// float -> bf16 bit pattern, round to nearest even (finite inputs).
__device__ __forceinline__ short f2bf(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__device__ __forceinline__ long long pad_index(int v, int ny, int nz)
{
    int iz = v % nz;
    int t = v / nz;
    int iy = t % ny;
    int ix = t / ny;
    return ((long long)(ix + 1) * (ny + 2) + (iy + 1)) * (nz + 2) + (iz + 1);
}

// ---------------------------------------------------------------------------
// map (fp32 MFMA).  Block = 64 voxels x 256 rows (row = p * UP + u), four
// waves each owning 64 rows (4 row tiles) and all 4 voxel tiles, i.e. 16
// independent 16x16 accumulators.  The c tile is staged transposed in LDS;
// the B operands come from a copy of Bu pre-swizzled into MFMA lane order
// (Bsw[(row_tile * Cp/4 + ks) * 64 + lane] = Bu[16 row_tile + lane % 16][4 ks + lane / 16]),
// so every operand load is one coalesced 256-byte read.
// ---------------------------------------------------------------------------
constexpr int kCtStride = 80;  // padded voxel stride of the transposed c tile in LDS

template <int UP>
__global__ __launch_bounds__(256) void k_map_fp32(const float *__restrict__ c, const float *__restrict__ Bsw,
                                                  int V, int C, int Cp, int ny, int nz, int s0, int np,
                                                  long long vol_pad, float *__restrict__ M)
{
    extern __shared__ float cT[];  // [Cp][kCtStride]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int v0 = blockIdx.x * 64;
    const int nv = min(64, V - v0);
    const float *cb = c + (long long)v0 * C;
    for (int e = tid; e < 64 * Cp; e += 256) cT[(e >> 6) * kCtStride + (e & 63)] = 0.0f;
    __syncthreads();
    const float invC = 1.0f / (float)C;
    for (int e = tid; e < nv * C; e += 256) {
        int v = (int)(((float)e + 0.5f) * invC);
        int k = e - v * C;
        cT[k * kCtStride + v] = cb[e];
    }
    __syncthreads();

    const int KS = Cp / 4;
    const int rt0 = (s0 * UP) / 16 + blockIdx.y * 16 + wave * 4;  // first row tile of this wave
    const int kq = lane >> 4;
    f4 acc[4][4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc[nt][mt] = f4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < KS / 4; ++kc) {
        float a[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) a[mt][kk] = Bsw[((long long)(rt0 + mt) * KS + kc * 4 + kk) * 64 + lane];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const float b = cT[(kc * 16 + kk * 4 + kq) * kCtStride + nt * 16 + (lane & 15)];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) acc[nt][mt] = mfma16x16x4(a[mt][kk], b, acc[nt][mt]);
            }
        }
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int v = v0 + nt * 16 + (lane & 15);
        if (v >= V) continue;
        const long long vp = pad_index(v, ny, nz);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const int row = blockIdx.y * 256 + wave * 64 + mt * 16 + 4 * kq;  // within the batch
            const int p = row / UP, u0 = row % UP;
            if (p < np) *reinterpret_cast<f4 *>(M + (long long)p * vol_pad * UP + vp * UP + u0) = acc[nt][mt];
        }
    }
}

// Register-resident variant for Cp <= 64 (ell_max <= 12): each wave keeps
// its B operands for every k-step in registers, and the block walks a range
// of consecutive voxel tiles, prefetching the next tile's coefficients
// into registers while the current tile's MFMAs run, so coefficient loads,
// MFMAs and the M stores of consecutive tiles overlap.  A block of NW waves
// covers the same 256 rows, each wave 16 / NW row tiles: eight waves of two
// row tiles (120 registers, four waves per SIMD) measured 2-3% faster than
// four waves of four (216 registers, two waves per SIMD).
constexpr int kCtStrideRb = 81;  // odd: the transposed tile writes hit distinct banks
constexpr int kMapWaves = 8;

template <int UP, int KS, int NW>
__global__ __launch_bounds__(64 * NW) void k_map_fp32_rb(const float *__restrict__ c, const float *__restrict__ Bsw,
                                                          int V, int C, int ny, int nz, int s0, int np,
                                                          long long vol_pad, float *__restrict__ M)
{
    constexpr int Cp = 4 * KS;
    constexpr int NT = 64 * NW;                 // threads of the block
    constexpr int MW = 16 / NW;                 // row tiles per wave (256 rows per block)
    constexpr int NPF = (16 * Cp + NT - 1) / NT;  // float4 per thread covering a 64 x C tile (C <= Cp)
    __shared__ float cT[Cp * kCtStrideRb];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kq = lane >> 4;
    const int rt0 = (s0 * UP) / 16 + blockIdx.y * 16 + wave * MW;
    float a[MW][KS];
#pragma unroll
    for (int mt = 0; mt < MW; ++mt)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) a[mt][ks] = Bsw[((long long)(rt0 + mt) * KS + ks) * 64 + lane];
    // padding coefficients C..Cp-1 stay zero for every tile
    for (int e = tid; e < (Cp - C) * 64; e += NT) cT[(C + e / 64) * kCtStrideRb + (e & 63)] = 0.0f;
    const int ntiles = (V + 63) / 64;
    const int n4 = 16 * C;  // float4 in a full tile
    const float invC = 1.0f / (float)C;
    f4 pf[NPF];
    auto prefetch = [&](int t) {
        const int nvals = min(64, V - t * 64) * C;
        const f4 *src = reinterpret_cast<const f4 *>(c + (long long)t * 64 * C);  // 256 C bytes per tile: aligned
        const float *srcf = c + (long long)t * 64 * C;
#pragma unroll
        for (int i = 0; i < NPF; ++i) {
            const int e4 = tid + NT * i;
            pf[i] = f4{0.f, 0.f, 0.f, 0.f};
            if (4 * e4 + 3 < nvals) {
                pf[i] = src[e4];
            } else if (4 * e4 < nvals) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (4 * e4 + q < nvals) pf[i][q] = srcf[4 * e4 + q];
            }
        }
    };
    // each block walks a contiguous range of tiles, so that its stores into
    // every projection's M are one sequential stream (scattered 1 KiB pieces
    // stall on DRAM write credits)
    const int per = (ntiles + (int)gridDim.x - 1) / (int)gridDim.x;
    const int tend = min(ntiles, (int)blockIdx.x * per + per);
    int tile = blockIdx.x * per;
    if (tile < tend) prefetch(tile);
    for (; tile < tend; ++tile) {
        __syncthreads();  // the previous tile's LDS reads are done
#pragma unroll
        for (int i = 0; i < NPF; ++i) {
            const int e4 = tid + NT * i;
            if (e4 < n4) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = 4 * e4 + q;
                    const int v = (int)(((float)e + 0.5f) * invC);
                    cT[(e - v * C) * kCtStrideRb + v] = pf[i][q];
                }
            }
        }
        __syncthreads();
        if (tile + 1 < tend) prefetch(tile + 1);  // in flight during the MFMAs
        f4 acc[4][MW];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int mt = 0; mt < MW; ++mt) acc[nt][mt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const float b = cT[(ks * 4 + kq) * kCtStrideRb + nt * 16 + (lane & 15)];
#pragma unroll
                for (int mt = 0; mt < MW; ++mt) acc[nt][mt] = mfma16x16x4(a[mt][ks], b, acc[nt][mt]);
            }
        }
        const int v0 = tile * 64;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int v = v0 + nt * 16 + (lane & 15);
            if (v >= V) continue;
            const long long vp = pad_index(v, ny, nz);
#pragma unroll
            for (int mt = 0; mt < MW; ++mt) {
                const int row = blockIdx.y * 256 + wave * 16 * MW + mt * 16 + 4 * kq;  // within the batch
                const int p = row / UP, u0 = row % UP;
                if (p < np) *reinterpret_cast<f4 *>(M + (long long)p * vol_pad * UP + vp * UP + u0) = acc[nt][mt];
            }
        }
    }
}

template <int UP, int KS>
static hipError_t map_fp32_rb_t(const Dims &d, const float *c, const float *Bsw, int s0, int np, float *M,
                                hipStream_t st)
{
    const int V = d.nx * d.ny * d.nz;
    const long long vol_pad = (long long)(d.nx + 2) * (d.ny + 2) * (d.nz + 2);
    const int gy = (np * UP + 255) / 256, ntiles = (V + 63) / 64;
    // one resident round of blocks over all row groups (measured 3% faster
    // than four rounds: fewer concurrent M store streams)
    static const int resident = [] {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_map_fp32_rb<UP, KS, kMapWaves>, 64 * kMapWaves,
                                                         0) != hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 512;
        return std::max(1, per_cu * cus);
    }();
    const int gx = std::max(1, std::min(ntiles, resident / gy));
    hipLaunchKernelGGL((k_map_fp32_rb<UP, KS, kMapWaves>), dim3(gx, gy), dim3(64 * kMapWaves), 0, st, c, Bsw, V, d.C,
                       d.ny, d.nz, s0, np, vol_pad, M);
    return hipGetLastError();
}

template <int UP>
static hipError_t map_fp32_t(const Dims &d, const float *c, const float *Bsw, int s0, int np, float *M,
                             hipStream_t st)
{
    const bool aligned = reinterpret_cast<uintptr_t>(c) % 16 == 0;  // float4 tile loads
    switch (aligned ? d.Cp : 0) {
    case 16: return map_fp32_rb_t<UP, 4>(d, c, Bsw, s0, np, M, st);
    case 32: return map_fp32_rb_t<UP, 8>(d, c, Bsw, s0, np, M, st);
    case 48: return map_fp32_rb_t<UP, 12>(d, c, Bsw, s0, np, M, st);
    case 64: return map_fp32_rb_t<UP, 16>(d, c, Bsw, s0, np, M, st);
    default: break;  // larger orders: B operands streamed from memory
    }
    const int V = d.nx * d.ny * d.nz;
    const long long vol_pad = (long long)(d.nx + 2) * (d.ny + 2) * (d.nz + 2);
    dim3 grid((V + 63) / 64, (np * UP + 255) / 256);
    size_t lds = (size_t)d.Cp * kCtStride * sizeof(float);
    hipLaunchKernelGGL(k_map_fp32<UP>, grid, dim3(256), lds, st, c, Bsw, V, d.C, d.Cp, d.ny, d.nz, s0, np,
                       vol_pad, M);
    return hipGetLastError();
}

hipError_t launch_map_fp32(const Dims &d, const float *c, const float *Bsw, int s0, int np, float *M,
                           hipStream_t st)
{
    if ((s0 * d.Up) % 16) return hipErrorInvalidValue;  // batches start on a row tile
    switch (d.Up) {
    case 4: return map_fp32_t<4>(d, c, Bsw, s0, np, M, st);
    case 8: return map_fp32_t<8>(d, c, Bsw, s0, np, M, st);
    case 16: return map_fp32_t<16>(d, c, Bsw, s0, np, M, st);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// map, bf16 tier: c is rounded to bf16 while it is staged in LDS, B comes as
// bf16 in MFMA lane order, products accumulate in fp32.  K = Cp runs in
// 32-coefficient steps on the 16x16x32 instruction and, when Cp / 16 is odd,
// a last 16-coefficient step on the 16x16x16 one.  Row tile rt of Bsw16
// (16 Cp shorts at rt * 16 Cp) holds for step kp < Cp / 32 and lane l the
// eight values Bu[16 rt + l % 16][32 kp + 8 (l / 16) + q] at (kp * 64 + l) * 8,
// then for the odd step the four values Bu[16 rt + l % 16][32 (Cp / 32) +
// 4 (l / 16) + q] at (Cp / 32) * 512 + l * 4.  Same tiling as the fp32 kernel.
// ---------------------------------------------------------------------------
template <int UP>
__global__ __launch_bounds__(256) void k_map_bf16(const float *__restrict__ c, const short *__restrict__ Bsw16,
                                                  int V, int C, int Cp, int ny, int nz, int s0, int np,
                                                  long long vol_pad, float *__restrict__ M)
{
    extern __shared__ short cb[];  // [64][Cp + 8] bf16, row = voxel (16-byte rows)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ld = Cp + 8;
    const int v0 = blockIdx.x * 64;
    const int nv = min(64, V - v0);
    const float *cg = c + (long long)v0 * C;
    for (int e = tid; e < 64 * ld; e += 256) cb[e] = 0;
    __syncthreads();
    const float invC = 1.0f / (float)C;
    for (int e = tid; e < nv * C; e += 256) {
        int v = (int)(((float)e + 0.5f) * invC);
        int k = e - v * C;
        cb[v * ld + k] = f2bf(cg[e]);
    }
    __syncthreads();

    const int KP = Cp / 32;
    const int rt0 = (s0 * UP) / 16 + blockIdx.y * 16 + wave * 4;
    const int kq = lane >> 4;
    f4 acc[4][4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc[nt][mt] = f4{0.f, 0.f, 0.f, 0.f};
    for (int kp = 0; kp < KP; ++kp) {
        s8 a[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            a[mt] = *reinterpret_cast<const s8 *>(Bsw16 + (long long)(rt0 + mt) * 16 * Cp + (kp * 64 + lane) * 8);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const s8 b = *reinterpret_cast<const s8 *>(cb + (nt * 16 + (lane & 15)) * ld + kp * 32 + 8 * kq);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) acc[nt][mt] = mfma16x16x32bf16(a[mt], b, acc[nt][mt]);
        }
    }
    if (Cp & 16) {
        s4 a[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            a[mt] = *reinterpret_cast<const s4 *>(Bsw16 + (long long)(rt0 + mt) * 16 * Cp + KP * 512 + lane * 4);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const s4 b = *reinterpret_cast<const s4 *>(cb + (nt * 16 + (lane & 15)) * ld + KP * 32 + 4 * kq);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) acc[nt][mt] = mfma16x16x16bf16(a[mt], b, acc[nt][mt]);
        }
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int v = v0 + nt * 16 + (lane & 15);
        if (v >= V) continue;
        const long long vp = pad_index(v, ny, nz);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const int row = blockIdx.y * 256 + wave * 64 + mt * 16 + 4 * kq;
            const int p = row / UP, u0 = row % UP;
            if (p < np) *reinterpret_cast<f4 *>(M + (long long)p * vol_pad * UP + vp * UP + u0) = acc[nt][mt];
        }
    }
}

// Register-resident bf16 variant for Cp <= 64, organised as k_map_fp32_rb: a
// block of kMapWaves waves covers 256 rows, each wave 16 / NW row tiles with
// its A operands for every k-step in registers; the block walks a contiguous
// range of 64-voxel tiles (sequential M store streams), prefetching the next
// tile's coefficients into registers during the MFMAs, and rounds them to
// bf16 while staging them in LDS.  Same rounding points and MFMA order as
// k_map_bf16, hence the same results.
template <int UP, int CPT, int NW>
__global__ __launch_bounds__(64 * NW) void k_map_bf16_rb(const float *__restrict__ c, const short *__restrict__ Bsw16,
                                                         int V, int C, int ny, int nz, int s0, int np,
                                                         long long vol_pad, float *__restrict__ M)
{
    constexpr int Cp = 16 * CPT, KP = CPT / 2, ODD = CPT & 1;
    constexpr int ld = Cp + 8;                  // LDS row of one voxel, in shorts (16-byte multiple)
    constexpr int NT = 64 * NW;                 // threads of the block
    constexpr int MW = 16 / NW;                 // row tiles per wave (256 rows per block)
    constexpr int NPF = (16 * Cp + NT - 1) / NT;  // float4 per thread covering a 64 x C tile (C <= Cp)
    __shared__ short cb[64 * ld];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kq = lane >> 4;
    const int rt0 = (s0 * UP) / 16 + blockIdx.y * 16 + wave * MW;
    s8 a8[MW][KP > 0 ? KP : 1];
    s4 a4[MW];
#pragma unroll
    for (int mt = 0; mt < MW; ++mt) {
        const short *rt = Bsw16 + (long long)(rt0 + mt) * 16 * Cp;
#pragma unroll
        for (int kp = 0; kp < KP; ++kp) a8[mt][kp] = *reinterpret_cast<const s8 *>(rt + (kp * 64 + lane) * 8);
        if constexpr (ODD) a4[mt] = *reinterpret_cast<const s4 *>(rt + KP * 512 + lane * 4);
    }
    // coefficients C..ld-1 of every voxel row stay zero for every tile
    for (int e = tid; e < 64 * (ld - C); e += NT) cb[(e / (ld - C)) * ld + C + e % (ld - C)] = 0;
    const int ntiles = (V + 63) / 64;
    const int n4 = 16 * C;  // float4 in a full tile
    const float invC = 1.0f / (float)C;
    f4 pf[NPF];
    auto prefetch = [&](int t) {
        const int nvals = min(64, V - t * 64) * C;
        const f4 *src = reinterpret_cast<const f4 *>(c + (long long)t * 64 * C);  // 256 C bytes per tile: aligned
        const float *srcf = c + (long long)t * 64 * C;
#pragma unroll
        for (int i = 0; i < NPF; ++i) {
            const int e4 = tid + NT * i;
            pf[i] = f4{0.f, 0.f, 0.f, 0.f};
            if (4 * e4 + 3 < nvals) {
                pf[i] = src[e4];
            } else if (4 * e4 < nvals) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (4 * e4 + q < nvals) pf[i][q] = srcf[4 * e4 + q];
            }
        }
    };
    const int per = (ntiles + (int)gridDim.x - 1) / (int)gridDim.x;
    const int tend = min(ntiles, (int)blockIdx.x * per + per);
    int tile = blockIdx.x * per;
    if (tile < tend) prefetch(tile);
    for (; tile < tend; ++tile) {
        __syncthreads();  // the previous tile's LDS reads are done
#pragma unroll
        for (int i = 0; i < NPF; ++i) {
            const int e4 = tid + NT * i;
            if (e4 < n4) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = 4 * e4 + q;
                    const int v = (int)(((float)e + 0.5f) * invC);
                    cb[v * ld + (e - v * C)] = f2bf(pf[i][q]);
                }
            }
        }
        __syncthreads();
        if (tile + 1 < tend) prefetch(tile + 1);  // in flight during the MFMAs
        f4 acc[4][MW];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int mt = 0; mt < MW; ++mt) acc[nt][mt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kp = 0; kp < KP; ++kp) {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const s8 b = *reinterpret_cast<const s8 *>(cb + (nt * 16 + (lane & 15)) * ld + kp * 32 + 8 * kq);
#pragma unroll
                for (int mt = 0; mt < MW; ++mt) acc[nt][mt] = mfma16x16x32bf16(a8[mt][kp], b, acc[nt][mt]);
            }
        }
        if constexpr (ODD) {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const s4 b = *reinterpret_cast<const s4 *>(cb + (nt * 16 + (lane & 15)) * ld + KP * 32 + 4 * kq);
#pragma unroll
                for (int mt = 0; mt < MW; ++mt) acc[nt][mt] = mfma16x16x16bf16(a4[mt], b, acc[nt][mt]);
            }
        }
        const int v0 = tile * 64;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int v = v0 + nt * 16 + (lane & 15);
            if (v >= V) continue;
            const long long vp = pad_index(v, ny, nz);
#pragma unroll
            for (int mt = 0; mt < MW; ++mt) {
                const int row = blockIdx.y * 256 + wave * 16 * MW + mt * 16 + 4 * kq;  // within the batch
                const int p = row / UP, u0 = row % UP;
                if (p < np) *reinterpret_cast<f4 *>(M + (long long)p * vol_pad * UP + vp * UP + u0) = acc[nt][mt];
            }
        }
    }
}

template <int UP, int CPT>
static hipError_t map_bf16_rb_t(const Dims &d, const float *c, const uint16_t *Bsw16, int s0, int np, float *M,
                                hipStream_t st)
{
    const int V = d.nx * d.ny * d.nz;
    const long long vol_pad = (long long)(d.nx + 2) * (d.ny + 2) * (d.nz + 2);
    const int gy = (np * UP + 255) / 256, ntiles = (V + 63) / 64;
    static const int resident = [] {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_map_bf16_rb<UP, CPT, kMapWaves>, 64 * kMapWaves,
                                                         0) != hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 512;
        return std::max(1, per_cu * cus);
    }();
    const int gx = std::max(1, std::min(ntiles, resident / gy));
    hipLaunchKernelGGL((k_map_bf16_rb<UP, CPT, kMapWaves>), dim3(gx, gy), dim3(64 * kMapWaves), 0, st, c,
                       reinterpret_cast<const short *>(Bsw16), V, d.C, d.ny, d.nz, s0, np, vol_pad, M);
    return hipGetLastError();
}

template <int UP>
static hipError_t map_bf16_t(const Dims &d, const float *c, const uint16_t *Bsw16, int s0, int np, float *M,
                             hipStream_t st)
{
    const bool aligned = reinterpret_cast<uintptr_t>(c) % 16 == 0;  // float4 tile loads
    switch (aligned ? d.Cp : 0) {
    case 16: return map_bf16_rb_t<UP, 1>(d, c, Bsw16, s0, np, M, st);
    case 32: return map_bf16_rb_t<UP, 2>(d, c, Bsw16, s0, np, M, st);
    case 48: return map_bf16_rb_t<UP, 3>(d, c, Bsw16, s0, np, M, st);
    case 64: return map_bf16_rb_t<UP, 4>(d, c, Bsw16, s0, np, M, st);
    default: break;  // larger orders: one tile per block, A operands loaded per step
    }
    const int V = d.nx * d.ny * d.nz;
    const long long vol_pad = (long long)(d.nx + 2) * (d.ny + 2) * (d.nz + 2);
    dim3 grid((V + 63) / 64, (np * UP + 255) / 256);
    size_t lds = (size_t)64 * (d.Cp + 8) * sizeof(short);
    hipLaunchKernelGGL(k_map_bf16<UP>, grid, dim3(256), lds, st, c, reinterpret_cast<const short *>(Bsw16), V, d.C,
                       d.Cp, d.ny, d.nz, s0, np, vol_pad, M);
    return hipGetLastError();
}

hipError_t launch_map_bf16(const Dims &d, const float *c, const uint16_t *Bsw16, int s0, int np, float *M,
                           hipStream_t st)
{
    if ((s0 * d.Up) % 16) return hipErrorInvalidValue;
    switch (d.Up) {
    case 4: return map_bf16_t<4>(d, c, Bsw16, s0, np, M, st);
    case 8: return map_bf16_t<8>(d, c, Bsw16, s0, np, M, st);
    case 16: return map_bf16_t<16>(d, c, Bsw16, s0, np, M, st);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// march: one thread per ray; block = 16 (j) x 16 (k) rays of one projection.
// Ray positions are set up in float64 in padded index coordinates (voxel ix
// sits at ix + 1, borders of M are zero), so no bounds test is needed inside
// the loop.  The staged path computes each slab's sample count and first
// position in float64 and steps its samples in float32 relative to the
// staged box; the global path steps in float64.
//
// The tile's rays are marched slab by slab: a slab is W planes of the
// horizontal axis A most aligned with the rays.  Before each slab the block
// stages the box of M that holds every corner its samples touch into LDS
// (rows along z, coalesced), then each thread walks its own samples in that
// slab and gathers the 8 corners from LDS.  The box size comes from the
// per-projection slab plan; projections without a plan (steep rays) gather
// straight from global memory.
// ---------------------------------------------------------------------------

// Ray setup shared by both paths: index-space base point b and step ds of the
// ray through pixel (j, k), and its sample range [n0, n1] (empty if n0 > n1).
// Joseph's method (jos): the samples are the ray's cuts with the voxel-centre
// planes of its dominant axis A, so the base point is moved to the cut with
// plane A = 0 and the spacing is d / |d_A|: sample n lies on plane
// n sign(d_A), and the same box constraints keep the planes 1..n_A and the
// cuts whose in-plane coordinates stay inside (0, n + 1).
__device__ __forceinline__ void ray_setup(const ProjFrame &f, int j, int k, int nx, int ny, int nz, float step,
                                          double b[3], double ds[3], int &n0, int &n1, bool jos = false)
{
    const double n3[3] = {(double)nx, (double)ny, (double)nz};
    double tlo = -1e300, thi = 1e300;
    double scale = (double)step;
#pragma unroll
    for (int a = 0; a < 3; ++a) b[a] = f.o[a] + j * f.ej[a] + k * f.ek[a] + 0.5 * (n3[a] + 1.0);
    if (jos) {
        const int A = f.jos_a;
        const double t0 = -b[A] * f.inv_d[A];
#pragma unroll
        for (int a = 0; a < 3; ++a) b[a] = a == A ? 0.0 : fma(t0, f.d[a], b[a]);
        scale = fabs(f.inv_d[A]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        ds[a] = (jos && a == f.jos_a) ? (f.d[a] > 0.0 ? 1.0 : -1.0) : scale * f.d[a];
        if (f.inv_d[a] != 0.0) {
            // index coordinate b + n ds must stay inside (0, n + 1)
            double ia = (jos && a == f.jos_a) ? ds[a] : f.inv_d[a] / scale;
            double t1 = -b[a] * ia, t2 = (n3[a] + 1.0 - b[a]) * ia;
            tlo = fmax(tlo, fmin(t1, t2));
            thi = fmin(thi, fmax(t1, t2));
        } else if (!(b[a] > 0.0 && b[a] < n3[a] + 1.0)) {
            thi = -1e300;
        }
    }
    n0 = 0;
    n1 = -1;
    if (tlo < thi) {
        n0 = (int)ceil(tlo);
        n1 = (int)floor(thi);
    }
}

template <int UP>
__device__ __forceinline__ void march_global(const float *__restrict__ Mp, const double b[3], const double ds[3], int n0,
                                             int n1, int nx, int ny, int nz, float acc[UP])
{
    const long long sz = UP, sy = (long long)(nz + 2) * UP, sx = (long long)(ny + 2) * sy;
    for (int n = n0; n <= n1; ++n) {
        double px = fma((double)n, ds[0], b[0]);
        double py = fma((double)n, ds[1], b[1]);
        double pz = fma((double)n, ds[2], b[2]);
        int ix = min(max((int)floor(px), 0), nx);
        int iy = min(max((int)floor(py), 0), ny);
        int iz = min(max((int)floor(pz), 0), nz);
        float fx = (float)(px - ix), fy = (float)(py - iy), fz = (float)(pz - iz);
        float gx = 1.0f - fx, gy = 1.0f - fy, gz = 1.0f - fz;
        float w00 = gx * gy, w01 = gx * fy, w10 = fx * gy, w11 = fx * fy;
        const float *q = Mp + ix * sx + iy * sy + iz * sz;
        float w[8] = {w00 * gz, w00 * fz, w01 * gz, w01 * fz, w10 * gz, w10 * fz, w11 * gz, w11 * fz};
        const long long off[8] = {0, sz, sy, sy + sz, sx, sx + sz, sx + sy, sx + sy + sz};
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
#pragma unroll
            for (int u4 = 0; u4 < UP; u4 += 4) {
                f4 m = *reinterpret_cast<const f4 *>(q + off[cc] + u4);
                acc[u4 + 0] = fmaf(w[cc], m.x, acc[u4 + 0]);
                acc[u4 + 1] = fmaf(w[cc], m.y, acc[u4 + 1]);
                acc[u4 + 2] = fmaf(w[cc], m.z, acc[u4 + 2]);
                acc[u4 + 3] = fmaf(w[cc], m.w, acc[u4 + 3]);
            }
        }
    }
}

// Global-memory march of the fused sparse forward: at every sample the 8
// corner voxels' coefficients are mapped to the unique segments with the
// projection's sparse map (tab[u * kk + t] = (basis index, constant)).
template <int UP>
__device__ __forceinline__ void march_global_fused(const float *__restrict__ cv, const int2 *tab, int kk, int C,
                                                   const double b[3], const double ds[3], int n0, int n1, int nx,
                                                   int ny, int nz, int U, float acc[UP])
{
    for (int n = n0; n <= n1; ++n) {
        const double px = fma((double)n, ds[0], b[0]);
        const double py = fma((double)n, ds[1], b[1]);
        const double pz = fma((double)n, ds[2], b[2]);
        // padded cell [i, i + 1] holds voxels i - 1 and i along each axis
        const int ix = min(max((int)floor(px), 0), nx);
        const int iy = min(max((int)floor(py), 0), ny);
        const int iz = min(max((int)floor(pz), 0), nz);
        const float fx = (float)(px - ix), fy = (float)(py - iy), fz = (float)(pz - iz);
        const float gx = 1.0f - fx, gy = 1.0f - fy, gz = 1.0f - fz;
        for (int cc = 0; cc < 8; ++cc) {
            const int x = ix - 1 + (cc >> 2), y = iy - 1 + ((cc >> 1) & 1), z = iz - 1 + (cc & 1);
            if ((unsigned)x >= (unsigned)nx || (unsigned)y >= (unsigned)ny || (unsigned)z >= (unsigned)nz) continue;
            const float wc = ((cc & 4) ? fx : gx) * ((cc & 2) ? fy : gy) * ((cc & 1) ? fz : gz);
            const float *src = cv + ((long long)(x * ny + y) * nz + z) * C;
#pragma unroll
            for (int u = 0; u < UP; ++u) {
                if (u < U) {
                    float v = 0.0f;
                    for (int t = 0; t < kk; ++t) {
                        const int2 e = tab[u * kk + t];
                        v = fmaf(__int_as_float(e.y), src[e.x], v);
                    }
                    acc[u] = fmaf(wc, v, acc[u]);
                }
            }
        }
    }
}

// With 4 unique segments (32 KiB boxes) five blocks fit a CU's LDS; asking
// for five waves per SIMD (a small spill of setup values) measured 4% faster
// than the four that 116 VGPRs allow.  Larger UP keep their registers: their
// spills were much larger and slower.
//
// FUSED: the sparse variant of the forward (sect. "Pipelines": the
// reciprocal-space map applied inside the ray-sum kernel, so no mapped volume
// is stored).  M is then the coefficient volume c[nx][ny][nz][C] itself, the
// grid covers all projections (s0 = 0), and each staged box voxel's unique
// segment values are formed while staging, m_u = sum_t tab[u][t].w *
// c[v][tab[u][t].i] over the kk kept basis functions of (s, u); one thread
// stages one (voxel, segment) pair.  The gather from the box is the same.
template <int UP, bool FUSED, int NCM = 8>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((UP == 4 && !FUSED) ? 5 : 1))) void k_march(const float *__restrict__ M, const ProjFrame *__restrict__ frames,
                                               int s0, int nx, int ny, int nz, int nj, int nk, int nseg, int U,
                                               float step, long long vol_pad, float *__restrict__ I,
                                               const int2 *__restrict__ sp, int kk, int C,
                                               const float *__restrict__ cT, const int *__restrict__ gtab, int ng,
                                               int jos)
{
    constexpr int Q = UP / 4;      // float4 per staged voxel
    // FUSED: the map table int2[UP][kk] (global-memory gathers), the channel
    // list int[ng] and its constants float[ng][UP] (staging), then the box
    extern __shared__ f4 lds[];
    __shared__ int arange[2];
    const int tab_f4 = FUSED ? (UP * kk * 8 + 15) / 16 + (ng * (UP + 1) * 4 + 15) / 16 : 0;
    f4 *box = lds + tab_f4;        // [Q][W + 1][eb][ez]
    const int ntj = (nj + kMarchTile - 1) / kMarchTile, ntk = (nk + kMarchTile - 1) / kMarchTile;
    const int lb = blockIdx.x;
    const int p = lb / (ntj * ntk), s = s0 + p;
    const int tj = (lb / ntk) % ntj, tk = lb % ntk;
    const int j = tj * kMarchTile + (threadIdx.x % kMarchTile);
    const int k = tk * kMarchTile + (threadIdx.x / kMarchTile);
    const bool live = j < nj && k < nk;
    const ProjFrame &f = frames[s];
    const float *Mp = FUSED ? M : M + (long long)p * vol_pad * UP;
    int2 *tab = reinterpret_cast<int2 *>(lds);
    int *gch = reinterpret_cast<int *>(lds + (UP * kk * 8 + 15) / 16);  // [ng] channels, then [ng][UP] constants
    const float *gw = reinterpret_cast<const float *>(gch + ng);
    if constexpr (FUSED) {
        const int2 *src = sp + (long long)s * UP * kk;
        for (int i = threadIdx.x; i < UP * kk; i += 256) tab[i] = src[i];
        const int *gsrc = gtab + (long long)s * ng * (UP + 1);
        for (int i = threadIdx.x; i < ng * (UP + 1); i += 256) gch[i] = gsrc[i];
        __syncthreads();
    }
    double b[3], ds[3];
    int n0 = 0, n1 = -1;
    if (live) ray_setup(f, j, k, nx, ny, nz, step, b, ds, n0, n1, jos != 0);
    float acc[UP];
#pragma unroll
    for (int u = 0; u < UP; ++u) acc[u] = 0.0f;

    const int W = f.slab_w;
    if (W == 0) {
        if (n0 <= n1) {
            if constexpr (FUSED)
                march_global_fused<UP>(M, tab, kk, C, b, ds, n0, n1, nx, ny, nz, U, acc);
            else
                march_global<UP>(Mp, b, ds, n0, n1, nx, ny, nz, acc);
        }
    } else {
        const int A = f.slab_a, B = 1 - A, EB = f.slab_eb, EZ = f.slab_ez;
        // samples are visited in increasing index coordinate along A
        const bool fwd = f.d[A] > 0.0;
        const int count = n1 - n0 + 1;
        if (threadIdx.x == 0) {
            arange[0] = INT_MAX;
            arange[1] = INT_MIN;
        }
        __syncthreads();
        if (count > 0) {
            const int nf = fwd ? n0 : n1, nl = fwd ? n1 : n0;
            atomicMin(&arange[0], (int)floor(fma((double)nf, ds[A], b[A])));
            atomicMax(&arange[1], (int)floor(fma((double)nl, ds[A], b[A])));
        }
        __syncthreads();
        const int amin = arange[0], amax = arange[1];
        // Staged box origin of slab A0: the lowest corner, along B and z, of the
        // tile's rays between planes A0 and A0 + W.  Each vertex coordinate is
        // affine in A0 with the common slope d_B / d_A (resp. d_z / d_A), so the
        // minimum over the 8 vertices is kb + A0 rB (resp. kz + A0 rZ).
        const double n3[3] = {(double)nx, (double)ny, (double)nz};
        double b00[3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            b00[a] = f.o[a] + (tj * kMarchTile) * f.ej[a] + (tk * kMarchTile) * f.ek[a] + 0.5 * (n3[a] + 1.0);
        const double rB = f.d[B] * f.inv_d[A], rZ = f.d[2] * f.inv_d[A];
        const double T = kMarchTile - 1;
        double kb = 1e300, kz = 1e300;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const double J = (v & 1) ? T : 0.0, K = (v & 2) ? T : 0.0, P = (v & 4) ? (double)W : 0.0;
            const double t = P - (b00[A] + J * f.ej[A] + K * f.ek[A]);
            kb = fmin(kb, b00[B] + J * f.ej[B] + K * f.ek[B] + t * rB);
            kz = fmin(kz, b00[2] + J * f.ej[2] + K * f.ek[2] + t * rZ);
        }
        const int plane = EB * EZ, nbox = (W + 1) * plane;
        const int nbs = (nbox + 63) & ~63;  // LDS stride of one float4 component array of the box
        // M strides (in voxels) of the box axes A and B; z is contiguous
        const int sy = nz + 2, sx = (ny + 2) * sy;
        const int sA = A == 0 ? sx : sy, sB = A == 0 ? sy : sx;
        const unsigned nAp = (A == 0 ? nx : ny) + 1, nBp = (A == 0 ? ny : nx) + 1, nZp = nz + 1;
        // LDS layout box[q][e]: the q-th float4 of all staged voxels, then the next
        const int da = plane, db = EZ, dz = 1;
        // Staging walk: thread t stages box elements e = t + 256 i.  Its first
        // element's (plane, row, z) and the step of 256 elements are decoded
        // once; every later element follows by adds and two carries, and its M
        // offset from the slab origin (in voxels, 32-bit) likewise.
        const int e_pl = threadIdx.x / plane, e_r = threadIdx.x - e_pl * plane;
        const int e_ib = e_r / EZ, e_iz = e_r - e_ib * EZ;
        const int s_pl = 256 / plane, s_r = 256 - s_pl * plane;
        const int s_ib = s_r / EZ, s_iz = s_r - s_ib * EZ;
        const int s_off = s_pl * sA + s_ib * sB + s_iz;  // M offset of one step without carries
        const int cz_off = sB - EZ, cb_off = sA - EB * sB;  // extra M offset of a z / row carry
        // Samples in sample order m have index position q0 + m dq with dq_A > 0.
        const int nstart = fwd ? n0 : n1;
        double q0[3], dq[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            q0[a] = fma((double)nstart, ds[a], b[a]);
            dq[a] = fwd ? ds[a] : -ds[a];
        }
        const double inv_dqA = 1.0 / dq[A];  // |d_A| >= 1/4 for a planned projection
        const float dqA = (float)dq[A], dqB = (float)dq[B], dqZ = (float)dq[2];
        const float wmax = (float)(W - 1), bmax = (float)(EB - 2), zmax = (float)(EZ - 2);
        int m = 0;
        for (int A0 = amin; A0 <= amax; A0 += W) {
            const int B0 = (int)floor(fma((double)A0, rB, kb)) - 1, Z0 = (int)floor(fma((double)A0, rZ, kz)) - 1;
            __syncthreads();  // the previous slab's gathers are done
            if constexpr (FUSED) {
              if (cT) {
                // thread t stages box elements e = t + 256 i (the walk of the
                // copying path), EPI of them per pass: the ng selected channels of
                // each voxel come from the channel-major copy cT[i][voxel], so a
                // wave's loads of one channel are 64 consecutive z voxels; the
                // unique segment values m_u = sum_g w[g][u] cT[g] are written as
                // Q float4s
                const long long V = (long long)nx * ny * nz;
                const int nA = A == 0 ? nx : ny, nB = A == 0 ? ny : nx;
                int pl = e_pl, ib = e_ib, iz = e_iz;
                auto voxel = [&](int e, long long &vox) {
                    const int a = A0 + pl - 1, bq = B0 + ib - 1, z = Z0 + iz - 1;
                    const bool in = e < nbox && (unsigned)a < (unsigned)nA && (unsigned)bq < (unsigned)nB &&
                                    (unsigned)z < (unsigned)nz;
                    const int x = A == 0 ? a : bq, y = A == 0 ? bq : a;
                    vox = in ? ((long long)x * ny + y) * nz + z : 0LL;
                    pl += s_pl;
                    ib += s_ib;
                    iz += s_iz;
                    if (iz >= EZ) {
                        iz -= EZ;
                        ++ib;
                    }
                    if (ib >= EB) {
                        ib -= EB;
                        ++pl;
                    }
                    return in;
                };
                // EPI voxels per thread and pass (e = t, t + 256, ...), all
                // their (ng <= NCM) channel loads in flight together, then the
                // weighted sums
                constexpr int EPI = NCM <= 16 ? 4 : 2;
                for (int e0 = threadIdx.x; e0 < nbox; e0 += 256 * EPI) {
                    long long vv[EPI];
                    bool in[EPI];
#pragma unroll
                    for (int i = 0; i < EPI; ++i) in[i] = voxel(e0 + 256 * i, vv[i]);
                    float x[EPI][NCM];
#pragma unroll
                    for (int g = 0; g < NCM; ++g) {
#pragma unroll
                        for (int i = 0; i < EPI; ++i) x[i][g] = 0.0f;
                        if (g < ng) {
                            const float *ch = cT + (long long)gch[g] * V;
#pragma unroll
                            for (int i = 0; i < EPI; ++i) x[i][g] = ch[vv[i]];
                        }
                    }
                    float m[EPI][UP];
#pragma unroll
                    for (int i = 0; i < EPI; ++i)
#pragma unroll
                        for (int u = 0; u < UP; ++u) m[i][u] = 0.0f;
#pragma unroll
                    for (int g = 0; g < NCM; ++g) {
                        if (g < ng) {
#pragma unroll
                            for (int u = 0; u < UP; ++u) {
                                const float wv = gw[g * UP + u];
#pragma unroll
                                for (int i = 0; i < EPI; ++i) m[i][u] = fmaf(wv, x[i][g], m[i][u]);
                            }
                        }
                    }
#pragma unroll
                    for (int q = 0; q < Q; ++q)
#pragma unroll
                        for (int i = 0; i < EPI; ++i)
                            if (e0 + 256 * i < nbox)
                                box[q * nbs + e0 + 256 * i] =
                                    in[i] ? f4{m[i][4 * q], m[i][4 * q + 1], m[i][4 * q + 2], m[i][4 * q + 3]}
                                          : f4{0.f, 0.f, 0.f, 0.f};
                }
              } else {
                // work item (box voxel e, segment u = thread mod UP), VS voxels per
                // pass; EF items per thread have their loads in flight together
                // (an item outside the volume reads c's first voxel and stores 0)
                constexpr int VS = 256 / UP, EF = 4;
                const int u = threadIdx.x & (UP - 1);
                float *boxf = reinterpret_cast<float *>(box) + (long long)(u >> 2) * nbs * 4 + (u & 3);
                const int2 *tu = tab + u * kk;
                const int v0 = threadIdx.x / UP;
                int pl = v0 / plane, ib = (v0 - pl * plane) / EZ, iz = v0 - pl * plane - ib * EZ;
                const int t_pl = VS / plane, t_r = VS - t_pl * plane, t_ib = t_r / EZ, t_iz = t_r - t_ib * EZ;
                const int nA = A == 0 ? nx : ny, nB = A == 0 ? ny : nx;
                for (int e0 = v0; e0 < nbox; e0 += VS * EF) {
                    const float *src[EF];
                    bool ok[EF];
#pragma unroll
                    for (int i = 0; i < EF; ++i) {
                        const int a = A0 + pl - 1, bq = B0 + ib - 1, z = Z0 + iz - 1;
                        ok[i] = u < U && e0 + VS * i < nbox && (unsigned)a < (unsigned)nA &&
                                (unsigned)bq < (unsigned)nB && (unsigned)z < (unsigned)nz;
                        const int x = A == 0 ? a : bq, y = A == 0 ? bq : a;
                        src[i] = M + (ok[i] ? ((long long)(x * ny + y) * nz + z) * C : 0LL);
                        pl += t_pl;
                        ib += t_ib;
                        iz += t_iz;
                        if (iz >= EZ) {
                            iz -= EZ;
                            ++ib;
                        }
                        if (ib >= EB) {
                            ib -= EB;
                            ++pl;
                        }
                    }
                    float v[EF];
#pragma unroll
                    for (int i = 0; i < EF; ++i) v[i] = 0.0f;
#pragma unroll 2
                    for (int t = 0; t < kk; ++t) {
                        const int2 te = tu[t];
                        const float wt = __int_as_float(te.y);
#pragma unroll
                        for (int i = 0; i < EF; ++i) v[i] = fmaf(wt, src[i][te.x], v[i]);
                    }
#pragma unroll
                    for (int i = 0; i < EF; ++i)
                        if (e0 + VS * i < nbox) boxf[(e0 + VS * i) * 4] = ok[i] ? v[i] : 0.0f;
                }
              }
            } else {
            // direct global -> LDS copies (gfx950 global_load_lds, 16 bytes a
            // lane): wave w copies elements e = 256 i + 64 w + lane of every
            // float4 component array, all in flight together; elements outside
            // the padded volume and the tail up to the 64-element stride copy
            // the zero border voxel at padded index 0
            const f4 *src0 = reinterpret_cast<const f4 *>(Mp) + ((long long)A0 * sA + (long long)B0 * sB + Z0) * Q;
            const f4 *zsrc = reinterpret_cast<const f4 *>(Mp);
            const int wb = threadIdx.x & ~63, lane = threadIdx.x & 63;
            int pl = e_pl, ib = e_ib, iz = e_iz, off = e_pl * sA + e_ib * sB + e_iz;
            for (int eb = wb; eb < nbox; eb += 256) {
                const bool in = eb + lane < nbox && (unsigned)(A0 + pl) <= nAp && (unsigned)(B0 + ib) <= nBp &&
                                (unsigned)(Z0 + iz) <= nZp;
                const f4 *gsrc = in ? src0 + (long long)off * Q : zsrc;
#pragma unroll
                for (int q = 0; q < Q; ++q)
                    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(gsrc + q),
                                                     (__attribute__((address_space(3))) void *)(box + q * nbs + eb),
                                                     16, 0, 0);
                // advance by 256 elements
                pl += s_pl;
                ib += s_ib;
                iz += s_iz;
                off += s_off;
                if (iz >= EZ) {
                    iz -= EZ;
                    ++ib;
                    off += cz_off;
                }
                if (ib >= EB) {
                    ib -= EB;
                    ++pl;
                    off += cb_off;
                }
            }
            __builtin_amdgcn_s_waitcnt(0);
            }
            __syncthreads();
            // samples of this slab: index position along A below A0 + W
            int m_end = m;
            if (m < count) m_end = min(count, max(m, (int)ceil((A0 + W - q0[A]) * inv_dqA)));
            // positions relative to the box origin, in float32 (magnitudes of a
            // few tens); the cell is clamped into the box and the fractions are
            // taken against the clamped cell, so a sample that rounding puts
            // on the far side of a slab face still interpolates correctly
            const float ra = (float)(fma((double)m, dq[A], q0[A]) - A0);
            const float rb = (float)(fma((double)m, dq[B], q0[B]) - B0);
            const float rz = (float)(fma((double)m, dq[2], q0[2]) - Z0);
            float mm = 0.0f;
            for (; m < m_end; ++m, mm += 1.0f) {
                const float pa = fmaf(mm, dqA, ra), pb = fmaf(mm, dqB, rb), pz = fmaf(mm, dqZ, rz);
                const float la = fminf(fmaxf(floorf(pa), 0.0f), wmax);
                const float lbb = fminf(fmaxf(floorf(pb), 0.0f), bmax);
                const float lz = fminf(fmaxf(floorf(pz), 0.0f), zmax);
                const float fa = pa - la, fb = pb - lbb, fz = pz - lz;
                const float ga_ = 1.0f - fa, gb_ = 1.0f - fb, gz_ = 1.0f - fz;
                const float w00 = ga_ * gb_, w01 = ga_ * fb, w10 = fa * gb_, w11 = fa * fb;
                const float w[8] = {w00 * gz_, w00 * fz, w01 * gz_, w01 * fz, w10 * gz_, w10 * fz, w11 * gz_, w11 * fz};
                const int off8[8] = {0, dz, db, db + dz, da, da + dz, da + db, da + db + dz};
                const int base = __umul24(__umul24((int)la, EB) + (int)lbb, EZ) + (int)lz;
#pragma unroll
                for (int cc = 0; cc < 8; ++cc) {
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const f4 mv = box[q * nbs + base + off8[cc]];
                        acc[4 * q + 0] = fmaf(w[cc], mv.x, acc[4 * q + 0]);
                        acc[4 * q + 1] = fmaf(w[cc], mv.y, acc[4 * q + 1]);
                        acc[4 * q + 2] = fmaf(w[cc], mv.z, acc[4 * q + 2]);
                        acc[4 * q + 3] = fmaf(w[cc], mv.w, acc[4 * q + 3]);
                    }
                }
            }
        }
    }
    if (!live) return;
    const float wgt = jos ? f.jos_w : step;  // Joseph: each cut weighs 1 / |d_A|
    float *out = I + (((long long)s * nj + j) * nk + k) * nseg;
#pragma unroll
    for (int u = 0; u < UP; ++u) {
        if (u < U) {
            for (int cseg = u; cseg < nseg; cseg += U) out[cseg] = wgt * acc[u];
        }
    }
}

template <int UP>
static hipError_t march_t(const Dims &d, const ProjFrame *frames, const float *M, int s0, int np, float *I,
                          hipStream_t st)
{
    const long long vol_pad = (long long)(d.nx + 2) * (d.ny + 2) * (d.nz + 2);
    dim3 grid(((d.nk + kMarchTile - 1) / kMarchTile) * ((d.nj + kMarchTile - 1) / kMarchTile) * np);
    hipLaunchKernelGGL((k_march<UP, false>), grid, dim3(kMarchTile * kMarchTile), d.march_lds, st, M, frames, s0,
                       d.nx, d.ny, d.nz, d.nj, d.nk, d.nseg, d.U, d.step, vol_pad, I, nullptr, 0, 0, nullptr, nullptr, 0,
                       d.joseph);
    return hipGetLastError();
}

template <int UP>
static hipError_t march_fused_t(const Dims &d, const ProjFrame *frames, const float *c, const int2 *sp,
                                const float *cT, const int *gtab, float *I, hipStream_t st)
{
    dim3 grid(((d.nk + kMarchTile - 1) / kMarchTile) * ((d.nj + kMarchTile - 1) / kMarchTile) * d.S);
    const int lds = (UP * d.sparse_k * 8 + 15) / 16 * 16 + (d.sparse_ng * (UP + 1) * 4 + 15) / 16 * 16 + d.march_lds;
    // channel-major staging unrolled for up to 8, 16 or kFusedCmChannels
    // channels (the wider forms cost registers that narrow lists do not need)
    static_assert(kFusedCmChannels == 32, "the widths below");
    if (cT && d.sparse_ng > kFusedCmChannels) return hipErrorInvalidValue;
    if (cT && d.sparse_ng > 16)
        hipLaunchKernelGGL((k_march<UP, true, 32>), grid, dim3(kMarchTile * kMarchTile), lds, st, c, frames, 0, d.nx,
                           d.ny, d.nz, d.nj, d.nk, d.nseg, d.U, d.step, 0LL, I, sp, d.sparse_k, d.C, cT, gtab,
                           d.sparse_ng, d.joseph);
    else if (cT && d.sparse_ng > 8)
        hipLaunchKernelGGL((k_march<UP, true, 16>), grid, dim3(kMarchTile * kMarchTile), lds, st, c, frames, 0, d.nx,
                           d.ny, d.nz, d.nj, d.nk, d.nseg, d.U, d.step, 0LL, I, sp, d.sparse_k, d.C, cT, gtab,
                           d.sparse_ng, d.joseph);
    else
        hipLaunchKernelGGL((k_march<UP, true, 8>), grid, dim3(kMarchTile * kMarchTile), lds, st, c, frames, 0, d.nx,
                           d.ny, d.nz, d.nj, d.nk, d.nseg, d.U, d.step, 0LL, I, sp, d.sparse_k, d.C, cT, gtab,
                           d.sparse_ng, d.joseph);
    return hipGetLastError();
}

// cT[i][v] = c[v][i]: 64 voxels per block step, staged in LDS (odd row stride)
__global__ __launch_bounds__(256) void k_channel_major(const float *__restrict__ c, long long V, int C,
                                                       float *__restrict__ cT)
{
    extern __shared__ float tile[];  // [64][C + 1]
    const int ld = C + 1;
    for (long long v0 = (long long)blockIdx.x * 64; v0 < V; v0 += (long long)gridDim.x * 64) {
        const int nv = (int)min(64LL, V - v0);
        __syncthreads();
        for (int e = threadIdx.x; e < nv * C; e += 256) {
            const int v = e / C, i = e - v * C;
            tile[v * ld + i] = c[v0 * C + e];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * C; e += 256) {
            const int i = e >> 6, v = e & 63;
            if (v < nv) cT[(long long)i * V + v0 + v] = tile[v * ld + i];
        }
    }
}

hipError_t launch_march_fused(const Dims &d, const ProjFrame *frames, const float *c, const int2 *sp,
                              const int *gtab, float *cT, float *I, hipStream_t st)
{
    if (d.sparse_k < 1) return hipErrorInvalidValue;
    const long long V = (long long)d.nx * d.ny * d.nz;
    if (d.sparse_cm)
        hipLaunchKernelGGL(k_channel_major, dim3((unsigned)std::min<long long>((V + 63) / 64, 4096)), dim3(256),
                           64 * (d.C + 1) * sizeof(float), st, c, V, d.C, cT);
    else
        cT = nullptr;  // stage from the coefficient records
    switch (d.Up) {
    case 4: return march_fused_t<4>(d, frames, c, sp, cT, gtab, I, st);
    case 8: return march_fused_t<8>(d, frames, c, sp, cT, gtab, I, st);
    case 16: return march_fused_t<16>(d, frames, c, sp, cT, gtab, I, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_march(const Dims &d, const ProjFrame *frames, const float *M, int s0, int np, float *I,
                        hipStream_t st)
{
    switch (d.Up) {
    case 4: return march_t<4>(d, frames, M, s0, np, I, st);
    case 8: return march_t<8>(d, frames, M, s0, np, I, st);
    case 16: return march_t<16>(d, frames, M, s0, np, I, st);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// fold: yf = scale * antipodal fold of y (zero beyond U).
// ---------------------------------------------------------------------------
template <int UP>
__global__ __launch_bounds__(256) void k_fold(const float *__restrict__ y, long long npix, int nseg, int U,
                                              float scale, float *__restrict__ yf)
{
    for (long long px = blockIdx.x * 256LL + threadIdx.x; px < npix; px += (long long)gridDim.x * 256) {
        const float *yr = y + px * nseg;
        float acc[UP];
#pragma unroll
        for (int u = 0; u < UP; ++u) acc[u] = 0.0f;
#pragma unroll
        for (int u = 0; u < UP; ++u)
            if (u < U)
                for (int cseg = u; cseg < nseg; cseg += U) acc[u] += yr[cseg];
        f4 *o = reinterpret_cast<f4 *>(yf + px * UP);
#pragma unroll
        for (int u4 = 0; u4 < UP; u4 += 4)
            o[u4 / 4] = f4{scale * acc[u4], scale * acc[u4 + 1], scale * acc[u4 + 2], scale * acc[u4 + 3]};
    }
}

static int grid_for(long long n) { return (int)min((n + 255) / 256, 4096LL); }

hipError_t launch_fold(const Dims &d, const float *y, float scale, float *yf, hipStream_t st)
{
    const long long npix = (long long)d.S * d.nj * d.nk;
    const int g = grid_for(npix);
    switch (d.Up) {
    case 4: hipLaunchKernelGGL(k_fold<4>, dim3(g), dim3(256), 0, st, y, npix, d.nseg, d.U, scale, yf); break;
    case 8: hipLaunchKernelGGL(k_fold<8>, dim3(g), dim3(256), 0, st, y, npix, d.nseg, d.U, scale, yf); break;
    case 16: hipLaunchKernelGGL(k_fold<16>, dim3(g), dim3(256), 0, st, y, npix, d.nseg, d.U, scale, yf); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// r = Ip - data; yf = step * fold(2 w r); partial sums of w r^2 per block.
template <int UP>
__global__ __launch_bounds__(256) void k_residual_fold(const float *__restrict__ Ip, const float *__restrict__ data,
                                                       const float *__restrict__ w, float *r, long long npix,
                                                       int nseg, int U, float step, float *__restrict__ yf,
                                                       double *__restrict__ partials)
{
    __shared__ double ws[4];
    double loss = 0.0;
    for (long long px = blockIdx.x * 256LL + threadIdx.x; px < npix; px += (long long)gridDim.x * 256) {
        float acc[UP];
#pragma unroll
        for (int u = 0; u < UP; ++u) acc[u] = 0.0f;
#pragma unroll
        for (int u = 0; u < UP; ++u) {
            if (u < U) {
                for (int cseg = u; cseg < nseg; cseg += U) {
                    long long e = px * nseg + cseg;
                    float rv = Ip[e] - data[e];
                    float wv = w ? w[e] : 1.0f;
                    if (r) r[e] = rv;
                    loss += (double)wv * (double)rv * (double)rv;
                    acc[u] += 2.0f * wv * rv;
                }
            }
        }
        f4 *o = reinterpret_cast<f4 *>(yf + px * UP);
#pragma unroll
        for (int u4 = 0; u4 < UP; u4 += 4)
            o[u4 / 4] = f4{step * acc[u4], step * acc[u4 + 1], step * acc[u4 + 2], step * acc[u4 + 3]};
    }
    double tot = block_sum(loss, ws);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

hipError_t launch_residual_fold(const Dims &d, const float *Ip, const float *data, const float *w, float *r,
                                float *yf, double *partials, int nblocks, hipStream_t st)
{
    const long long npix = (long long)d.S * d.nj * d.nk;
    switch (d.Up) {
    case 4:
        hipLaunchKernelGGL(k_residual_fold<4>, dim3(nblocks), dim3(256), 0, st, Ip, data, w, r, npix, d.nseg, d.U,
                           d.step, yf, partials);
        break;
    case 8:
        hipLaunchKernelGGL(k_residual_fold<8>, dim3(nblocks), dim3(256), 0, st, Ip, data, w, r, npix, d.nseg, d.U,
                           d.step, yf, partials);
        break;
    case 16:
        hipLaunchKernelGGL(k_residual_fold<16>, dim3(nblocks), dim3(256), 0, st, Ip, data, w, r, npix, d.nseg,
                           d.U, d.step, yf, partials);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// backproject: block = brick of 4 (x) x 8 (y) x 8 (z) voxels; wave w owns the
// x-slice w (64 voxels = 4 column tiles of 16).  Loops over all projections.
// ---------------------------------------------------------------------------
// Q tile entry (u = 4 ks + lane / 16) of voxel column 16 nt + lane % 16 (row stride UP + 1)
template <int UP>
__device__ __forceinline__ float qw_at(const float *Qw, int nt, int ks, int lane)
{
    return Qw[(nt * 16 + (lane & 15)) * (UP + 1) + ks * 4 + (lane >> 4)];
}

template <int UP, int MT, bool BF16, bool JOS>
__global__ __launch_bounds__(256) void k_backproject(const float *__restrict__ yf, const ProjFrame *__restrict__ frames,
                                                     const float *__restrict__ Bu, const s4 *__restrict__ BuT16, int S, int nx, int ny, int nz,
                                                     int nj, int nk, int C, int Cp, float step,
                                                     float *__restrict__ g, float beta, const float *__restrict__ c,
                                                     double *__restrict__ partials)
{
    __shared__ float Qs[4][64 * (UP + 1)];
    __shared__ double ws[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nbx = (nx + 3) / 4, nby = (ny + 7) / 8;
    const int bid = xcd_block(blockIdx.x, gridDim.x);
    const int bx = bid % nbx, by = (bid / nbx) % nby, bz = bid / (nbx * nby);
    const int ix = bx * 4 + wave, iy = by * 8 + (lane >> 3), iz = bz * 8 + (lane & 7);
    const bool valid = ix < nx && iy < ny && iz < nz;
    const double xv[3] = {ix - 0.5 * (nx - 1), iy - 0.5 * (ny - 1), iz - 0.5 * (nz - 1)};
    const double inv_step = 1.0 / (double)step;
    const float stepf = step, inv_stepf = (float)inv_step;

    f4 acc[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};

    // float32 trilinear path with 8+ unique segments: the last KD of the KS
    // k-steps of projection s's MFMA chain run at the top of projection s + 1,
    // beside that projection's set-up arithmetic, so that no wave issues the
    // whole chain at once (Q_s is still in the wave's LDS tile then)
    constexpr int KS = UP / 4, KD = (BF16 || JOS) ? 0 : KS / 2, KE = KS - KD;
    float pend[KD > 0 ? KD : 1][MT];
    auto deferred_mfma = [&]() {
#pragma unroll
        for (int kd = 0; kd < KD; ++kd) {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const float bv = qw_at<UP>(Qs[wave], nt, KE + kd, lane);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma16x16x4(pend[kd][mt], bv, acc[mt][nt]);
            }
        }
    };
    float *Qw = Qs[wave];
    for (int s = 0; s < S; ++s) {
        const ProjFrame &f = frames[s];
        // this projection's B_s^T operands, loaded now so that the gather below
        // hides their latency (they are only read by the MFMAs at its end)
        s4 avb[MT];
        float avf[UP / 4][MT];
        if constexpr (BF16) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                avb[mt] = BuT16[((long long)s * Cp + mt * 16 + (lane & 15)) * 4 + (lane >> 4)];
        } else {
            const float *Bs = Bu + (long long)s * UP * Cp;
#pragma unroll
            for (int ks = 0; ks < UP / 4; ++ks)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) avf[ks][mt] = Bs[(ks * 4 + (lane >> 4)) * Cp + mt * 16 + (lane & 15)];
        }
        float q[UP];
#pragma unroll
        for (int u = 0; u < UP; ++u) q[u] = 0.0f;
        if (JOS && valid) {
            // Joseph's method: the rays whose cut with the voxel's own layer
            // (normal to the dominant axis) lies within one voxel along the two
            // in-plane axes; weight (1 - |Delta_B|)(1 - |Delta_C|) / |d_A|.
            const double w0 = xv[0] - f.o[0], w1 = xv[1] - f.o[1], w2 = xv[2] - f.o[2];
            const double a = w0 * f.ej[0] + w1 * f.ej[1] + w2 * f.ej[2];
            const double bb = w0 * f.ek[0] + w1 * f.ek[1] + w2 * f.ek[2];
            const double af = floor(a), bf = floor(bb);
            const int ai = (int)af, bi = (int)bf;
            const float ar = (float)(a - af), br = (float)(bb - bf);
            const float gjB = f.jos_gj[0], gjC = f.jos_gj[1], gkB = f.jos_gk[0], gkC = f.jos_gk[1];
            const int jlo = max(0, ai + (int)ceilf(ar - f.jos_rj)), jhi = min(nj - 1, ai + (int)floorf(ar + f.jos_rj));
            for (int j = jlo; j <= jhi; ++j) {
                const float dj = (float)(j - ai) - ar;
                const float eB = dj * gjB, eC = dj * gjC;
                // dk range with |dk gk + e| < 1 on both in-plane axes, branch-free: a
                // flat axis (kFlatInv) gives all dk or none, and the other axis is
                // never flat, so a non-empty range is finite
                const float xB1 = (-1.0f - eB) * f.jos_igk[0], xB2 = (1.0f - eB) * f.jos_igk[0];
                const float xC1 = (-1.0f - eC) * f.jos_igk[1], xC2 = (1.0f - eC) * f.jos_igk[1];
                const float lo = fmaxf(fminf(xB1, xB2), fminf(xC1, xC2));
                const float hi = fminf(fmaxf(xB1, xB2), fmaxf(xC1, xC2));
                if (!(lo < hi)) continue;
                const int klo = max(0, bi + (int)ceilf(br + lo - 1e-4f));
                const int khi = min(nk - 1, bi + (int)floorf(br + hi + 1e-4f));
                const f4 *yrow = reinterpret_cast<const f4 *>(yf + ((long long)s * nj + j) * nk * UP);
                for (int k = klo; k <= khi; ++k) {
                    f4 yv[UP / 4];
#pragma unroll
                    for (int u4 = 0; u4 < UP / 4; ++u4) yv[u4] = yrow[k * (UP / 4) + u4];
                    const float dk = (float)(k - bi) - br;
                    const float wB = fmaxf(0.0f, 1.0f - fabsf(fmaf(dk, gkB, eB)));
                    const float wC = fmaxf(0.0f, 1.0f - fabsf(fmaf(dk, gkC, eC)));
                    const float wt = wB * wC * f.jos_w;
#pragma unroll
                    for (int u4 = 0; u4 < UP; u4 += 4) {
                        q[u4 + 0] = fmaf(wt, yv[u4 / 4].x, q[u4 + 0]);
                        q[u4 + 1] = fmaf(wt, yv[u4 / 4].y, q[u4 + 1]);
                        q[u4 + 2] = fmaf(wt, yv[u4 / 4].z, q[u4 + 2]);
                        q[u4 + 3] = fmaf(wt, yv[u4 / 4].w, q[u4 + 3]);
                    }
                }
            }
        }
        if (!JOS && (KD > 0 || valid)) {
            // (with deferred MFMAs evaluated for every lane, so that they share
            // this block; lanes outside the volume visit no rows)
            // Voxel centre in the ray frame: detector coordinates (a, bb) and
            // the along-ray coordinate t / step, in float64 (magnitudes up to
            // the volume size), each split into an integer and a fraction in
            // [0, 1) so that every offset below is a small float32 number.
            const double w0 = xv[0] - f.o[0], w1 = xv[1] - f.o[1], w2 = xv[2] - f.o[2];
            const double a = w0 * f.ej[0] + w1 * f.ej[1] + w2 * f.ej[2];
            const double bb = w0 * f.ek[0] + w1 * f.ek[1] + w2 * f.ek[2];
            const double ts = (w0 * f.d[0] + w1 * f.d[1] + w2 * f.d[2]) * inv_step;
            const double af = floor(a), bf = floor(bb), tf = floor(ts);
            const int ai = (int)af, bi = (int)bf, ti = (int)tf;
            const float ar = (float)(a - af), br = (float)(bb - bf), tr = (float)(ts - tf);
            const float hinv[3] = {fabsf(f.inv_df[0]), fabsf(f.inv_df[1]), fabsf(f.inv_df[2])};
            // -|1/d| per axis, held in vector registers: the range fma below
            // already reads 1/d from a scalar register, and a VOP3 takes one
            float nhv[3] = {-hinv[0], -hinv[1], -hinv[2]};
            asm volatile("" : "+v"(nhv[0]), "+v"(nhv[1]), "+v"(nhv[2]));
            const float ljf = (float)f.lj;
            const int jlo = max(0, ai + (int)ceilf(ar - ljf));
            const int jhi = valid ? min(nj - 1, ai + (int)floorf(ar + ljf)) : jlo - 1;
            if constexpr (KD > 0) {
                if (s > 0) deferred_mfma();
            }
            // hull intercepts shifted by this voxel's fraction br and the 1e-4 slack
            const float cu[3] = {f.hull[1] + (br + 1e-4f), f.hull[3] + (br + 1e-4f), f.hull[5] + (br + 1e-4f)};
            const float cl[3] = {f.hull[7] + (br - 1e-4f), f.hull[9] + (br - 1e-4f), f.hull[11] + (br - 1e-4f)};
            const f4 *ys = reinterpret_cast<const f4 *>(yf + (long long)s * nj * nk * UP);
            for (int j = jlo; j <= jhi; ++j) {
                // rays of this row that can meet the open cube around the voxel
                const float dj = (float)(j - ai) - ar;
                const float zmax = fminf(fminf(fmaf(f.hull[0], dj, cu[0]), fmaf(f.hull[2], dj, cu[1])),
                                         fmaf(f.hull[4], dj, cu[2]));
                const float zmin = fmaxf(fmaxf(fmaf(f.hull[6], dj, cl[0]), fmaf(f.hull[8], dj, cl[1])),
                                         fmaf(f.hull[10], dj, cl[2]));
                const int klo = max(0, bi + (int)ceilf(zmin));
                const int khi = min(nk - 1, bi + (int)floorf(zmax));
                const float pj0 = dj * f.ejf[0], pj1 = dj * f.ejf[1], pj2 = dj * f.ejf[2];
                const f4 *yrow = ys + __umul24(j, nk * (UP / 4));  // row offsets stay below 2^24 float4
                float dk = (float)(klo - bi) - br;
                for (int k = klo; k <= khi; ++k, dk += 1.0f) {
                    f4 yv[UP / 4];
#pragma unroll
                    for (int u4 = 0; u4 < UP / 4; ++u4) yv[u4] = yrow[k * (UP / 4) + u4];  // in flight meanwhile
                    const float P[3] = {fmaf(dk, f.ekf[0], pj0), fmaf(dk, f.ekf[1], pj1), fmaf(dk, f.ekf[2], pj2)};
                    // parameter range along the ray inside the open cube: |P_m + tau d_m| < 1
                    // for every axis (branch-free: see kFlatInv for rays parallel to a face)
                    float tlo = fmaf(-P[0], f.inv_df[0], nhv[0]), thi = fmaf(-P[0], f.inv_df[0], hinv[0]);
#pragma unroll
                    for (int m = 1; m < 3; ++m) {
                        tlo = fmaxf(tlo, fmaf(-P[m], f.inv_df[m], nhv[m]));
                        thi = fminf(thi, fmaf(-P[m], f.inv_df[m], hinv[m]));
                    }
                    // samples n with tau = n step - t inside (tlo, thi): n from m0 to m1
                    // (none if the range is empty); there every |P_m + tau d_m| < 1, so
                    // the tent factors need no clamp at 0 (a sample at the boundary
                    // gives a factor of rounding size).  The loop runs on tau itself,
                    // whose end is put half a step past the last sample.
                    float wsum = 0.0f;
                    const float m0 = ceilf(fmaf(tlo, inv_stepf, tr)), m1 = floorf(fmaf(thi, inv_stepf, tr));
                    const float tend = (m1 - tr + 0.5f) * stepf;
                    for (float tau = (m0 - tr) * stepf; tau < tend; tau += stepf) {
                        const float wx = 1.0f - fabsf(fmaf(tau, f.df[0], P[0]));
                        const float wy = 1.0f - fabsf(fmaf(tau, f.df[1], P[1]));
                        const float wz = 1.0f - fabsf(fmaf(tau, f.df[2], P[2]));
                        wsum = fmaf(wx * wy, wz, wsum);
                    }
#pragma unroll
                    for (int u4 = 0; u4 < UP; u4 += 4) {
                        q[u4 + 0] = fmaf(wsum, yv[u4 / 4].x, q[u4 + 0]);
                        q[u4 + 1] = fmaf(wsum, yv[u4 / 4].y, q[u4 + 1]);
                        q[u4 + 2] = fmaf(wsum, yv[u4 / 4].z, q[u4 + 2]);
                        q[u4 + 3] = fmaf(wsum, yv[u4 / 4].w, q[u4 + 3]);
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < UP; ++u) Qw[lane * (UP + 1) + u] = q[u];
        // Qw is private to this wave, whose LDS accesses complete in program
        // order: only compiler reordering has to be fenced.
        __builtin_amdgcn_wave_barrier();
        // g tile += B_s^T (coefficients x u) * Q^T (u x voxels)
        if constexpr (BF16) {
            // K = 16 (u padded with zeros): A from BuT16[s][coefficient][u], B = Q rounded to bf16
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const float *qv = Qw + (nt * 16 + (lane & 15)) * (UP + 1);
                const int u0 = 4 * (lane >> 4);
                s4 bv;
                bv.x = u0 + 0 < UP ? f2bf(qv[min(u0 + 0, UP - 1)]) : (short)0;
                bv.y = u0 + 1 < UP ? f2bf(qv[min(u0 + 1, UP - 1)]) : (short)0;
                bv.z = u0 + 2 < UP ? f2bf(qv[min(u0 + 2, UP - 1)]) : (short)0;
                bv.w = u0 + 3 < UP ? f2bf(qv[min(u0 + 3, UP - 1)]) : (short)0;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma16x16x16bf16(avb[mt], bv, acc[mt][nt]);
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < KE; ++ks) {
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const float bv = qw_at<UP>(Qw, nt, ks, lane);
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma16x16x4(avf[ks][mt], bv, acc[mt][nt]);
                }
            }
#pragma unroll
            for (int kd = 0; kd < KD; ++kd)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) pend[kd][mt] = avf[KE + kd][mt];
        }
        __builtin_amdgcn_wave_barrier();
    }
    if constexpr (KD > 0) {
        if (S > 0) deferred_mfma();
    }

    // epilogue: lane holds rows (coefficients) 16 mt + 4 (lane/16) + r of voxel column 16 nt + lane % 16
    double c2 = 0.0;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int lv = nt * 16 + (lane & 15);
        const int vy = by * 8 + (lv >> 3), vz = bz * 8 + (lv & 7);
        if (ix < nx && vy < ny && vz < nz) {
            const long long base = (((long long)ix * ny + vy) * nz + vz) * C;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = mt * 16 + 4 * (lane >> 4) + r;
                    if (i < C) {
                        float val = acc[mt][nt][r];
                        if (c) {
                            float cv = c[base + i];
                            val += beta * cv;
                            c2 += (double)cv * (double)cv;
                        }
                        g[base + i] = val;
                    }
                }
            }
        }
    }
    if (partials) {
        double tot = block_sum(c2, ws);
        if (tid == 0) partials[bid] = tot;
    }
}


// ---------------------------------------------------------------------------
// backproject, paired by point inversion (trilinear model, no detector
// offsets, even nx, four unique segments).  The sample lattice of a projection,
// o + j e_j + k e_k + n step d with o = -((nj-1)/2 e_j + (nk-1)/2 e_k), is
// symmetric under x -> -x with (j, k, n) -> (nj-1-j, nk-1-k, -n); the voxel
// grid and the tent are symmetric too.  So the weight of ray (j, k) at voxel
// v equals the weight of ray (nj-1-j, nk-1-k) at the inverted voxel
// v' = (nx-1-ix, ny-1-iy, nz-1-iz), and one enumeration of v's rays and
// samples gives Q_s(v) and Q_s(v') (the second from the mirrored residual
// rows).  Block: waves 0, 1 own x-slices 2 bx + w of the lower half
// (ix < nx / 2) over an 8 x 8 (y, z) tile; waves 2, 3 own the inverses of
// waves 0, 1's voxels lane by lane.  Per pair of projections (s, s + 1) the
// lower waves enumerate s and the upper waves s + 1; each hands the
// partner's Q through LDS, and each wave then contracts both projections'
// Q with B^T on MFMA into its own accumulators.  Enumeration work per voxel
// and projection is halved; the transpose maps are unchanged.
// ---------------------------------------------------------------------------
template <int UP, int MT, bool BF16, bool JOS>
__global__ __launch_bounds__(256) void k_backproject_inv(const float *__restrict__ yf,
                                                         const ProjFrame *__restrict__ frames,
                                                         const float *__restrict__ Bu, const s4 *__restrict__ BuT16,
                                                         int S, int nx, int ny, int nz, int nj, int nk, int C, int Cp,
                                                         float step, float *__restrict__ g, float beta,
                                                         const float *__restrict__ c, double *__restrict__ partials)
{
    constexpr int QS = 64 * (UP + 1);
    __shared__ float Qs[4][QS];      // each wave's own Q (wave-private)
    __shared__ float Qx[2][4][QS];   // Q handed over by the partner wave, double-buffered
    __shared__ double ws[4];
    const int tid = threadIdx.x, lane = tid & 63;
    // wave-uniform (scalar) wave index: the projection each wave enumerates, and
    // hence its frame loads, stay in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool upper = wave >= 2;
    const int nxh = nx >> 1;
    const int nbx = (nxh + 1) / 2, nby = (ny + 7) / 8;
    const int bid = xcd_block(blockIdx.x, gridDim.x);
    const int bx = bid % nbx, by = (bid / nbx) % nby, bz = bid / (nbx * nby);
    // the lower-half voxel of this lane's pair, and this wave's own voxel
    const int px = bx * 2 + (wave & 1), py = by * 8 + (lane >> 3), pz = bz * 8 + (lane & 7);
    const bool valid = px < nxh && py < ny && pz < nz;
    const int ix = upper ? nx - 1 - px : px, iy = upper ? ny - 1 - py : py, iz = upper ? nz - 1 - pz : pz;
    const double xv[3] = {ix - 0.5 * (nx - 1), iy - 0.5 * (ny - 1), iz - 0.5 * (nz - 1)};
    const double inv_step = 1.0 / (double)step;
    const float stepf = step, inv_stepf = (float)inv_step;

    f4 acc[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};

    // B_s^T operands of one projection in MFMA lane order (loaded at the top of
    // an iteration, so that the enumeration hides their latency)
    struct BOps {
        s4 b16[BF16 ? MT : 1];
        float f[BF16 ? 1 : UP / 4][MT];
    };
    auto load_ops = [&](int s, BOps &o) {
        if constexpr (BF16) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                o.b16[mt] = BuT16[((long long)s * Cp + mt * 16 + (lane & 15)) * 4 + (lane >> 4)];
        } else {
            const float *Bs = Bu + (long long)s * UP * Cp;
#pragma unroll
            for (int ks = 0; ks < UP / 4; ++ks)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) o.f[ks][mt] = Bs[(ks * 4 + (lane >> 4)) * Cp + mt * 16 + (lane & 15)];
        }
    };
    // g tile += B_s^T (coefficients x u) * Q^T (u x voxels), Q from the LDS tile Qt
    auto contract = [&](const BOps &o, const float *Qt) {
        if constexpr (BF16) {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const float *qv = Qt + (nt * 16 + (lane & 15)) * (UP + 1);
                const int u0 = 4 * (lane >> 4);
                s4 bv;
                bv.x = u0 + 0 < UP ? f2bf(qv[min(u0 + 0, UP - 1)]) : (short)0;
                bv.y = u0 + 1 < UP ? f2bf(qv[min(u0 + 1, UP - 1)]) : (short)0;
                bv.z = u0 + 2 < UP ? f2bf(qv[min(u0 + 2, UP - 1)]) : (short)0;
                bv.w = u0 + 3 < UP ? f2bf(qv[min(u0 + 3, UP - 1)]) : (short)0;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma16x16x16bf16(o.b16[mt], bv, acc[mt][nt]);
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < UP / 4; ++ks) {
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const float bv = qw_at<UP>(Qt, nt, ks, lane);
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma16x16x4(o.f[ks][mt], bv, acc[mt][nt]);
                }
            }
        }
    };

    int buf = 0;
    for (int s0 = 0; s0 < S; s0 += 2) {
        const int s_own = s0 + (upper ? 1 : 0), s_oth = s0 + (upper ? 0 : 1);
        const bool has_own = s_own < S, has_oth = s_oth < S;
        BOps ops_own, ops_oth;
        load_ops(has_own ? s_own : s0, ops_own);
        load_ops(has_oth ? s_oth : s0, ops_oth);
        float q[UP], qm[UP];
#pragma unroll
        for (int u = 0; u < UP; ++u) q[u] = qm[u] = 0.0f;
        if (has_own && valid) {
            const ProjFrame &f = frames[s_own];
            if constexpr (JOS) {
                // Joseph's method: the rays whose cut with the voxel's layer lies
                // within one voxel in-plane, weight (1 - |Delta_B|)(1 - |Delta_C|) /
                // |d_A|; the inverse voxel's cut of the mirrored ray is the negated
                // cut point, so the same weight serves both voxels of the pair
                const double w0 = xv[0] - f.o[0], w1 = xv[1] - f.o[1], w2 = xv[2] - f.o[2];
                const double a = w0 * f.ej[0] + w1 * f.ej[1] + w2 * f.ej[2];
                const double bb = w0 * f.ek[0] + w1 * f.ek[1] + w2 * f.ek[2];
                const double af = floor(a), bf = floor(bb);
                const int ai = (int)af, bi = (int)bf;
                const float ar = (float)(a - af), br = (float)(bb - bf);
                const float gjB = f.jos_gj[0], gjC = f.jos_gj[1], gkB = f.jos_gk[0], gkC = f.jos_gk[1];
                const int jlo = max(0, ai + (int)ceilf(ar - f.jos_rj));
                const int jhi = min(nj - 1, ai + (int)floorf(ar + f.jos_rj));
                const f4 *ys = reinterpret_cast<const f4 *>(yf + (long long)s_own * nj * nk * UP);
                for (int j = jlo; j <= jhi; ++j) {
                    const float dj = (float)(j - ai) - ar;
                    const float eB = dj * gjB, eC = dj * gjC;
                    // dk range with |dk gk + e| < 1 on both in-plane axes (a flat
                    // axis gives all dk or none; the other one is never flat)
                    const float xB1 = (-1.0f - eB) * f.jos_igk[0], xB2 = (1.0f - eB) * f.jos_igk[0];
                    const float xC1 = (-1.0f - eC) * f.jos_igk[1], xC2 = (1.0f - eC) * f.jos_igk[1];
                    const float lo = fmaxf(fminf(xB1, xB2), fminf(xC1, xC2));
                    const float hi = fminf(fmaxf(xB1, xB2), fmaxf(xC1, xC2));
                    if (!(lo < hi)) continue;
                    const int klo = max(0, bi + (int)ceilf(br + lo - 1e-4f));
                    const int khi = min(nk - 1, bi + (int)floorf(br + hi + 1e-4f));
                    const f4 *yrow = ys + __umul24(j, nk * (UP / 4));
                    // mirrored ray (nj-1-j, nk-1-k): row nj-1-j read backwards from column nk-1
                    const f4 *yrowm = ys + __umul24(nj - 1 - j, nk * (UP / 4)) + (nk - 1) * (UP / 4);
                    for (int k = klo; k <= khi; ++k) {
                        f4 yv[UP / 4], ym[UP / 4];
#pragma unroll
                        for (int u4 = 0; u4 < UP / 4; ++u4) {
                            yv[u4] = yrow[k * (UP / 4) + u4];
                            ym[u4] = yrowm[u4 - k * (UP / 4)];
                        }
                        const float dk = (float)(k - bi) - br;
                        const float wB = fmaxf(0.0f, 1.0f - fabsf(fmaf(dk, gkB, eB)));
                        const float wC = fmaxf(0.0f, 1.0f - fabsf(fmaf(dk, gkC, eC)));
                        const float wt = wB * wC * f.jos_w;
#pragma unroll
                        for (int u4 = 0; u4 < UP; u4 += 4) {
                            q[u4 + 0] = fmaf(wt, yv[u4 / 4].x, q[u4 + 0]);
                            q[u4 + 1] = fmaf(wt, yv[u4 / 4].y, q[u4 + 1]);
                            q[u4 + 2] = fmaf(wt, yv[u4 / 4].z, q[u4 + 2]);
                            q[u4 + 3] = fmaf(wt, yv[u4 / 4].w, q[u4 + 3]);
                            qm[u4 + 0] = fmaf(wt, ym[u4 / 4].x, qm[u4 + 0]);
                            qm[u4 + 1] = fmaf(wt, ym[u4 / 4].y, qm[u4 + 1]);
                            qm[u4 + 2] = fmaf(wt, ym[u4 / 4].z, qm[u4 + 2]);
                            qm[u4 + 3] = fmaf(wt, ym[u4 / 4].w, qm[u4 + 3]);
                        }
                    }
                }
            } else {
                // voxel centre in the ray frame (float64), split into integer + fraction
                const double w0 = xv[0] - f.o[0], w1 = xv[1] - f.o[1], w2 = xv[2] - f.o[2];
                const double a = w0 * f.ej[0] + w1 * f.ej[1] + w2 * f.ej[2];
                const double bb = w0 * f.ek[0] + w1 * f.ek[1] + w2 * f.ek[2];
                const double ts = (w0 * f.d[0] + w1 * f.d[1] + w2 * f.d[2]) * inv_step;
                const double af = floor(a), bf = floor(bb), tf = floor(ts);
                const int ai = (int)af, bi = (int)bf;
                const float ar = (float)(a - af), br = (float)(bb - bf), tr = (float)(ts - tf);
                const float hinv[3] = {fabsf(f.inv_df[0]), fabsf(f.inv_df[1]), fabsf(f.inv_df[2])};
                float nhv[3] = {-hinv[0], -hinv[1], -hinv[2]};
                asm volatile("" : "+v"(nhv[0]), "+v"(nhv[1]), "+v"(nhv[2]));
                // the sample step in vector registers: reloading it from the frame per
                // ray (scalar pressure) made each ray wait on the scalar load
                float dfv[3] = {f.df[0], f.df[1], f.df[2]};
                asm volatile("" : "+v"(dfv[0]), "+v"(dfv[1]), "+v"(dfv[2]));
                const float ljf = (float)f.lj;
                const int jlo = max(0, ai + (int)ceilf(ar - ljf));
                const int jhi = min(nj - 1, ai + (int)floorf(ar + ljf));
                const float cu[3] = {f.hull[1] + (br + 1e-4f), f.hull[3] + (br + 1e-4f), f.hull[5] + (br + 1e-4f)};
                const float cl[3] = {f.hull[7] + (br - 1e-4f), f.hull[9] + (br - 1e-4f), f.hull[11] + (br - 1e-4f)};
                const f4 *ys = reinterpret_cast<const f4 *>(yf + (long long)s_own * nj * nk * UP);
                for (int j = jlo; j <= jhi; ++j) {
                    const float dj = (float)(j - ai) - ar;
                    const float zmax = fminf(fminf(fmaf(f.hull[0], dj, cu[0]), fmaf(f.hull[2], dj, cu[1])),
                                             fmaf(f.hull[4], dj, cu[2]));
                    const float zmin = fmaxf(fmaxf(fmaf(f.hull[6], dj, cl[0]), fmaf(f.hull[8], dj, cl[1])),
                                             fmaf(f.hull[10], dj, cl[2]));
                    const int klo = max(0, bi + (int)ceilf(zmin));
                    const int khi = min(nk - 1, bi + (int)floorf(zmax));
                    const float pj0 = dj * f.ejf[0], pj1 = dj * f.ejf[1], pj2 = dj * f.ejf[2];
                    const f4 *yrow = ys + __umul24(j, nk * (UP / 4));
                    // mirrored ray (nj-1-j, nk-1-k): row nj-1-j read backwards from column nk-1
                    const f4 *yrowm = ys + __umul24(nj - 1 - j, nk * (UP / 4)) + (nk - 1) * (UP / 4);
                    float dk = (float)(klo - bi) - br;
                    for (int k = klo; k <= khi; ++k, dk += 1.0f) {
                        f4 yv[UP / 4], ym[UP / 4];
#pragma unroll
                        for (int u4 = 0; u4 < UP / 4; ++u4) {
                            yv[u4] = yrow[k * (UP / 4) + u4];
                            ym[u4] = yrowm[u4 - k * (UP / 4)];
                        }
                        const float P[3] = {fmaf(dk, f.ekf[0], pj0), fmaf(dk, f.ekf[1], pj1), fmaf(dk, f.ekf[2], pj2)};
                        float tlo = fmaf(-P[0], f.inv_df[0], nhv[0]), thi = fmaf(-P[0], f.inv_df[0], hinv[0]);
#pragma unroll
                        for (int m = 1; m < 3; ++m) {
                            tlo = fmaxf(tlo, fmaf(-P[m], f.inv_df[m], nhv[m]));
                            thi = fminf(thi, fmaf(-P[m], f.inv_df[m], hinv[m]));
                        }
                        float wsum = 0.0f;
                        const float m0 = ceilf(fmaf(tlo, inv_stepf, tr)), m1 = floorf(fmaf(thi, inv_stepf, tr));
                        const float tend = (m1 - tr + 0.5f) * stepf;
                        for (float tau = (m0 - tr) * stepf; tau < tend; tau += stepf) {
                            const float wx = 1.0f - fabsf(fmaf(tau, dfv[0], P[0]));
                            const float wy = 1.0f - fabsf(fmaf(tau, dfv[1], P[1]));
                            const float wz = 1.0f - fabsf(fmaf(tau, dfv[2], P[2]));
                            wsum = fmaf(wx * wy, wz, wsum);
                        }
#pragma unroll
                        for (int u4 = 0; u4 < UP; u4 += 4) {
                            q[u4 + 0] = fmaf(wsum, yv[u4 / 4].x, q[u4 + 0]);
                            q[u4 + 1] = fmaf(wsum, yv[u4 / 4].y, q[u4 + 1]);
                            q[u4 + 2] = fmaf(wsum, yv[u4 / 4].z, q[u4 + 2]);
                            q[u4 + 3] = fmaf(wsum, yv[u4 / 4].w, q[u4 + 3]);
                            qm[u4 + 0] = fmaf(wsum, ym[u4 / 4].x, qm[u4 + 0]);
                            qm[u4 + 1] = fmaf(wsum, ym[u4 / 4].y, qm[u4 + 1]);
                            qm[u4 + 2] = fmaf(wsum, ym[u4 / 4].z, qm[u4 + 2]);
                            qm[u4 + 3] = fmaf(wsum, ym[u4 / 4].w, qm[u4 + 3]);
                        }
                    }
                }
            }
        }
        float *Qown = Qs[wave];
        float *Qout = Qx[buf][wave ^ 2];
#pragma unroll
        for (int u = 0; u < UP; ++u) {
            Qown[lane * (UP + 1) + u] = q[u];
            Qout[lane * (UP + 1) + u] = qm[u];
        }
        // the partner's tile is complete; the tile of the other buffer was last
        // read before this barrier's predecessor, so one barrier per pair suffices
        __syncthreads();
        if (has_own) contract(ops_own, Qown);
        if (has_oth) contract(ops_oth, Qx[buf][wave]);
        buf ^= 1;
    }

    // epilogue: lane holds rows (coefficients) 16 mt + 4 (lane/16) + r of voxel column 16 nt + lane % 16
    double c2 = 0.0;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int lv = nt * 16 + (lane & 15);
        const int qy = by * 8 + (lv >> 3), qz = bz * 8 + (lv & 7);
        if (px < nxh && qy < ny && qz < nz) {
            const int vx = ix, vy = upper ? ny - 1 - qy : qy, vz = upper ? nz - 1 - qz : qz;
            const long long base = (((long long)vx * ny + vy) * nz + vz) * C;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = mt * 16 + 4 * (lane >> 4) + r;
                    if (i < C) {
                        float val = acc[mt][nt][r];
                        if (c) {
                            float cv = c[base + i];
                            val += beta * cv;
                            c2 += (double)cv * (double)cv;
                        }
                        g[base + i] = val;
                    }
                }
            }
        }
    }
    if (partials) {
        double tot = block_sum(c2, ws);
        if (tid == 0) partials[bid] = tot;
    }
}

// ---------------------------------------------------------------------------
// backproject with the residual window staged in LDS (trilinear model).  Each
// block's 4 x 8 x 8 voxel brick reads, per projection, only the residual rays
// of a small detector window (its shadow widened by the cube's L1 reach); the
// window is copied from HBM into LDS by the direct global-to-LDS loads of
// gfx950 one projection ahead (into the other of two buffers), so that the
// per-ray residual reads of the enumeration are LDS reads instead of
// scattered L2 / HBM loads.  One block barrier per projection (the four
// waves process neighbouring x-slices of the same projection).
// ---------------------------------------------------------------------------
constexpr int kWinMax = 22;  // window rows and columns (the host checks every projection)

template <int UP, int MT, bool BF16>
__global__ __launch_bounds__(256) void k_backproject_win(const float *__restrict__ yf,
                                                         const ProjFrame *__restrict__ frames,
                                                         const float *__restrict__ Bu, const s4 *__restrict__ BuT16,
                                                         int S, int nx, int ny, int nz, int nj, int nk, int C, int Cp,
                                                         float step, float *__restrict__ g, float beta,
                                                         const float *__restrict__ c, double *__restrict__ partials)
{
    constexpr int Q = UP / 4;                 // float4 per ray
    constexpr int WROW = kWinMax * Q;         // float4 per window row
    __shared__ f4 winA[kWinMax * WROW];
    __shared__ f4 winB[kWinMax * WROW];
    __shared__ float Qs[4][64 * (UP + 1)];
    __shared__ double ws[4];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nbx = (nx + 3) / 4, nby = (ny + 7) / 8;
    const int bid = xcd_block(blockIdx.x, gridDim.x);
    const int bx = bid % nbx, by = (bid / nbx) % nby, bz = bid / (nbx * nby);
    const int ix = bx * 4 + wave, iy = by * 8 + (lane >> 3), iz = bz * 8 + (lane & 7);
    const bool valid = ix < nx && iy < ny && iz < nz;
    const double xv[3] = {ix - 0.5 * (nx - 1), iy - 0.5 * (ny - 1), iz - 0.5 * (nz - 1)};
    const double inv_step = 1.0 / (double)step;
    const float stepf = step, inv_stepf = (float)inv_step;

    // detector window of projection s: rows and columns every voxel of the
    // brick can reach (its L1 reach lj, lk around its detector position, one
    // more on each side for rounding), clipped to the detector
    auto window = [&](int s, int &j0, int &k0, int &nr, int &nc) {
        const ProjFrame &f = frames[s];
        // the brick's voxel-centre box (clipped to the volume), centred coordinates
        const double lo3[3] = {bx * 4 - 0.5 * (nx - 1), by * 8 - 0.5 * (ny - 1), bz * 8 - 0.5 * (nz - 1)};
        const double hi3[3] = {min(nx, bx * 4 + 4) - 1 - 0.5 * (nx - 1), min(ny, by * 8 + 8) - 1 - 0.5 * (ny - 1),
                               min(nz, bz * 8 + 8) - 1 - 0.5 * (nz - 1)};
        double amin = 0.0, amax = 0.0, bmin = 0.0, bmax = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double ea = f.ej[a], ka = f.ek[a];
            amin += (ea >= 0.0 ? lo3[a] - f.o[a] : hi3[a] - f.o[a]) * ea;
            amax += (ea >= 0.0 ? hi3[a] - f.o[a] : lo3[a] - f.o[a]) * ea;
            bmin += (ka >= 0.0 ? lo3[a] - f.o[a] : hi3[a] - f.o[a]) * ka;
            bmax += (ka >= 0.0 ? hi3[a] - f.o[a] : lo3[a] - f.o[a]) * ka;
        }
        const int ja = max(0, (int)ceil(amin - f.lj) - 1), jb = min(nj - 1, (int)floor(amax + f.lj) + 1);
        const int ka0 = max(0, (int)ceil(bmin - f.lk) - 1), kb = min(nk - 1, (int)floor(bmax + f.lk) + 1);
        j0 = __builtin_amdgcn_readfirstlane(ja);
        k0 = __builtin_amdgcn_readfirstlane(ka0);
        nr = __builtin_amdgcn_readfirstlane(max(0, min(kWinMax, jb - ja + 1)));
        nc = __builtin_amdgcn_readfirstlane(max(0, min(kWinMax, kb - ka0 + 1)));
    };
    // asynchronous copy of projection s's window into win (rows spread over the waves)
    auto stage = [&](int s, f4 *win, int j0, int k0, int nr, int nc) {
        const f4 *src = reinterpret_cast<const f4 *>(yf) + (((long long)s * nj + j0) * nk + k0) * Q;
        const int rowf4 = nc * Q;
        for (int r = wave; r < nr; r += 4) {
#pragma unroll
            for (int l0 = 0; l0 < WROW; l0 += 64) {
                if (l0 + lane < rowf4)
                    __builtin_amdgcn_global_load_lds(
                        (const __attribute__((address_space(1))) void *)(src + (long long)r * nk * Q + l0 + lane),
                        (__attribute__((address_space(3))) void *)(win + r * WROW + l0), 16, 0, 0);
            }
        }
    };

    f4 acc[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
    float *Qw = Qs[wave];

    // projection s: enumerate from the staged window, then contract on MFMA
    auto body = [&](int s, const f4 *win, int wj0, int wk0, int wnr, int wnc) {
        const ProjFrame &f = frames[s];
        s4 avb[MT];
        float avf[UP / 4][MT];
        if constexpr (BF16) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                avb[mt] = BuT16[((long long)s * Cp + mt * 16 + (lane & 15)) * 4 + (lane >> 4)];
        } else {
            const float *Bs = Bu + (long long)s * UP * Cp;
#pragma unroll
            for (int ks = 0; ks < UP / 4; ++ks)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) avf[ks][mt] = Bs[(ks * 4 + (lane >> 4)) * Cp + mt * 16 + (lane & 15)];
        }
        float q[UP];
#pragma unroll
        for (int u = 0; u < UP; ++u) q[u] = 0.0f;
        if (valid) {
            const double w0 = xv[0] - f.o[0], w1 = xv[1] - f.o[1], w2 = xv[2] - f.o[2];
            const double a = w0 * f.ej[0] + w1 * f.ej[1] + w2 * f.ej[2];
            const double bb = w0 * f.ek[0] + w1 * f.ek[1] + w2 * f.ek[2];
            const double ts = (w0 * f.d[0] + w1 * f.d[1] + w2 * f.d[2]) * inv_step;
            const double af = floor(a), bf = floor(bb), tf = floor(ts);
            const int ai = (int)af, bi = (int)bf;
            const float ar = (float)(a - af), br = (float)(bb - bf), tr = (float)(ts - tf);
            const float hinv[3] = {fabsf(f.inv_df[0]), fabsf(f.inv_df[1]), fabsf(f.inv_df[2])};
            float nhv[3] = {-hinv[0], -hinv[1], -hinv[2]};
            asm volatile("" : "+v"(nhv[0]), "+v"(nhv[1]), "+v"(nhv[2]));
            // the sample step in vector registers: reloading it from the frame per
            // ray (scalar pressure) made each ray wait on the scalar load
            float dfv[3] = {f.df[0], f.df[1], f.df[2]};
            asm volatile("" : "+v"(dfv[0]), "+v"(dfv[1]), "+v"(dfv[2]));
            const float ljf = (float)f.lj;
            // rows and columns stay inside the staged window (it contains every ray
            // the voxel can reach; the clamps only guard the LDS indices)
            const int jlo = max(wj0, ai + (int)ceilf(ar - ljf));
            const int jhi = min(wj0 + wnr - 1, ai + (int)floorf(ar + ljf));
            const float cu[3] = {f.hull[1] + (br + 1e-4f), f.hull[3] + (br + 1e-4f), f.hull[5] + (br + 1e-4f)};
            const float cl[3] = {f.hull[7] + (br - 1e-4f), f.hull[9] + (br - 1e-4f), f.hull[11] + (br - 1e-4f)};
            for (int j = jlo; j <= jhi; ++j) {
                const float dj = (float)(j - ai) - ar;
                const float zmax = fminf(fminf(fmaf(f.hull[0], dj, cu[0]), fmaf(f.hull[2], dj, cu[1])),
                                         fmaf(f.hull[4], dj, cu[2]));
                const float zmin = fmaxf(fmaxf(fmaf(f.hull[6], dj, cl[0]), fmaf(f.hull[8], dj, cl[1])),
                                         fmaf(f.hull[10], dj, cl[2]));
                const int klo = max(wk0, bi + (int)ceilf(zmin));
                const int khi = min(wk0 + wnc - 1, bi + (int)floorf(zmax));
                const float pj0 = dj * f.ejf[0], pj1 = dj * f.ejf[1], pj2 = dj * f.ejf[2];
                const f4 *wrow = win + (j - wj0) * WROW - wk0 * Q;
                float dk = (float)(klo - bi) - br;
                for (int k = klo; k <= khi; ++k, dk += 1.0f) {
                    f4 yv[Q];
#pragma unroll
                    for (int u4 = 0; u4 < Q; ++u4) yv[u4] = wrow[k * Q + u4];
                    const float P[3] = {fmaf(dk, f.ekf[0], pj0), fmaf(dk, f.ekf[1], pj1), fmaf(dk, f.ekf[2], pj2)};
                    float tlo = fmaf(-P[0], f.inv_df[0], nhv[0]), thi = fmaf(-P[0], f.inv_df[0], hinv[0]);
#pragma unroll
                    for (int m = 1; m < 3; ++m) {
                        tlo = fmaxf(tlo, fmaf(-P[m], f.inv_df[m], nhv[m]));
                        thi = fminf(thi, fmaf(-P[m], f.inv_df[m], hinv[m]));
                    }
                    float wsum = 0.0f;
                    const float m0 = ceilf(fmaf(tlo, inv_stepf, tr)), m1 = floorf(fmaf(thi, inv_stepf, tr));
                    const float tend = (m1 - tr + 0.5f) * stepf;
                    for (float tau = (m0 - tr) * stepf; tau < tend; tau += stepf) {
                        const float wx = 1.0f - fabsf(fmaf(tau, dfv[0], P[0]));
                        const float wy = 1.0f - fabsf(fmaf(tau, dfv[1], P[1]));
                        const float wz = 1.0f - fabsf(fmaf(tau, dfv[2], P[2]));
                        wsum = fmaf(wx * wy, wz, wsum);
                    }
#pragma unroll
                    for (int u4 = 0; u4 < UP; u4 += 4) {
                        q[u4 + 0] = fmaf(wsum, yv[u4 / 4].x, q[u4 + 0]);
                        q[u4 + 1] = fmaf(wsum, yv[u4 / 4].y, q[u4 + 1]);
                        q[u4 + 2] = fmaf(wsum, yv[u4 / 4].z, q[u4 + 2]);
                        q[u4 + 3] = fmaf(wsum, yv[u4 / 4].w, q[u4 + 3]);
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < UP; ++u) Qw[lane * (UP + 1) + u] = q[u];
        __builtin_amdgcn_wave_barrier();
        if constexpr (BF16) {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const float *qv = Qw + (nt * 16 + (lane & 15)) * (UP + 1);
                const int u0 = 4 * (lane >> 4);
                s4 bv;
                bv.x = u0 + 0 < UP ? f2bf(qv[min(u0 + 0, UP - 1)]) : (short)0;
                bv.y = u0 + 1 < UP ? f2bf(qv[min(u0 + 1, UP - 1)]) : (short)0;
                bv.z = u0 + 2 < UP ? f2bf(qv[min(u0 + 2, UP - 1)]) : (short)0;
                bv.w = u0 + 3 < UP ? f2bf(qv[min(u0 + 3, UP - 1)]) : (short)0;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma16x16x16bf16(avb[mt], bv, acc[mt][nt]);
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < UP / 4; ++ks) {
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const float bv = qw_at<UP>(Qw, nt, ks, lane);
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma16x16x4(avf[ks][mt], bv, acc[mt][nt]);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    };

    // two buffers: projection s reads one while the copy of projection s + 1
    // fills the other
    int cj0, ck0, cnr, cnc;
    window(0, cj0, ck0, cnr, cnc);
    stage(0, winA, cj0, ck0, cnr, cnc);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int s = 0; s < S; ++s) {
        f4 *cur = (s & 1) ? winB : winA;
        f4 *nxt = (s & 1) ? winA : winB;
        int nj0 = 0, nk0 = 0, nnr = 0, nnc = 0;
        if (s + 1 < S) {
            window(s + 1, nj0, nk0, nnr, nnc);
            stage(s + 1, nxt, nj0, nk0, nnr, nnc);
        }
        body(s, cur, cj0, ck0, cnr, cnc);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        cj0 = nj0; ck0 = nk0; cnr = nnr; cnc = nnc;
    }

    // epilogue: lane holds rows (coefficients) 16 mt + 4 (lane/16) + r of voxel column 16 nt + lane % 16
    double c2 = 0.0;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int lv = nt * 16 + (lane & 15);
        const int vy = by * 8 + (lv >> 3), vz = bz * 8 + (lv & 7);
        if (ix < nx && vy < ny && vz < nz) {
            const long long base = (((long long)ix * ny + vy) * nz + vz) * C;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = mt * 16 + 4 * (lane >> 4) + r;
                    if (i < C) {
                        float val = acc[mt][nt][r];
                        if (c) {
                            float cv = c[base + i];
                            val += beta * cv;
                            c2 += (double)cv * (double)cv;
                        }
                        g[base + i] = val;
                    }
                }
            }
        }
    }
    if (partials) {
        double tot = block_sum(c2, ws);
        if (tid == 0) partials[bid] = tot;
    }
}

// ---------------------------------------------------------------------------
// backproject, paired by point inversion and with LDS-staged residual windows
// (trilinear model, centred detector, even nx, eight unique segments).  Block
// as in k_backproject_inv: waves 0, 1 own two lower-half x-slices, waves 2, 3
// their inverses; per pair of projections (s0, s0 + 1) the lower group
// enumerates s0 and the upper group s0 + 1.  Each group stages, for its
// projection, the residual window of its own 2 x 8 x 8 voxels and the
// point-reflected window (row nj-1-j, column nk-1-k at the position of
// (j, k)), so a ray's own and mirrored reads use the same offset in two LDS
// buffers.  The copies for the next pair are issued before this pair's
// MFMAs.  Two block barriers per pair: windows staged, Q handed over.
// ---------------------------------------------------------------------------
template <int UP, int MT, bool BF16, bool JOS>
__global__ __launch_bounds__(256) void k_backproject_pw(const float *__restrict__ yf,
                                                        const ProjFrame *__restrict__ frames,
                                                        const float *__restrict__ Bu, const s4 *__restrict__ BuT16,
                                                        int S, int nx, int ny, int nz, int nj, int nk, int C, int Cp,
                                                        float step, float *__restrict__ g, float beta,
                                                        const float *__restrict__ c, double *__restrict__ partials,
                                                        int WR, int WC)
{
    constexpr int Q = UP / 4;
    constexpr int QS = 64 * (UP + 1);
    extern __shared__ f4 wins[];     // [group][own, reflected][WR][WC][Q]
    __shared__ float Qs[4][QS];      // each wave's own Q
    __shared__ float Qx[4][QS];      // Q handed over by the partner wave
    __shared__ double ws[4];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool upper = wave >= 2;
    const int grp = upper ? 1 : 0;
    const int nxh = nx >> 1;
    const int nbx = (nxh + 1) / 2, nby = (ny + 7) / 8;
    const int bid = xcd_block(blockIdx.x, gridDim.x);
    const int bx = bid % nbx, by = (bid / nbx) % nby, bz = bid / (nbx * nby);
    const int px = bx * 2 + (wave & 1), py = by * 8 + (lane >> 3), pz = bz * 8 + (lane & 7);
    const bool valid = px < nxh && py < ny && pz < nz;
    const int ix = upper ? nx - 1 - px : px, iy = upper ? ny - 1 - py : py, iz = upper ? nz - 1 - pz : pz;
    const double xv[3] = {ix - 0.5 * (nx - 1), iy - 0.5 * (ny - 1), iz - 0.5 * (nz - 1)};
    const double inv_step = 1.0 / (double)step;
    const float stepf = step, inv_stepf = (float)inv_step;
    const int WROW = WC * Q, WSZ = WR * WROW;
    f4 *win_own = wins + (2 * grp) * WSZ, *win_ref = wins + (2 * grp + 1) * WSZ;

    // window of this group's voxel box for projection s (its L1 reach lj, lk
    // around the detector positions, one more on each side for rounding)
    auto window = [&](int s, int &j0, int &k0, int &nr, int &nc) {
        const ProjFrame &f = frames[s];
        const double lo0[3] = {bx * 2 - 0.5 * (nx - 1), by * 8 - 0.5 * (ny - 1), bz * 8 - 0.5 * (nz - 1)};
        const double hi0[3] = {min(nxh, bx * 2 + 2) - 1 - 0.5 * (nx - 1), min(ny, by * 8 + 8) - 1 - 0.5 * (ny - 1),
                               min(nz, bz * 8 + 8) - 1 - 0.5 * (nz - 1)};
        double amin = 0.0, amax = 0.0, bmin = 0.0, bmax = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // the upper group's box is the point inverse of the lower group's
            const double lo = upper ? -hi0[a] : lo0[a], hi = upper ? -lo0[a] : hi0[a];
            const double ea = f.ej[a], ka = f.ek[a];
            amin += (ea >= 0.0 ? lo - f.o[a] : hi - f.o[a]) * ea;
            amax += (ea >= 0.0 ? hi - f.o[a] : lo - f.o[a]) * ea;
            bmin += (ka >= 0.0 ? lo - f.o[a] : hi - f.o[a]) * ka;
            bmax += (ka >= 0.0 ? hi - f.o[a] : lo - f.o[a]) * ka;
        }
        const double rj = JOS ? (double)f.jos_rj : f.lj, rk = JOS ? (double)f.jos_rk : f.lk;
        const int ja = max(0, (int)ceil(amin - rj) - 1), jb = min(nj - 1, (int)floor(amax + rj) + 1);
        const int ka0 = max(0, (int)ceil(bmin - rk) - 1), kb = min(nk - 1, (int)floor(bmax + rk) + 1);
        j0 = __builtin_amdgcn_readfirstlane(ja);
        k0 = __builtin_amdgcn_readfirstlane(ka0);
        nr = __builtin_amdgcn_readfirstlane(max(0, min(WR, jb - ja + 1)));
        nc = __builtin_amdgcn_readfirstlane(max(0, min(WC, kb - ka0 + 1)));
    };
    // asynchronous copies of the window and of its point reflection (rows spread
    // over the group's two waves)
    auto stage = [&](int s, int j0, int k0, int nr, int nc) {
        const f4 *ys = reinterpret_cast<const f4 *>(yf) + (long long)s * nj * nk * Q;
        const int rowf4 = nc * Q;
        for (int r = wave & 1; r < nr; r += 2) {
            for (int l0 = 0; l0 < rowf4; l0 += 64) {
                const int l = l0 + lane;
                if (l < rowf4) {
                    const int cc = l / Q, q = l - cc * Q;
                    const f4 *so = ys + ((long long)(j0 + r) * nk + k0) * Q + l;
                    const f4 *sr = ys + ((long long)(nj - 1 - j0 - r) * nk + (nk - 1 - k0 - cc)) * Q + q;
                    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)so,
                                                     (__attribute__((address_space(3))) void *)(win_own + r * WROW + l0),
                                                     16, 0, 0);
                    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)sr,
                                                     (__attribute__((address_space(3))) void *)(win_ref + r * WROW + l0),
                                                     16, 0, 0);
                }
            }
        }
    };

    f4 acc[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};

    struct BOps {
        s4 b16[BF16 ? MT : 1];
        float f[BF16 ? 1 : UP / 4][MT];
    };
    auto load_ops = [&](int s, BOps &o) {
        if constexpr (BF16) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                o.b16[mt] = BuT16[((long long)s * Cp + mt * 16 + (lane & 15)) * 4 + (lane >> 4)];
        } else {
            const float *Bs = Bu + (long long)s * UP * Cp;
#pragma unroll
            for (int ks = 0; ks < UP / 4; ++ks)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) o.f[ks][mt] = Bs[(ks * 4 + (lane >> 4)) * Cp + mt * 16 + (lane & 15)];
        }
    };
    auto contract = [&](const BOps &o, const float *Qt) {
        if constexpr (BF16) {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const float *qv = Qt + (nt * 16 + (lane & 15)) * (UP + 1);
                const int u0 = 4 * (lane >> 4);
                s4 bv;
                bv.x = u0 + 0 < UP ? f2bf(qv[min(u0 + 0, UP - 1)]) : (short)0;
                bv.y = u0 + 1 < UP ? f2bf(qv[min(u0 + 1, UP - 1)]) : (short)0;
                bv.z = u0 + 2 < UP ? f2bf(qv[min(u0 + 2, UP - 1)]) : (short)0;
                bv.w = u0 + 3 < UP ? f2bf(qv[min(u0 + 3, UP - 1)]) : (short)0;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma16x16x16bf16(o.b16[mt], bv, acc[mt][nt]);
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < UP / 4; ++ks) {
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const float bv = qw_at<UP>(Qt, nt, ks, lane);
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) acc[mt][nt] = mfma16x16x4(o.f[ks][mt], bv, acc[mt][nt]);
                }
            }
        }
    };

    int wj0 = 0, wk0 = 0, wnr = 0, wnc = 0;  // this group's window of the current pair
    if (grp < S) {
        window(grp, wj0, wk0, wnr, wnc);
        stage(grp, wj0, wk0, wnr, wnc);
    }
    for (int s0 = 0; s0 < S; s0 += 2) {
        const int s_own = s0 + grp, s_oth = s0 + 1 - grp;
        const bool has_own = s_own < S, has_oth = s_oth < S;
        BOps ops_own, ops_oth;
        load_ops(has_own ? s_own : s0, ops_own);
        load_ops(has_oth ? s_oth : s0, ops_oth);
        float q[UP], qm[UP];
#pragma unroll
        for (int u = 0; u < UP; ++u) q[u] = qm[u] = 0.0f;
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();  // this pair's windows are staged
        if (has_own && valid) {
            const ProjFrame &f = frames[s_own];
            if constexpr (JOS) {
                // Joseph's method: the rays whose cut with the voxel's layer lies
                // within one voxel in-plane, weight (1 - |Delta_B|)(1 - |Delta_C|) /
                // |d_A|.  The inverse voxel's cut of the reflected ray is the negated
                // cut point, so the same weight serves both voxels of the pair.
                const double w0 = xv[0] - f.o[0], w1 = xv[1] - f.o[1], w2 = xv[2] - f.o[2];
                const double a = w0 * f.ej[0] + w1 * f.ej[1] + w2 * f.ej[2];
                const double bb = w0 * f.ek[0] + w1 * f.ek[1] + w2 * f.ek[2];
                const double af = floor(a), bf = floor(bb);
                const int ai = (int)af, bi = (int)bf;
                const float ar = (float)(a - af), br = (float)(bb - bf);
                const float gjB = f.jos_gj[0], gjC = f.jos_gj[1], gkB = f.jos_gk[0], gkC = f.jos_gk[1];
                const int jlo = max(wj0, ai + (int)ceilf(ar - f.jos_rj));
                const int jhi = min(wj0 + wnr - 1, ai + (int)floorf(ar + f.jos_rj));
                for (int j = jlo; j <= jhi; ++j) {
                    const float dj = (float)(j - ai) - ar;
                    const float eB = dj * gjB, eC = dj * gjC;
                    // dk range with |dk gk + e| < 1 on both in-plane axes (a flat
                    // axis gives all dk or none; the other one is never flat)
                    const float xB1 = (-1.0f - eB) * f.jos_igk[0], xB2 = (1.0f - eB) * f.jos_igk[0];
                    const float xC1 = (-1.0f - eC) * f.jos_igk[1], xC2 = (1.0f - eC) * f.jos_igk[1];
                    const float lo = fmaxf(fminf(xB1, xB2), fminf(xC1, xC2));
                    const float hi = fminf(fmaxf(xB1, xB2), fmaxf(xC1, xC2));
                    if (!(lo < hi)) continue;
                    const int klo = max(wk0, bi + (int)ceilf(br + lo - 1e-4f));
                    const int khi = min(wk0 + wnc - 1, bi + (int)floorf(br + hi + 1e-4f));
                    const int rowoff = (j - wj0) * WROW - wk0 * Q;
                    const f4 *wo = win_own + rowoff, *wr = win_ref + rowoff;
                    for (int k = klo; k <= khi; ++k) {
                        f4 yv[Q], ym[Q];
#pragma unroll
                        for (int u4 = 0; u4 < Q; ++u4) {
                            yv[u4] = wo[k * Q + u4];
                            ym[u4] = wr[k * Q + u4];
                        }
                        const float dk = (float)(k - bi) - br;
                        const float wB = fmaxf(0.0f, 1.0f - fabsf(fmaf(dk, gkB, eB)));
                        const float wC = fmaxf(0.0f, 1.0f - fabsf(fmaf(dk, gkC, eC)));
                        const float wt = wB * wC * f.jos_w;
#pragma unroll
                        for (int u4 = 0; u4 < UP; u4 += 4) {
                            q[u4 + 0] = fmaf(wt, yv[u4 / 4].x, q[u4 + 0]);
                            q[u4 + 1] = fmaf(wt, yv[u4 / 4].y, q[u4 + 1]);
                            q[u4 + 2] = fmaf(wt, yv[u4 / 4].z, q[u4 + 2]);
                            q[u4 + 3] = fmaf(wt, yv[u4 / 4].w, q[u4 + 3]);
                            qm[u4 + 0] = fmaf(wt, ym[u4 / 4].x, qm[u4 + 0]);
                            qm[u4 + 1] = fmaf(wt, ym[u4 / 4].y, qm[u4 + 1]);
                            qm[u4 + 2] = fmaf(wt, ym[u4 / 4].z, qm[u4 + 2]);
                            qm[u4 + 3] = fmaf(wt, ym[u4 / 4].w, qm[u4 + 3]);
                        }
                    }
                }
            } else {
                const double w0 = xv[0] - f.o[0], w1 = xv[1] - f.o[1], w2 = xv[2] - f.o[2];
                const double a = w0 * f.ej[0] + w1 * f.ej[1] + w2 * f.ej[2];
                const double bb = w0 * f.ek[0] + w1 * f.ek[1] + w2 * f.ek[2];
                const double ts = (w0 * f.d[0] + w1 * f.d[1] + w2 * f.d[2]) * inv_step;
                const double af = floor(a), bf = floor(bb), tf = floor(ts);
                const int ai = (int)af, bi = (int)bf;
                const float ar = (float)(a - af), br = (float)(bb - bf), tr = (float)(ts - tf);
                const float hinv[3] = {fabsf(f.inv_df[0]), fabsf(f.inv_df[1]), fabsf(f.inv_df[2])};
                float nhv[3] = {-hinv[0], -hinv[1], -hinv[2]};
                asm volatile("" : "+v"(nhv[0]), "+v"(nhv[1]), "+v"(nhv[2]));
                float dfv[3] = {f.df[0], f.df[1], f.df[2]};
                asm volatile("" : "+v"(dfv[0]), "+v"(dfv[1]), "+v"(dfv[2]));
                const float ljf = (float)f.lj;
                const int jlo = max(wj0, ai + (int)ceilf(ar - ljf));
                const int jhi = min(wj0 + wnr - 1, ai + (int)floorf(ar + ljf));
                const float cu[3] = {f.hull[1] + (br + 1e-4f), f.hull[3] + (br + 1e-4f), f.hull[5] + (br + 1e-4f)};
                const float cl[3] = {f.hull[7] + (br - 1e-4f), f.hull[9] + (br - 1e-4f), f.hull[11] + (br - 1e-4f)};
                for (int j = jlo; j <= jhi; ++j) {
                    const float dj = (float)(j - ai) - ar;
                    const float zmax = fminf(fminf(fmaf(f.hull[0], dj, cu[0]), fmaf(f.hull[2], dj, cu[1])),
                                             fmaf(f.hull[4], dj, cu[2]));
                    const float zmin = fmaxf(fmaxf(fmaf(f.hull[6], dj, cl[0]), fmaf(f.hull[8], dj, cl[1])),
                                             fmaf(f.hull[10], dj, cl[2]));
                    const int klo = max(wk0, bi + (int)ceilf(zmin));
                    const int khi = min(wk0 + wnc - 1, bi + (int)floorf(zmax));
                    const float pj0 = dj * f.ejf[0], pj1 = dj * f.ejf[1], pj2 = dj * f.ejf[2];
                    const int rowoff = (j - wj0) * WROW - wk0 * Q;
                    const f4 *wo = win_own + rowoff, *wr = win_ref + rowoff;
                    float dk = (float)(klo - bi) - br;
                    for (int k = klo; k <= khi; ++k, dk += 1.0f) {
                        f4 yv[Q], ym[Q];
#pragma unroll
                        for (int u4 = 0; u4 < Q; ++u4) {
                            yv[u4] = wo[k * Q + u4];
                            ym[u4] = wr[k * Q + u4];
                        }
                        const float P[3] = {fmaf(dk, f.ekf[0], pj0), fmaf(dk, f.ekf[1], pj1), fmaf(dk, f.ekf[2], pj2)};
                        float tlo = fmaf(-P[0], f.inv_df[0], nhv[0]), thi = fmaf(-P[0], f.inv_df[0], hinv[0]);
#pragma unroll
                        for (int m = 1; m < 3; ++m) {
                            tlo = fmaxf(tlo, fmaf(-P[m], f.inv_df[m], nhv[m]));
                            thi = fminf(thi, fmaf(-P[m], f.inv_df[m], hinv[m]));
                        }
                        float wsum = 0.0f;
                        const float m0 = ceilf(fmaf(tlo, inv_stepf, tr)), m1 = floorf(fmaf(thi, inv_stepf, tr));
                        const float tend = (m1 - tr + 0.5f) * stepf;
                        for (float tau = (m0 - tr) * stepf; tau < tend; tau += stepf) {
                            const float wx = 1.0f - fabsf(fmaf(tau, dfv[0], P[0]));
                            const float wy = 1.0f - fabsf(fmaf(tau, dfv[1], P[1]));
                            const float wz = 1.0f - fabsf(fmaf(tau, dfv[2], P[2]));
                            wsum = fmaf(wx * wy, wz, wsum);
                        }
#pragma unroll
                        for (int u4 = 0; u4 < UP; u4 += 4) {
                            q[u4 + 0] = fmaf(wsum, yv[u4 / 4].x, q[u4 + 0]);
                            q[u4 + 1] = fmaf(wsum, yv[u4 / 4].y, q[u4 + 1]);
                            q[u4 + 2] = fmaf(wsum, yv[u4 / 4].z, q[u4 + 2]);
                            q[u4 + 3] = fmaf(wsum, yv[u4 / 4].w, q[u4 + 3]);
                            qm[u4 + 0] = fmaf(wsum, ym[u4 / 4].x, qm[u4 + 0]);
                            qm[u4 + 1] = fmaf(wsum, ym[u4 / 4].y, qm[u4 + 1]);
                            qm[u4 + 2] = fmaf(wsum, ym[u4 / 4].z, qm[u4 + 2]);
                            qm[u4 + 3] = fmaf(wsum, ym[u4 / 4].w, qm[u4 + 3]);
                        }
                    }
                }
            }
        }
        float *Qown = Qs[wave];
        float *Qout = Qx[wave ^ 2];
#pragma unroll
        for (int u = 0; u < UP; ++u) {
            Qown[lane * (UP + 1) + u] = q[u];
            Qout[lane * (UP + 1) + u] = qm[u];
        }
        __syncthreads();  // the partner's Q is complete; the windows are free
        // copies for the next pair run during this pair's MFMAs
        const int s_next = s0 + 2 + grp;
        if (s_next < S) {
            window(s_next, wj0, wk0, wnr, wnc);
            stage(s_next, wj0, wk0, wnr, wnc);
        }
        if (has_own) contract(ops_own, Qown);
        if (has_oth) contract(ops_oth, Qx[wave]);
    }

    double c2 = 0.0;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int lv = nt * 16 + (lane & 15);
        const int qy = by * 8 + (lv >> 3), qz = bz * 8 + (lv & 7);
        if (px < nxh && qy < ny && qz < nz) {
            const int vx = ix, vy = upper ? ny - 1 - qy : qy, vz = upper ? nz - 1 - qz : qz;
            const long long base = (((long long)vx * ny + vy) * nz + vz) * C;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = mt * 16 + 4 * (lane >> 4) + r;
                    if (i < C) {
                        float val = acc[mt][nt][r];
                        if (c) {
                            float cv = c[base + i];
                            val += beta * cv;
                            c2 += (double)cv * (double)cv;
                        }
                        g[base + i] = val;
                    }
                }
            }
        }
    }
    if (partials) {
        double tot = block_sum(c2, ws);
        if (tid == 0) partials[bid] = tot;
    }
}

// Window extent (rows, columns) of a voxel box with centre spans (sx, sy, sz)
// over the projections: span . |e| + 2 l + 3 (L1 reach on both sides and the
// rounding margins); 0 if some projection exceeds lim.
static void window_extent(const std::vector<ProjFrame> &frames, double sx, double sy, double sz, bool jos, int &wr,
                          int &wc)
{
    wr = wc = 0;
    for (const ProjFrame &f : frames) {
        // reach of one voxel's rays: the L1 radius of the trilinear support, or
        // the parallelogram of Joseph cuts within one voxel
        const double rj = jos ? (double)f.jos_rj : f.lj, rk = jos ? (double)f.jos_rk : f.lk;
        const double sj = sx * fabs(f.ej[0]) + sy * fabs(f.ej[1]) + sz * fabs(f.ej[2]) + 2 * rj;
        const double sk = sx * fabs(f.ek[0]) + sy * fabs(f.ek[1]) + sz * fabs(f.ek[2]) + 2 * rk;
        wr = std::max(wr, (int)floor(sj) + 3);
        wc = std::max(wc, (int)floor(sk) + 3);
    }
}

// Paired + windowed adjoint: four windows of wr x wc rays x 8 floats beside
// 18 KiB of Q tiles must leave three blocks per CU (<= 52 KiB per block).
int backproject_pw_lds(const std::vector<ProjFrame> &frames, int up, bool jos, int &wr, int &wc)
{
    window_extent(frames, 1.0, 7.0, 7.0, jos, wr, wc);
    const int bytes = 4 * wr * wc * up * 4;
    return bytes + 2 * 4 * 64 * (up + 1) * 4 <= 52 * 1024 ? bytes : 0;
}

// Largest detector window of a 4 x 8 x 8 brick over the projections: rows
// <= 3|e_jx| + 7|e_jy| + 7|e_jz| + 2 l_j + 3 (the voxel-centre span, the L1 reach
// on both sides, and the rounding margins), columns likewise with e_k.
bool backproject_window_fits(const std::vector<ProjFrame> &frames)
{
    for (const ProjFrame &f : frames) {
        const double sj = 3 * fabs(f.ej[0]) + 7 * fabs(f.ej[1]) + 7 * fabs(f.ej[2]) + 2 * f.lj;
        const double sk = 3 * fabs(f.ek[0]) + 7 * fabs(f.ek[1]) + 7 * fabs(f.ek[2]) + 2 * f.lk;
        if (floor(sj) + 3 > kWinMax || floor(sk) + 3 > kWinMax) return false;
    }
    return true;
}

// Pairing pays with four unique segments (C2-like workloads: the adjoint
// 4.21 -> 3.21 ms at 100^3 / 240 projections).  With eight, its own and
// mirrored residual loads and accumulators raise the register count from 78
// to 102 (three waves per SIMD instead of four) and the kernel, then bound by
// load latency rather than by VALU issue, measured 10% slower than the
// unpaired one (5% of it the per-pair barrier), so it is not used there.
static bool use_inv_pair(const Dims &d) { return d.inv_pair && d.Up == 4; }
static bool use_window(const Dims &d) { return d.win_ok && !d.joseph && d.Up == 8; }
static bool use_pw(const Dims &d) { return (d.joseph ? d.pwj_lds : d.pw_lds) > 0 && d.inv_pair && d.Up == 8; }
static int backproject_inv_blocks(const Dims &d) { return ((d.nx / 2 + 1) / 2) * ((d.ny + 7) / 8) * ((d.nz + 7) / 8); }

int backproject_blocks(const Dims &d)
{
    return use_inv_pair(d) || use_pw(d) ? backproject_inv_blocks(d) : ((d.nx + 3) / 4) * ((d.ny + 7) / 8) * ((d.nz + 7) / 8);
}
int backproject_blocks_max(const Dims &d) { return ((d.nx + 3) / 4) * ((d.ny + 7) / 8) * ((d.nz + 7) / 8); }

template <int UP, int MT>
static hipError_t bp_t(const Dims &d, const ProjFrame *frames, const float *yf, const float *Bu, const uint16_t *BuT16,
                       int bf16, float *g, float beta, const float *c, double *partials, hipStream_t st)
{
    const s4 *bt = reinterpret_cast<const s4 *>(BuT16);
    const dim3 grid(backproject_blocks(d)), block(256);
    if constexpr (UP == 4) {
        if (use_inv_pair(d)) {
            if (bf16 && d.joseph)
                hipLaunchKernelGGL((k_backproject_inv<UP, MT, true, true>), grid, block, 0, st, yf, frames, Bu, bt,
                                   d.S, d.nx, d.ny, d.nz, d.nj, d.nk, d.C, d.Cp, d.step, g, beta, c, partials);
            else if (bf16)
                hipLaunchKernelGGL((k_backproject_inv<UP, MT, true, false>), grid, block, 0, st, yf, frames, Bu, bt,
                                   d.S, d.nx, d.ny, d.nz, d.nj, d.nk, d.C, d.Cp, d.step, g, beta, c, partials);
            else if (d.joseph)
                hipLaunchKernelGGL((k_backproject_inv<UP, MT, false, true>), grid, block, 0, st, yf, frames, Bu, bt,
                                   d.S, d.nx, d.ny, d.nz, d.nj, d.nk, d.C, d.Cp, d.step, g, beta, c, partials);
            else
                hipLaunchKernelGGL((k_backproject_inv<UP, MT, false, false>), grid, block, 0, st, yf, frames, Bu, bt,
                                   d.S, d.nx, d.ny, d.nz, d.nj, d.nk, d.C, d.Cp, d.step, g, beta, c, partials);
            return hipGetLastError();
        }
    }
    if constexpr (UP == 8) {
        if (use_pw(d)) {
            // residual windows sized for the model's reach
            const int lds = d.joseph ? d.pwj_lds : d.pw_lds;
            const int wr = d.joseph ? d.pwj_wr : d.pw_wr, wc = d.joseph ? d.pwj_wc : d.pw_wc;
            if (bf16 && d.joseph)
                hipLaunchKernelGGL((k_backproject_pw<UP, MT, true, true>), grid, block, lds, st, yf, frames, Bu, bt,
                                   d.S, d.nx, d.ny, d.nz, d.nj, d.nk, d.C, d.Cp, d.step, g, beta, c, partials, wr, wc);
            else if (bf16)
                hipLaunchKernelGGL((k_backproject_pw<UP, MT, true, false>), grid, block, lds, st, yf, frames, Bu, bt,
                                   d.S, d.nx, d.ny, d.nz, d.nj, d.nk, d.C, d.Cp, d.step, g, beta, c, partials, wr, wc);
            else if (d.joseph)
                hipLaunchKernelGGL((k_backproject_pw<UP, MT, false, true>), grid, block, lds, st, yf, frames, Bu, bt,
                                   d.S, d.nx, d.ny, d.nz, d.nj, d.nk, d.C, d.Cp, d.step, g, beta, c, partials, wr, wc);
            else
                hipLaunchKernelGGL((k_backproject_pw<UP, MT, false, false>), grid, block, lds, st, yf, frames, Bu, bt,
                                   d.S, d.nx, d.ny, d.nz, d.nj, d.nk, d.C, d.Cp, d.step, g, beta, c, partials, wr, wc);
            return hipGetLastError();
        }
        if (use_window(d)) {
            if (bf16)
                hipLaunchKernelGGL((k_backproject_win<UP, MT, true>), grid, block, 0, st, yf, frames, Bu, bt, d.S,
                                   d.nx, d.ny, d.nz, d.nj, d.nk, d.C, d.Cp, d.step, g, beta, c, partials);
            else
                hipLaunchKernelGGL((k_backproject_win<UP, MT, false>), grid, block, 0, st, yf, frames, Bu, bt, d.S,
                                   d.nx, d.ny, d.nz, d.nj, d.nk, d.C, d.Cp, d.step, g, beta, c, partials);
            return hipGetLastError();
        }
    }
    if (bf16 && d.joseph)
        hipLaunchKernelGGL((k_backproject<UP, MT, true, true>), grid, block, 0, st, yf, frames, Bu, bt, d.S, d.nx,
                           d.ny, d.nz, d.nj, d.nk, d.C, d.Cp, d.step, g, beta, c, partials);
    else if (bf16)
        hipLaunchKernelGGL((k_backproject<UP, MT, true, false>), grid, block, 0, st, yf, frames, Bu, bt, d.S, d.nx,
                           d.ny, d.nz, d.nj, d.nk, d.C, d.Cp, d.step, g, beta, c, partials);
    else if (d.joseph)
        hipLaunchKernelGGL((k_backproject<UP, MT, false, true>), grid, block, 0, st, yf, frames, Bu, bt, d.S, d.nx,
                           d.ny, d.nz, d.nj, d.nk, d.C, d.Cp, d.step, g, beta, c, partials);
    else
        hipLaunchKernelGGL((k_backproject<UP, MT, false, false>), grid, block, 0, st, yf, frames, Bu, bt, d.S, d.nx,
                           d.ny, d.nz, d.nj, d.nk, d.C, d.Cp, d.step, g, beta, c, partials);
    return hipGetLastError();
}

template <int UP>
static hipError_t bp_mt(const Dims &d, const ProjFrame *frames, const float *yf, const float *Bu,
                        const uint16_t *BuT16, int bf16, float *g, float beta, const float *c, double *partials,
                        hipStream_t st)
{
    switch (d.Cp / 16) {
    case 1: return bp_t<UP, 1>(d, frames, yf, Bu, BuT16, bf16, g, beta, c, partials, st);
    case 2: return bp_t<UP, 2>(d, frames, yf, Bu, BuT16, bf16, g, beta, c, partials, st);
    case 3: return bp_t<UP, 3>(d, frames, yf, Bu, BuT16, bf16, g, beta, c, partials, st);
    case 4: return bp_t<UP, 4>(d, frames, yf, Bu, BuT16, bf16, g, beta, c, partials, st);
    case 5: return bp_t<UP, 5>(d, frames, yf, Bu, BuT16, bf16, g, beta, c, partials, st);
    case 6: return bp_t<UP, 6>(d, frames, yf, Bu, BuT16, bf16, g, beta, c, partials, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_backproject(const Dims &d, const ProjFrame *frames, const float *yf, const float *Bu,
                              const uint16_t *BuT16, int bf16, float *g, float beta, const float *c, double *partials,
                              hipStream_t st)
{
    switch (d.Up) {
    case 4: return bp_mt<4>(d, frames, yf, Bu, BuT16, bf16, g, beta, c, partials, st);
    case 8: return bp_mt<8>(d, frames, yf, Bu, BuT16, bf16, g, beta, c, partials, st);
    case 16: return bp_mt<16>(d, frames, yf, Bu, BuT16, bf16, g, beta, c, partials, st);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// out[0] (+)= scale * sum(partials[0..n))
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sum_partials(const double *__restrict__ partials, int n, double *out,
                                                      double scale, int accumulate)
{
    __shared__ double ws[4];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) v += partials[i];
    double tot = block_sum(v, ws);
    if (threadIdx.x == 0) out[0] = (accumulate ? out[0] : 0.0) + scale * tot;
}

hipError_t launch_sum_partials(const double *partials, int n, double *out, double scale, int accumulate,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, partials, n, out, scale, accumulate);
    return hipGetLastError();
}

}  // namespace tt
