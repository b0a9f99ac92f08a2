// Per-voxel quantities derived from reconstructed SH coefficients (the
// paper's section on deriving standard quantities from the output):
//   mean       <f> = c_0 Y_00
//   variance   <(f - <f>)^2> = (1 / 4 pi) sum_{i >= 1} c_i^2   (Parseval)
//   rel. anisotropy  sqrt(variance) / mean
//   M_ab       <q_a q_b f>, a linear map of the l = 0 and l = 2 coefficients
//   eigenvalues (descending) and unit eigenvectors of M (cyclic Jacobi),
//   each eigenvector with its largest-magnitude component positive
//   FA         from the eigenvalues
// <g> is the average over the unit sphere.  Everything is evaluated in
// float32 (the inputs are float32; the sums have at most C terms and the
// Jacobi sweeps converge to float32 rounding).  Each voxel reads C floats and
// writes kPropFields floats.  One wave per block handles 64 voxels:
// the coefficient block and the result block both pass through LDS so that
// every global access is a contiguous float4 stream.
#include "tt_device.h"
#include "tt_internal.h"

namespace tt {

typedef float f4 __attribute__((ext_vector_type(4)));

struct PropTable {
    float m[6][6];  // M_e = sum_k m[e][k] c_k for e in (xx, yy, zz, xy, xz, yz)
};

// One Jacobi rotation in the (p, q) plane: A <- J^T A J, V <- V J, with the
// angle that zeroes a_pq (t = tan of the angle, the smaller root).  For a
// theta too large to square in float32 t is taken as 1 / (2 theta).
__device__ __forceinline__ void jacobi_rotate(float a[3][3], float v[3][3], int p, int q)
{
    const float apq = a[p][q];
    if (apq == 0.0f) return;
    const float theta = (a[q][q] - a[p][p]) / (2.0f * apq);
    const float at = fabsf(theta);
    const float t = (theta >= 0.0f ? 1.0f : -1.0f) / (at < 1e18f ? at + sqrtf(theta * theta + 1.0f) : 2.0f * at);
    const float c = 1.0f / sqrtf(t * t + 1.0f), s = t * c;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float arp = a[r][p], arq = a[r][q];
        a[r][p] = c * arp - s * arq;
        a[r][q] = s * arp + c * arq;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float apr = a[p][r], aqr = a[q][r];
        a[p][r] = c * apr - s * aqr;
        a[q][r] = s * apr + c * aqr;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float vrp = v[r][p], vrq = v[r][q];
        v[r][p] = c * vrp - s * vrq;
        v[r][q] = s * vrp + c * vrq;
    }
}

__global__ __launch_bounds__(64) void k_tensor_props(const float *__restrict__ c, long long nvox, int C, int ldc,
                                                     PropTable tab, float *__restrict__ out)
{
    extern __shared__ float sh[];  // max(64 * ldc, 64 * kPropFields) floats
    const int lane = threadIdx.x;
    const long long v0 = (long long)blockIdx.x * 64;
    const int nv = (int)min(64LL, nvox - v0);
    // coefficient block: nv * C contiguous floats, 16-byte aligned (64 C floats per block)
    const float *cb = c + v0 * C;
    const int nin = nv * C;
    if (nv == 64) {
        const f4 *cb4 = reinterpret_cast<const f4 *>(cb);
        for (int e4 = lane; e4 < nin / 4; e4 += 64) {
            const f4 x = cb4[e4];
            const int e = 4 * e4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int v = (e + q) / C, i = (e + q) - v * C;
                sh[v * ldc + i] = x[q];
            }
        }
    } else {
        for (int e = lane; e < nin; e += 64) {
            const int v = e / C, i = e - v * C;
            sh[v * ldc + i] = cb[e];
        }
    }
    __syncthreads();
    float res[kPropFields];
    if (lane < nv) {
        const float *cv = sh + lane * ldc;
        const float c0 = cv[0];
        float ss = 0.0f;
        for (int i = 1; i < C; ++i) ss = fmaf(cv[i], cv[i], ss);
        const float kInv4Pi = 0.0795774715459476679f, kInvSqrt4Pi = 0.282094791773878143f;  // 1/(4 pi), 1/sqrt(4 pi)
        const float mean = c0 * kInvSqrt4Pi, var = ss * kInv4Pi;
        float m6[6];
        const int kc = C < 6 ? C : 6;
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            float acc = 0.0f;
            for (int k = 0; k < kc; ++k) acc = fmaf(tab.m[e][k], cv[k], acc);
            m6[e] = acc;
        }
        float a[3][3] = {{m6[0], m6[3], m6[4]}, {m6[3], m6[1], m6[5]}, {m6[4], m6[5], m6[2]}};
        float vv[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        for (int sweep = 0; sweep < 5; ++sweep) {
            jacobi_rotate(a, vv, 0, 1);
            jacobi_rotate(a, vv, 0, 2);
            jacobi_rotate(a, vv, 1, 2);
        }
        const float lam[3] = {a[0][0], a[1][1], a[2][2]};
        int ord[3] = {0, 1, 2};
        // descending, stable
        if (lam[ord[1]] > lam[ord[0]]) { int t = ord[0]; ord[0] = ord[1]; ord[1] = t; }
        if (lam[ord[2]] > lam[ord[1]]) { int t = ord[1]; ord[1] = ord[2]; ord[2] = t; }
        if (lam[ord[1]] > lam[ord[0]]) { int t = ord[0]; ord[0] = ord[1]; ord[1] = t; }
        res[0] = mean;
        res[1] = var;
        res[2] = sqrtf(fmaxf(var, 0.0f)) / mean;
#pragma unroll
        for (int e = 0; e < 6; ++e) res[3 + e] = m6[e];
        float l[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            l[r] = lam[ord[r]];
            res[9 + r] = l[r];
            const int col = ord[r];
            float x = vv[0][col], y = vv[1][col], z = vv[2][col];
            const float nrm = 1.0f / sqrtf(x * x + y * y + z * z);
            x *= nrm; y *= nrm; z *= nrm;
            // largest-magnitude component positive (first one on ties)
            float big = x;
            if (fabsf(y) > fabsf(big)) big = y;
            if (fabsf(z) > fabsf(big)) big = z;
            const float sg = big < 0.0f ? -1.0f : 1.0f;
            res[12 + 3 * r + 0] = sg * x;
            res[12 + 3 * r + 1] = sg * y;
            res[12 + 3 * r + 2] = sg * z;
        }
        const float d01 = l[0] - l[1], d12 = l[1] - l[2], d20 = l[2] - l[0];
        const float num = sqrtf(d01 * d01 + d12 * d12 + d20 * d20);
        const float den = sqrtf(2.0f * (l[0] * l[0] + l[1] * l[1] + l[2] * l[2]));
        res[21] = den > 0.0f ? num / den : 0.0f;
    }
    __syncthreads();  // coefficient block consumed
    if (lane < nv) {
#pragma unroll
        for (int e = 0; e < kPropFields; ++e) sh[lane * kPropFields + e] = res[e];
    }
    __syncthreads();
    float *ob = out + v0 * kPropFields;
    const int nout = nv * kPropFields;
    if (nv == 64) {
        f4 *ob4 = reinterpret_cast<f4 *>(ob);
        for (int e4 = lane; e4 < nout / 4; e4 += 64)
            ob4[e4] = f4{sh[4 * e4], sh[4 * e4 + 1], sh[4 * e4 + 2], sh[4 * e4 + 3]};
    } else {
        for (int e = lane; e < nout; e += 64) ob[e] = sh[e];
    }
}

// <q_a q_b Y_k> for k < 6 by a product rule exact for degree-4 polynomials on
// the sphere (3 Gauss-Legendre nodes in cos(theta), 6 equispaced phi).
static PropTable prop_table()
{
    PropTable t{};
    double m[6][6] = {};
    const double xs[3] = {-std::sqrt(0.6), 0.0, std::sqrt(0.6)};
    const double ws[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
    double y[6 + 3];
    for (int it = 0; it < 3; ++it)
        for (int ip = 0; ip < 6; ++ip) {
            const double x = xs[it], st = std::sqrt(1.0 - x * x), phi = 2.0 * M_PI * ip / 6.0;
            const double q[3] = {st * std::cos(phi), st * std::sin(phi), x};
            const double w = ws[it] / 2.0 / 6.0;
            sh_eval_one(2, q, y);
            const double qq[6] = {q[0] * q[0], q[1] * q[1], q[2] * q[2], q[0] * q[1], q[0] * q[2], q[1] * q[2]};
            for (int e = 0; e < 6; ++e)
                for (int k = 0; k < 6; ++k) m[e][k] += w * qq[e] * y[k];
        }
    for (int e = 0; e < 6; ++e)
        for (int k = 0; k < 6; ++k) t.m[e][k] = (float)m[e][k];
    return t;
}

hipError_t launch_tensor_props(const float *c, long long nvox, int C, float *out, hipStream_t st)
{
    static const PropTable tab = prop_table();
    const int ldc = C | 1;  // odd row stride: conflict-free per-lane rows
    const size_t lds = sizeof(float) * (size_t)std::max(64 * ldc, 64 * kPropFields);
    const long long blocks = (nvox + 63) / 64;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_tensor_props, dim3((unsigned)blocks), dim3(64), lds, st, c, nvox, C, ldc, tab, out);
    return hipGetLastError();
}

}  // namespace tt
