// Per-voxel quantities derived from reconstructed SH coefficients (the
// paper's section on deriving standard quantities from the output):
//   mean       <f> = c_0 Y_00
//   variance   <(f - <f>)^2> = (1 / 4 pi) sum_{i >= 1} c_i^2   (Parseval)
//   rel. anisotropy  sqrt(variance) / mean
//   M_ab       <q_a q_b f>, a linear map of the l = 0 and l = 2 coefficients
//   eigenvalues (descending) and unit eigenvectors of M (cyclic Jacobi, fp64),
//   each eigenvector with its largest-magnitude component positive
//   FA         from the eigenvalues
// <g> is the average over the unit sphere.  HBM-bound: each voxel reads C
// floats and writes kPropFields floats.  One wave per block handles 64 voxels:
// the coefficient block and the result block both pass through LDS so that
// every global access is a contiguous float4 stream.
#include "tt_device.h"
#include "tt_internal.h"

namespace tt {

typedef float f4 __attribute__((ext_vector_type(4)));

struct PropTable {
    double m[6][6];  // M_e = sum_k m[e][k] c_k for e in (xx, yy, zz, xy, xz, yz)
};

__device__ __forceinline__ void jacobi_rotate(double a[3][3], double v[3][3], int p, int q)
{
    const double apq = a[p][q];
    if (apq == 0.0) return;
    const double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
    const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
    const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
    // A <- J^T A J with J the rotation in the (p, q) plane
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double arp = a[r][p], arq = a[r][q];
        a[r][p] = c * arp - s * arq;
        a[r][q] = s * arp + c * arq;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double apr = a[p][r], aqr = a[q][r];
        a[p][r] = c * apr - s * aqr;
        a[q][r] = s * apr + c * aqr;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double vrp = v[r][p], vrq = v[r][q];
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
        const double c0 = cv[0];
        double ss = 0.0;
        for (int i = 1; i < C; ++i) ss += (double)cv[i] * (double)cv[i];
        const double kInv4Pi = 0.25 / M_PI;
        const double mean = c0 * sqrt(kInv4Pi), var = ss * kInv4Pi;
        double m6[6];
        const int kc = C < 6 ? C : 6;
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            double acc = 0.0;
            for (int k = 0; k < kc; ++k) acc += tab.m[e][k] * (double)cv[k];
            m6[e] = acc;
        }
        double a[3][3] = {{m6[0], m6[3], m6[4]}, {m6[3], m6[1], m6[5]}, {m6[4], m6[5], m6[2]}};
        double vv[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        for (int sweep = 0; sweep < 6; ++sweep) {
            jacobi_rotate(a, vv, 0, 1);
            jacobi_rotate(a, vv, 0, 2);
            jacobi_rotate(a, vv, 1, 2);
        }
        double lam[3] = {a[0][0], a[1][1], a[2][2]};
        int ord[3] = {0, 1, 2};
        // descending, stable
        if (lam[ord[1]] > lam[ord[0]]) { int t = ord[0]; ord[0] = ord[1]; ord[1] = t; }
        if (lam[ord[2]] > lam[ord[1]]) { int t = ord[1]; ord[1] = ord[2]; ord[2] = t; }
        if (lam[ord[1]] > lam[ord[0]]) { int t = ord[0]; ord[0] = ord[1]; ord[1] = t; }
        res[0] = (float)mean;
        res[1] = (float)var;
        res[2] = (float)(sqrt(fmax(var, 0.0)) / mean);
#pragma unroll
        for (int e = 0; e < 6; ++e) res[3 + e] = (float)m6[e];
        double l[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            l[r] = lam[ord[r]];
            res[9 + r] = (float)l[r];
            const int col = ord[r];
            double x = vv[0][col], y = vv[1][col], z = vv[2][col];
            const double nrm = 1.0 / sqrt(x * x + y * y + z * z);
            x *= nrm; y *= nrm; z *= nrm;
            // largest-magnitude component positive (first one on ties)
            double big = x;
            if (fabs(y) > fabs(big)) big = y;
            if (fabs(z) > fabs(big)) big = z;
            const double sg = big < 0.0 ? -1.0 : 1.0;
            res[12 + 3 * r + 0] = (float)(sg * x);
            res[12 + 3 * r + 1] = (float)(sg * y);
            res[12 + 3 * r + 2] = (float)(sg * z);
        }
        const double num = sqrt((l[0] - l[1]) * (l[0] - l[1]) + (l[1] - l[2]) * (l[1] - l[2]) + (l[2] - l[0]) * (l[2] - l[0]));
        const double den = sqrt(2.0 * (l[0] * l[0] + l[1] * l[1] + l[2] * l[2]));
        res[21] = den > 0.0 ? (float)(num / den) : 0.0f;
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
                for (int k = 0; k < 6; ++k) t.m[e][k] += w * qq[e] * y[k];
        }
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
