// L-BFGS on the device (paper section 3.5, "Optimization"), in the Gram-matrix
// form of the two-loop recursion: the search direction d = -H g is a linear
// combination of the stored pairs (s_i, y_i) and the gradient g, and every
// inner product the two-loop recursion needs is an entry of the float64 Gram
// matrix of those vectors.  One iteration therefore makes two streaming
// passes over the history: the combination d = sum coef_a b_a (which also
// yields d . b_a), and the dot products of the new gradient with the history.
// Small float64 "planner" kernels (one thread) run the recursion on the Gram
// matrix, the exact line search and the pair update, so no host sync is
// needed inside an iteration.
#include "tt_device.h"
#include "tt_internal.h"
#include "tt_lbfgs.h"

#include <cmath>

namespace tt {

typedef float f4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kBlocks = 1024;  // fixed grid of the streaming kernels (deterministic partials)

struct VecList {
    const float *p[kMaxBasis + 1];
};

// Sum `nv` accumulators across the block; thread 0 writes partials[blockIdx*stride + a].
template <int NV>
__device__ void block_sums(double (&acc)[NV], int nv, double *partials, int stride)
{
    __shared__ double ws[4][NV];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < NV; ++a) {
        double v = acc[a];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if (lane == 0) ws[w][a] = v;
    }
    __syncthreads();
    if (threadIdx.x < nv) {
        double t = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += ws[i][threadIdx.x];
        partials[(long long)blockIdx.x * stride + threadIdx.x] = t;
    }
}

// d = sum_a coef[a] b_a over masked a;  partials: d . b_a (a < nb) and d . d (index kMaxBasis).
// One float per thread and step: every b_a value stays live until the dots
// are formed, and with float4 steps those registers held the kernel to two
// waves per SIMD and ~4.7 TB/s; scalar steps give four waves and ~6.5 TB/s.
__global__ __launch_bounds__(256) void k_combine(VecList b, int nb, const double *__restrict__ coef,
                                                 const int *__restrict__ mask, long long n, float *__restrict__ d,
                                                 double *__restrict__ partials)
{
    double acc[kMaxBasis + 1];
    float cf[kMaxBasis];
    bool mk[kMaxBasis];
#pragma unroll
    for (int a = 0; a <= kMaxBasis; ++a) acc[a] = 0.0;
#pragma unroll
    for (int a = 0; a < kMaxBasis; ++a) {
        mk[a] = a < nb && mask[a];
        cf[a] = mk[a] ? (float)coef[a] : 0.0f;
    }
    const long long stride = (long long)gridDim.x * 256;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += stride) {
        float bv[kMaxBasis];
        float dv = 0.0f;
#pragma unroll
        for (int a = 0; a < kMaxBasis; ++a) {
            bv[a] = mk[a] ? b.p[a][e] : 0.0f;
            dv = fmaf(cf[a], bv[a], dv);
        }
        d[e] = dv;
#pragma unroll
        for (int a = 0; a < kMaxBasis; ++a) acc[a] += (double)dv * (double)bv[a];
        acc[kMaxBasis] += (double)dv * (double)dv;
    }
    block_sums<kMaxBasis + 1>(acc, kMaxBasis + 1, partials, kMaxBasis + 1);
}

// partials: x . b_a for masked a < nb.  If ycand is set, also writes
// y[cand] = x - b[gold] (the new curvature vector, in the same pass).
__global__ __launch_bounds__(256) void k_multidot(const float *__restrict__ x, VecList b, int nb,
                                                  const int *__restrict__ mask, long long n,
                                                  double *__restrict__ partials, VecList ys,
                                                  const int *__restrict__ ist, int gold)
{
    double acc[kMaxBasis + 1];
    bool mk[kMaxBasis + 1];
#pragma unroll
    for (int a = 0; a <= kMaxBasis; ++a) {
        acc[a] = 0.0;
        mk[a] = a < nb && mask[a];
    }
    float *yc = ist ? const_cast<float *>(ys.p[ist[kCand]]) : nullptr;
    const float *go = ist ? b.p[gold] : nullptr;
    const long long n4 = n >> 2;
    const long long stride = (long long)gridDim.x * 256;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n4; e += stride) {
        const f4 xv = reinterpret_cast<const f4 *>(x)[e];
#pragma unroll
        for (int a = 0; a <= kMaxBasis; ++a)
            if (mk[a]) {
                const f4 bv = reinterpret_cast<const f4 *>(b.p[a])[e];
                acc[a] += (double)xv.x * bv.x + (double)xv.y * bv.y + (double)xv.z * bv.z + (double)xv.w * bv.w;
            }
        if (yc) reinterpret_cast<f4 *>(yc)[e] = xv - reinterpret_cast<const f4 *>(go)[e];
    }
    for (long long e = 4 * n4 + blockIdx.x * 256LL + threadIdx.x; e < n; e += stride) {
        const double xv = x[e];
#pragma unroll
        for (int a = 0; a <= kMaxBasis; ++a)
            if (mk[a]) acc[a] += xv * (double)b.p[a][e];
        if (yc) yc[e] = x[e] - go[e];
    }
    block_sums<kMaxBasis + 1>(acc, nb, partials, kMaxBasis + 1);
}

// out[a] = sum over blocks of partials[blk * stride + a], one block per a.
__global__ __launch_bounds__(256) void k_sum_columns(const double *__restrict__ partials, int nblk, int stride,
                                                     double *__restrict__ out)
{
    __shared__ double ws[4];
    double v = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) v += partials[(long long)i * stride + blockIdx.x];
    double t = block_sum(v, ws);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// sum of w q^2
__global__ __launch_bounds__(256) void k_wnorm2(const float *__restrict__ q, const float *__restrict__ w, long long n,
                                                double *__restrict__ partials)
{
    __shared__ double ws[4];
    double acc = 0.0;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
        double v = q[e];
        acc += (w ? (double)w[e] : 1.0) * v * v;
    }
    double t = block_sum(acc, ws);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// c += alpha d;  s[cand] = alpha d
__global__ __launch_bounds__(256) void k_update_c(float *__restrict__ c, const float *__restrict__ d, VecList s,
                                                  const double *__restrict__ st, const int *__restrict__ ist,
                                                  long long n)
{
    const float alpha = (float)st[kAlpha];
    float *sc = const_cast<float *>(s.p[ist[kCand]]);
    const long long n4 = n >> 2;
    const long long stride = (long long)gridDim.x * 256;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n4; e += stride) {
        const f4 ad = alpha * reinterpret_cast<const f4 *>(d)[e];
        reinterpret_cast<f4 *>(c)[e] += ad;
        reinterpret_cast<f4 *>(sc)[e] = ad;
    }
    for (long long e = 4 * n4 + blockIdx.x * 256LL + threadIdx.x; e < n; e += stride) {
        const float ad = alpha * d[e];
        c[e] += ad;
        sc[e] = ad;
    }
}

// y[cand] = g_new - g_old
__global__ __launch_bounds__(256) void k_make_y(VecList y, const int *__restrict__ ist, const float *__restrict__ gn,
                                                const float *__restrict__ go, long long n)
{
    float *yc = const_cast<float *>(y.p[ist[kCand]]);
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < n; e += (long long)gridDim.x * 256) yc[e] = gn[e] - go[e];
}

// r += alpha q;  yf = step * fold(2 w r);  partials: [blk][0] = sum w r^2, [blk][1] = sum r^2
template <int UP>
__global__ __launch_bounds__(256) void k_resid_update(float *__restrict__ r, const float *__restrict__ q,
                                                      const float *__restrict__ w, const double *__restrict__ st,
                                                      long long npix, int nseg, int U, float step,
                                                      float *__restrict__ yf, double *__restrict__ partials)
{
    const float alpha = q ? (float)st[kAlpha] : 0.0f;
    double acc[2] = {0.0, 0.0};
    for (long long px = blockIdx.x * 256LL + threadIdx.x; px < npix; px += (long long)gridDim.x * 256) {
        float f[UP];
#pragma unroll
        for (int u = 0; u < UP; ++u) f[u] = 0.0f;
#pragma unroll
        for (int u = 0; u < UP; ++u) {
            if (u < U) {
                for (int cseg = u; cseg < nseg; cseg += U) {
                    long long e = px * nseg + cseg;
                    float rv = r[e];
                    if (q) {
                        rv = fmaf(alpha, q[e], rv);
                        r[e] = rv;
                    }
                    float wv = w ? w[e] : 1.0f;
                    acc[0] += (double)wv * (double)rv * (double)rv;
                    acc[1] += (double)rv * (double)rv;
                    f[u] += 2.0f * wv * rv;
                }
            }
        }
        f4 *o = reinterpret_cast<f4 *>(yf + px * UP);
#pragma unroll
        for (int u4 = 0; u4 < UP; u4 += 4) o[u4 / 4] = f4{step * f[u4], step * f[u4 + 1], step * f[u4 + 2], step * f[u4 + 3]};
    }
    block_sums<2>(acc, 2, partials, 2);
}

// Same update for the common layout n_seg = 2 U = 2 UP (no padded unique
// segments): each pixel's n_seg values are UP/2 float4 per half, and the fold
// pairs segment u with u + U, in the same order as above.  Requires 16-byte
// aligned r, q, w.
template <int UP>
__global__ __launch_bounds__(256) void k_resid_update_v(float *__restrict__ r, const float *__restrict__ q,
                                                        const float *__restrict__ w, const double *__restrict__ st,
                                                        long long npix, float step, float *__restrict__ yf,
                                                        double *__restrict__ partials)
{
    constexpr int H = UP / 4;  // float4 per half pixel
    const float alpha = q ? (float)st[kAlpha] : 0.0f;
    double acc[2] = {0.0, 0.0};
    for (long long px = blockIdx.x * 256LL + threadIdx.x; px < npix; px += (long long)gridDim.x * 256) {
        f4 *rp = reinterpret_cast<f4 *>(r) + px * 2 * H;
        const f4 *qp = q ? reinterpret_cast<const f4 *>(q) + px * 2 * H : nullptr;
        const f4 *wp = w ? reinterpret_cast<const f4 *>(w) + px * 2 * H : nullptr;
        f4 fold[H];
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
#pragma unroll
            for (int i = 0; i < H; ++i) {
                f4 rv = rp[hh * H + i];
                if (qp) {
                    rv = f4{fmaf(alpha, qp[hh * H + i].x, rv.x), fmaf(alpha, qp[hh * H + i].y, rv.y),
                            fmaf(alpha, qp[hh * H + i].z, rv.z), fmaf(alpha, qp[hh * H + i].w, rv.w)};
                    rp[hh * H + i] = rv;
                }
                const f4 wv = wp ? wp[hh * H + i] : f4{1.f, 1.f, 1.f, 1.f};
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                    acc[0] += (double)wv[l] * (double)rv[l] * (double)rv[l];
                    acc[1] += (double)rv[l] * (double)rv[l];
                }
                const f4 t = 2.0f * wv * rv;
                fold[i] = hh == 0 ? t : fold[i] + t;
            }
        }
        f4 *o = reinterpret_cast<f4 *>(yf + px * UP);
#pragma unroll
        for (int i = 0; i < H; ++i) o[i] = step * fold[i];
    }
    block_sums<2>(acc, 2, partials, 2);
}

// ---------------------------------------------------------------------------
// Planner kernels (single thread, float64).
// Basis index: s slot i -> i, y slot i -> ns + i, gradient -> 2 ns  (ns = m + 1).
// ---------------------------------------------------------------------------
__device__ inline double &Gm(double *st, int a, int b) { return st[kGram + a * kMaxBasis + b]; }

__device__ void valid_list(const int *ist, int ns, int *idx, int &nidx)
{
    nidx = 0;
    for (int t = 0; t < ist[kCount]; ++t) {
        int i = ist[kOrder + t];
        idx[nidx++] = i;
        idx[nidx++] = ns + i;
    }
    idx[nidx++] = 2 * ns;
}

// The block stages the Gram matrix in LDS; thread 0 then runs the recursion
// (each step depends on the previous one) on LDS operands.
__global__ __launch_bounds__(64) void k_plan_direction(double *st, int *ist, int m)
{
    __shared__ double G[kMaxBasis * kMaxBasis];
    __shared__ double del[kMaxBasis];
    __shared__ int idx[kMaxBasis];
    for (int e = threadIdx.x; e < kMaxBasis * kMaxBasis; e += blockDim.x) G[e] = st[kGram + e];
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int ns = m + 1, nb = 2 * ns + 1, gi = 2 * ns;
    int nidx;
    valid_list(ist, ns, idx, nidx);
    for (int a = 0; a < nb; ++a) del[a] = 0.0;
    del[gi] = 1.0;
    const int cnt = ist[kCount];
    for (int t = cnt - 1; t >= 0; --t) {
        const int i = ist[kOrder + t];
        double v = 0.0;
        for (int q = 0; q < nidx; ++q) v += del[idx[q]] * G[i * kMaxBasis + idx[q]];
        const double al = st[kRho + i] * v;
        st[kAlphaTmp + i] = al;
        del[ns + i] -= al;
    }
    const double gamma = st[kGamma];
    for (int a = 0; a < nb; ++a) del[a] *= gamma;
    for (int t = 0; t < cnt; ++t) {
        const int i = ist[kOrder + t];
        double v = 0.0;
        for (int q = 0; q < nidx; ++q) v += del[idx[q]] * G[(ns + i) * kMaxBasis + idx[q]];
        const double be = st[kRho + i] * v;
        del[i] += st[kAlphaTmp + i] - be;
    }
    for (int a = 0; a < nb; ++a) {
        st[kCoef + a] = -del[a];
        ist[kMask + a] = 0;
    }
    for (int q = 0; q < nidx; ++q) ist[kMask + idx[q]] = 1;
    // candidate slot for the next pair: the first slot not in the ring
    int cand = 0;
    for (int i = 0; i < ns; ++i) {
        bool used = false;
        for (int t = 0; t < cnt; ++t) used |= ist[kOrder + t] == i;
        if (!used) {
            cand = i;
            break;
        }
    }
    ist[kCand] = cand;
}

// Bookkeeping for a step along a caller-supplied direction: combine mask =
// the valid history and the gradient, candidate slot = first free slot.
__global__ void k_plan_user_direction(double *st, int *ist, int m)
{
    const int ns = m + 1, nb = 2 * ns + 1;
    int idx[kMaxBasis];
    int nidx;
    valid_list(ist, ns, idx, nidx);
    for (int a = 0; a < nb; ++a) ist[kMask + a] = 0;
    for (int q = 0; q < nidx; ++q) ist[kMask + idx[q]] = 1;
    const int cnt = ist[kCount];
    int cand = 0;
    for (int i = 0; i < ns; ++i) {
        bool used = false;
        for (int t = 0; t < cnt; ++t) used |= ist[kOrder + t] == i;
        if (!used) {
            cand = i;
            break;
        }
    }
    ist[kCand] = cand;
}

__global__ void k_plan_alpha(double *st, int *ist, int m, double mu)
{
    const int ns = m + 1, gi = 2 * ns, nb = 2 * ns + 1;
    const double gd = st[kDotsD + gi], dd = st[kDotsD + kMaxBasis], qq = st[kQQ];
    const double denom = 2.0 * (qq + mu * dd);
    double alpha = (denom > 0.0 && isfinite(denom) && isfinite(gd)) ? -gd / denom : 0.0;
    st[kAlpha] = alpha;
    // multidot list: [s slots | y slots | g_old | g_new]; mask valid pairs, the candidate s, both gradients
    for (int a = 0; a < 2 * ns + 2; ++a) ist[kMask2 + a] = 0;
    for (int t = 0; t < ist[kCount]; ++t) {
        int i = ist[kOrder + t];
        ist[kMask2 + i] = 1;
        ist[kMask2 + ns + i] = 1;
    }
    ist[kMask2 + ist[kCand]] = 1;
    ist[kMask2 + 2 * ns] = 1;
    ist[kMask2 + 2 * ns + 1] = 1;
}

__global__ void k_plan_update(double *st, int *ist, int m, double mu)
{
    const int ns = m + 1, gi = 2 * ns, nb = 2 * ns + 1;
    const int cand = ist[kCand];
    const double a = st[kAlpha];
    const double *dd = st + kDotsD;  // d . b (old basis), dd[kMaxBasis] = d . d
    const double *dg = st + kDotsG;  // g_new . [s slots | y slots | g_old | g_new]
    const double gn_go = dg[2 * ns], gn_gn = dg[2 * ns + 1];
    const double sc_go = a * dd[gi], sc_sc = a * a * dd[kMaxBasis], sc_gn = dg[cand];
    const double yc_sc = sc_gn - sc_go;
    const double yc_yc = gn_gn - 2.0 * gn_go + Gm(st, gi, gi);
    const double yc_gn = gn_gn - gn_go;
    const double sy = yc_sc, ss = sc_sc, yy = yc_yc;
    // old valid pairs
    int cnt = ist[kCount];
    double sc_b[kMaxBasis], yc_b[kMaxBasis];
    for (int t = 0; t < cnt; ++t) {
        const int i = ist[kOrder + t];
        sc_b[i] = a * dd[i];
        sc_b[ns + i] = a * dd[ns + i];
        yc_b[i] = dg[i] - Gm(st, gi, i);
        yc_b[ns + i] = dg[ns + i] - Gm(st, gi, ns + i);
    }
    // g row against the old pairs
    for (int t = 0; t < cnt; ++t) {
        const int i = ist[kOrder + t];
        Gm(st, gi, i) = Gm(st, i, gi) = dg[i];
        Gm(st, gi, ns + i) = Gm(st, ns + i, gi) = dg[ns + i];
    }
    Gm(st, gi, gi) = gn_gn;
    const bool accept = isfinite(sy) && isfinite(ss) && isfinite(yy) && a != 0.0 && sy > 1e-12 * sqrt(ss * yy);
    if (accept) {
        if (cnt == m) {  // drop the oldest pair
            for (int t = 1; t < cnt; ++t) ist[kOrder + t - 1] = ist[kOrder + t];
            --cnt;
        }
        for (int t = 0; t < cnt; ++t) {
            const int i = ist[kOrder + t];
            Gm(st, cand, i) = Gm(st, i, cand) = sc_b[i];
            Gm(st, cand, ns + i) = Gm(st, ns + i, cand) = sc_b[ns + i];
            Gm(st, ns + cand, i) = Gm(st, i, ns + cand) = yc_b[i];
            Gm(st, ns + cand, ns + i) = Gm(st, ns + i, ns + cand) = yc_b[ns + i];
        }
        Gm(st, cand, cand) = ss;
        Gm(st, ns + cand, ns + cand) = yy;
        Gm(st, cand, ns + cand) = Gm(st, ns + cand, cand) = sy;
        Gm(st, gi, cand) = Gm(st, cand, gi) = sc_gn;
        Gm(st, gi, ns + cand) = Gm(st, ns + cand, gi) = yc_gn;
        ist[kOrder + cnt] = cand;
        ist[kCount] = cnt + 1;
        st[kRho + cand] = 1.0 / sy;
        st[kGamma] = sy / yy;
        ist[kAccepted] += 1;
    }
    st[kLoss] = st[kLossR] + mu * st[kCC];
    ist[kIter] += 1;
}

}  // namespace

// ---------------------------------------------------------------------------
// Host-side launchers used by tt_api.cpp
// ---------------------------------------------------------------------------
hipError_t lbfgs_plan_direction(double *st, int *ist, int m, hipStream_t s)
{
    hipLaunchKernelGGL(k_plan_direction, dim3(1), dim3(64), 0, s, st, ist, m);
    return hipGetLastError();
}

hipError_t lbfgs_plan_user_direction(double *st, int *ist, int m, hipStream_t s)
{
    hipLaunchKernelGGL(k_plan_user_direction, dim3(1), dim3(1), 0, s, st, ist, m);
    return hipGetLastError();
}

hipError_t lbfgs_plan_alpha(double *st, int *ist, int m, double mu, hipStream_t s)
{
    hipLaunchKernelGGL(k_plan_alpha, dim3(1), dim3(1), 0, s, st, ist, m, mu);
    return hipGetLastError();
}

hipError_t lbfgs_plan_update(double *st, int *ist, int m, double mu, hipStream_t s)
{
    hipLaunchKernelGGL(k_plan_update, dim3(1), dim3(1), 0, s, st, ist, m, mu);
    return hipGetLastError();
}

static VecList make_list(const float *const *p, int n)
{
    VecList v{};
    for (int i = 0; i < n && i <= kMaxBasis; ++i) v.p[i] = p[i];
    return v;
}

// Blocks of one resident round of a streaming kernel on the current device
// (fixed per kernel, so its partial sums stay deterministic).
template <typename K>
static int resident_blocks(K kern)
{
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return kBlocks;
    return std::max(1, per_cu * cus);
}

static int combine_blocks()
{
    static const int b = resident_blocks(k_combine);
    return b;
}

static int multidot_blocks()
{
    static const int b = resident_blocks(k_multidot);
    return b;
}

hipError_t lbfgs_combine(const float *const *basis, int nb, const double *coef, const int *mask, long long n,
                         float *d, double *partials, double *out, hipStream_t s)
{
    const int nblk = combine_blocks();
    hipLaunchKernelGGL(k_combine, dim3(nblk), dim3(256), 0, s, make_list(basis, nb), nb, coef, mask, n, d, partials);
    hipLaunchKernelGGL(k_sum_columns, dim3(kMaxBasis + 1), dim3(256), 0, s, partials, nblk, kMaxBasis + 1, out);
    return hipGetLastError();
}

hipError_t lbfgs_multidot(const float *x, const float *const *vecs, int nv, const int *mask, long long n,
                          double *partials, double *out, hipStream_t s, const float *const *y_slots, int ns,
                          const int *ist, int gold)
{
    VecList ys = y_slots ? make_list(y_slots, ns) : VecList{};
    const int nblk = multidot_blocks();
    hipLaunchKernelGGL(k_multidot, dim3(nblk), dim3(256), 0, s, x, make_list(vecs, nv), nv, mask, n, partials, ys,
                       y_slots ? ist : nullptr, gold);
    hipLaunchKernelGGL(k_sum_columns, dim3(nv), dim3(256), 0, s, partials, nblk, kMaxBasis + 1, out);
    return hipGetLastError();
}

hipError_t lbfgs_wnorm2(const float *q, const float *w, long long n, double *partials, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_wnorm2, dim3(kBlocks), dim3(256), 0, s, q, w, n, partials);
    return launch_sum_partials(partials, kBlocks, out, 1.0, 0, s);
}

hipError_t lbfgs_update_c(float *c, const float *d, const float *const *s_slots, int ns, const double *st,
                          const int *ist, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_update_c, dim3(kBlocks), dim3(256), 0, s, c, d, make_list(s_slots, ns), st, ist, n);
    return hipGetLastError();
}

hipError_t lbfgs_make_y(const float *const *y_slots, int ns, const int *ist, const float *gn, const float *go,
                        long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_make_y, dim3(kBlocks), dim3(256), 0, s, make_list(y_slots, ns), ist, gn, go, n);
    return hipGetLastError();
}

// r += alpha q (q may be null: r unchanged), yf = step fold(2 w r);
// out[0] = sum w r^2, out[1] = sum r^2.
hipError_t lbfgs_resid_update(const Dims &d, float *r, const float *q, const float *w, const double *st, float *yf,
                              double *partials, double *out, hipStream_t s)
{
    const long long npix = (long long)d.S * d.nj * d.nk;
    const bool vec = d.nseg == 2 * d.U && d.U == d.Up && (d.Up == 4 || d.Up == 8) &&
                     ((reinterpret_cast<uintptr_t>(r) | reinterpret_cast<uintptr_t>(q) |
                       reinterpret_cast<uintptr_t>(w) | reinterpret_cast<uintptr_t>(yf)) & 15) == 0;
    if (vec) {
        if (d.Up == 4)
            hipLaunchKernelGGL(k_resid_update_v<4>, dim3(kBlocks), dim3(256), 0, s, r, q, w, st, npix, d.step, yf,
                               partials);
        else
            hipLaunchKernelGGL(k_resid_update_v<8>, dim3(kBlocks), dim3(256), 0, s, r, q, w, st, npix, d.step, yf,
                               partials);
        hipLaunchKernelGGL(k_sum_columns, dim3(2), dim3(256), 0, s, partials, kBlocks, 2, out);
        return hipGetLastError();
    }
    switch (d.Up) {
    case 4:
        hipLaunchKernelGGL(k_resid_update<4>, dim3(kBlocks), dim3(256), 0, s, r, q, w, st, npix, d.nseg, d.U, d.step, yf,
                           partials);
        break;
    case 8:
        hipLaunchKernelGGL(k_resid_update<8>, dim3(kBlocks), dim3(256), 0, s, r, q, w, st, npix, d.nseg, d.U, d.step, yf,
                           partials);
        break;
    case 16:
        hipLaunchKernelGGL(k_resid_update<16>, dim3(kBlocks), dim3(256), 0, s, r, q, w, st, npix, d.nseg, d.U, d.step,
                           yf, partials);
        break;
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_sum_columns, dim3(2), dim3(256), 0, s, partials, kBlocks, 2, out);
    return hipGetLastError();
}

int lbfgs_blocks() { return std::max(kBlocks, std::max(combine_blocks(), multidot_blocks())); }

}  // namespace tt
