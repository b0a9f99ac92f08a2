// Internal declarations shared by the host API and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "tt.h"

namespace tt {

// Geometry copied out of tt_geometry, with offsets defaulted to zero.
struct Geometry {
    int nx, ny, nz, ell_max, n_proj, nj, nk, n_seg, n_sub;
    double step, seg_span;
    std::vector<double> inner, outer, joff, koff;
    double p[3], j[3], k[3], q0[3], q90[3], alpha_axis[3], beta_axis[3];
    int basis = TT_BASIS_SH;
    std::vector<double> dirs;  // [n][3], unit length (kernel bases)
    double kernel_width = 0.0;
};

// Number of basis functions of a geometry (SH count or grid size).
int basis_count(const Geometry &g);

// Stand-in for 1 / 0 in branch-free parameter ranges (see ProjFrame::inv_df).
constexpr float kFlatInv = 1.0e30f;

// Ray frame of one projection, float64, in centred sample coordinates.
// The ray through pixel (j, k) is o + j e_j + k e_k + t d.
struct ProjFrame {
    double o[3];
    double ej[3], ek[3], d[3];
    double inv_d[3];  // 1 / d_a, or 0 when the ray is parallel to plane a
    double lj, lk;    // L1 norms of e_j and e_k (bounds of the pixel window)
    // Shadow of the cube [-1, 1]^3 on the detector plane in (j, k) offsets:
    // for a row offset y = j - a the rays that can meet the cube have
    // k - b in [max_i(lo_i y + lo_i'), min_i(up_i y + up_i')] (hull[0..5] the
    // upper chain as (slope, intercept) pairs, hull[6..11] the lower chain).
    float hull[12];
    float ejf[3], ekf[3], df[3];  // float copies for the small offsets inside the cube
    // 1 / d_a, or kFlatInv when the ray is parallel to plane a: the adjoint's
    // parameter range |P_a + tau d_a| < 1 then reads (-P_a - 1, -P_a + 1) *
    // kFlatInv, which is all tau for |P_a| < 1 and empty otherwise, and some
    // other axis (|d_b| >= 1/sqrt 3) always bounds the range.
    float inv_df[3];
    // Slab plan of the LDS-staged march (tiles of kMarchTile x kMarchTile
    // rays): slabs are planes of axis slab_a (0 = x, 1 = y); each slab holds
    // the samples whose cell lies in slab_w consecutive planes, and stages a
    // box of (slab_w + 1) x slab_eb (the other horizontal axis) x slab_ez (z)
    // voxels that contains every corner those samples touch.  slab_w = 0:
    // the projection's rays gather from global memory instead.
    int slab_a, slab_w, slab_eb, slab_ez;
    // Joseph's method: dominant axis A of d (ties within 1e-9 go to the lower
    // axis) and the cut weight 1/|d_A|; for the adjoint, the in-plane offset of
    // a ray's cut from a voxel centre in the voxel's layer is
    // Delta_{B,C} = dj * jos_gj + dk * jos_gk (B = (A+1)%3, C = (A+2)%3) for
    // detector offsets (dj, dk) from the voxel's own position, and the
    // support |Delta_B|, |Delta_C| < 1 needs |dj| < jos_rj and |dk| < jos_rk.
    int jos_a;
    float jos_w;
    float jos_gj[2], jos_gk[2];
    float jos_igk[2];  // 1 / jos_gk, or kFlatInv where |jos_gk| <= 1e-6 (see inv_df)
    float jos_rj, jos_rk;
};

constexpr int kMarchTile = 16;  // rays per tile edge in the forward march

int num_coeffs(int ell_max);
void sh_eval_one(int ell_max, const double *dir, double *out);
void build_frames(const Geometry &g, std::vector<ProjFrame> &frames, std::vector<double> &B);
// Fills the slab plan of every frame for staged voxels of `up` floats within
// `lds_budget` bytes; returns the largest staging size in bytes (0 if none).
int plan_slabs(std::vector<ProjFrame> &frames, int up, int lds_budget);

// ---------------------------------------------------------------------------
// Kernel launchers (tt_proj.hip, tt_vec.hip).  All asynchronous on `st`.
// ---------------------------------------------------------------------------
struct Dims {
    int nx, ny, nz;     // volume
    int C, Cp;          // coefficients, padded to a multiple of 16
    int S, nj, nk;      // projections and detector
    int nseg, U, Up;    // segments, unique segments, padded unique segments
    float step;         // sample spacing of the trilinear model (1 for Joseph: no step factor)
    int march_lds;      // dynamic LDS bytes of the staged march (0: no projection staged)
    int joseph;         // 0: unit-step trilinear samples, 1: Joseph's method
    int inv_pair;       // 1: point-inversion-symmetric geometry (no detector offsets, even nx):
                        //    the adjoint (either model) with four or eight unique segments
                        //    enumerates each voxel pair (v, -v) once
    int win_ok;         // 1: every projection's residual window of a 4 x 8 x 8 brick fits the
                        //    adjoint's LDS window (trilinear model, eight unique segments)
    int pw_lds, pw_wr, pw_wc;  // paired + windowed adjoint: dynamic LDS bytes (0: not used) and
                               // window rows / columns
    int pwj_lds, pwj_wr, pwj_wc;  // the same for Joseph's method
    int sparse_k = 0;   // 0: exact basis constants, map + march; >= 1: kept basis functions per
                        //    (projection, segment) of the sparse map, fused forward
    int sparse_ng = 0;  // fused forward: channels per projection's list (the most any projection uses)
    int sparse_cm = 0;  // fused forward stages from a channel-major copy of c (few channels per projection)
};

// The fused forward stages from a channel-major copy of c when no projection
// keeps more than this many basis functions over its unique segments, and
// from the coefficient records c[v][0..C) otherwise (the per-channel arrays,
// whose loads run together, cost less than whole 4C-byte records).
constexpr int kFusedCmChannels = 32;

// M[p][(nx+2)(ny+2)(nz+2)][Up] = Bu[s0+p] c for p < np (zero border untouched).
hipError_t launch_map_fp32(const Dims &d, const float *c, const float *Bu, int s0, int np, float *M,
                           hipStream_t st);
hipError_t launch_map_bf16(const Dims &d, const float *c, const uint16_t *Bsw16, int s0, int np,
                           float *M, hipStream_t st);
// I[s0+p][j][k][c] = step * ray sums of M[p] along the rays of projection s0+p.
hipError_t launch_march(const Dims &d, const ProjFrame *frames, const float *M, int s0, int np,
                        float *I, hipStream_t st);
// Fused sparse forward: I[s][j][k][c] = step * ray sums over projection s of
// m_u(v) = sum_t w_t c[v][i_t] with (i_t, w_t) = sp[s][u][t] (int2: basis index,
// float bits), t < d.sparse_k, u = c mod U; all projections in one launch.
// With d.sparse_cm the staged voxels read the channel-major copy cT[i][v]
// (written first, V C floats of caller workspace) through the per-projection
// channel list gtab[s] = {ng channel indices, then ng x Up constants as float
// bits}; otherwise they read the coefficient records c[v][i] through sp.  Rays
// that gather from global memory use sp and c.
hipError_t launch_march_fused(const Dims &d, const ProjFrame *frames, const float *c, const int2 *sp,
                              const int *gtab, float *cT, float *I, hipStream_t st);
// yf[s][j][k][u] = scale * sum_{c: c mod U = u} y[s][j][k][c] (optionally
// y = 2 w (Ip - data) with the loss partials, see launch_residual_fold).
hipError_t launch_fold(const Dims &d, const float *y, float scale, float *yf, hipStream_t st);
// r = Ip - data (stored to r if non-null), yf = fold(2 w r) * step, and the
// float64 partial sums of w r^2 per block into partials.
hipError_t launch_residual_fold(const Dims &d, const float *Ip, const float *data, const float *w,
                                float *r, float *yf, double *partials, int nblocks, hipStream_t st);
// g = A^T-part(yf) + beta c, with float64 partials of sum c^2 when c != null.
// bf16 != 0: the transpose map runs on bf16 MFMA with Q rounded to bf16 and
// BuT16[s][Cp][16] (bf16, u padded to 16 with zeros).
hipError_t launch_backproject(const Dims &d, const ProjFrame *frames, const float *yf,
                              const float *Bu, const uint16_t *BuT16, int bf16, float *g, float beta,
                              const float *c, double *partials, hipStream_t st);
// Blocks (= float64 partials) of the adjoint launch; the largest over the
// adjoint variants of a geometry.
int backproject_blocks(const Dims &d);
int backproject_blocks_max(const Dims &d);
bool backproject_window_fits(const std::vector<ProjFrame> &frames);
int backproject_pw_lds(const std::vector<ProjFrame> &frames, int up, bool jos, int &wr, int &wc);

// Derived per-voxel quantities: out[v][kPropFields] from c[v][C] (tt_props.hip).
constexpr int kPropFields = 22;
hipError_t launch_tensor_props(const float *c, long long nvox, int C, float *out, hipStream_t st);

// Regularisers and the gradient-descent update (tt_reg.hip).
constexpr int kLapMaxC = 1024;  // coefficients per voxel supported by the Laplacian
// Value reductions write one float64 partial per block (at most kReduceBlocks)
// into `partials` and add them in block order: value[0] += scale * sum.
constexpr int kReduceBlocks = 4096;
hipError_t launch_laplacian_reg(const float *c, int nx, int ny, int nz, int C, double lam, float *work, float *grad,
                                double *value, double *partials, hipStream_t st);
hipError_t launch_huber_reg(const float *c, long long n, double delta, double lam, float *grad, double *value,
                            double *partials, hipStream_t st);
hipError_t launch_huber_loss(const float *I, const float *data, const float *w, long long n, double delta, float *y,
                             double *value, double *partials, hipStream_t st);
hipError_t launch_sumsq(const float *x, long long n, double scale, double *value, double *partials, hipStream_t st);
hipError_t launch_nesterov(float *c, float *y, const float *g, const float *p, long long n, float step, float m,
                           hipStream_t st);

// Normal-operator diagonal and input statistics (tt_stats.hip).
// u[v][i] = (i == 0) for nvox voxels of C coefficients.
hipError_t launch_fill_iso(float *u, long long nvox, int C, hipStream_t st);
// out[0] = lower median of g[v][ch] over the voxels v whose centre lies within
// `radius` of the volume centre (NaN if there are none); work holds
// ball_median_work_bytes() bytes.
size_t ball_median_work_bytes();
hipError_t launch_ball_median(const float *g, int nx, int ny, int nz, int C, int ch, double radius, void *work,
                              float *out, hipStream_t st);
// In place: p[v][i] = 1 / max(p[v][0], floor_frac * max_v p[v][0]) for all i;
// partial holds 1024 floats.
hipError_t launch_voxel_precond(float *p, long long nvox, int C, float floor_frac, float *partial, hipStream_t st);
// shift[c] = mean of pre x[v][c], scale[c] = 1 / (unbiased standard deviation,
// floored at 1e-12), c < nch <= 64; work holds chstats_work_doubles() doubles.
size_t chstats_work_doubles();
hipError_t launch_channel_stats(const float *x, long long nvox, int cstride, int nch, float pre, float *shift,
                                float *scale, double *work, hipStream_t st);

// Library-owned scratch of the allocation-free loss/gradient entry point
// (tt_static.hip): a fixed array per device, looked up once per device.
constexpr size_t kStaticScratchBytes = TT_NOALLOC_SCRATCH_BYTES;
// Looks up this device's scratch address (once; `device` must be current).
hipError_t static_scratch_init(int device);
// Device address of the scratch on `device` (null before a successful init).
void *static_scratch(int device);
// p[0 .. bytes) = 0 with a fill kernel (bytes and p 16-byte aligned).
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);

// Reductions: out[slot] = scale * sum of partials[0..n).
hipError_t launch_sum_partials(const double *partials, int n, double *out, double scale,
                               int accumulate, hipStream_t st);

// Warm-start network layers (tt_net.hip).  epi: 0 bias + ReLU -> bf16,
// 1 bias -> fp32, 2 zero where mask <= 0 -> bf16 (dgrad with the ReLU mask).
hipError_t net_conv(int epi, int ci, int co, const uint16_t *x, const void *wsw, const float *bias,
                    const uint16_t *mask, void *y, int N, int X, int Y, int Z, hipStream_t st);
int net_wgrad_chunks(int N, int X, int Y, int Z);
size_t net_wgrad_work_bytes(int ci, int co, int N, int X, int Y, int Z);
hipError_t net_wgrad(int ci, int co, const uint16_t *x, const uint16_t *gy, int N, int X, int Y, int Z, float *work,
                     float *gw, float *gb, hipStream_t st);
hipError_t net_swizzle(const float *w, int ci, int co, void *wf, void *wd, hipStream_t st);
hipError_t net_adam(float *w, const float *g, float *m, float *v, long long n, int t, float lr, float b1, float b2,
                    float eps, hipStream_t st);
hipError_t net_mse(const float *y, const float *t, long long nvox, int cpad, int creal, float scale, uint16_t *gy,
                   double *partials, int nblocks, double *loss, hipStream_t st);
hipError_t net_pack(const float *x, long long nvox, int cin, int cpad, float pre, const float *shift,
                    const float *scale, uint16_t *out, hipStream_t st);
hipError_t net_tile_gather(const float *vol, int X, int Y, int Z, int cv, int cin, int cpad, const int *ox, int ntx,
                           const int *oy, int nty, const int *oz, int ntz, int T, float pre, const float *shift,
                           const float *scale, int t0, int nt, uint16_t *out, hipStream_t st);
hipError_t net_tile_blend(const float *y, int cy, int creal, int X, int Y, int Z, const int *ox, int ntx, const int *oy,
                          int nty, const int *oz, int ntz, int T, int ramp, int cout, float *out, hipStream_t st);

}  // namespace tt
