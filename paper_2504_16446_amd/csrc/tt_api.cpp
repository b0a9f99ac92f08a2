// C ABI of the tensor-tomography hot path (see include/tt.h).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "tt_internal.h"
#include "tt_lbfgs.h"

using namespace tt;

namespace {

thread_local std::string g_last_error = "no error";

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

#define TT_HIP(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(TT_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));         \
    } while (0)

int round_up(int v, int m) { return (v + m - 1) / m * m; }

}  // namespace

struct tt_ctx {
    Geometry g;
    Dims d;
    int device = 0;
    hipStream_t stream = nullptr;
    int precision = TT_MAP_FP32;
    std::vector<ProjFrame> frames;
    std::vector<double> B;  // [S][nseg][C] float64, the constants in use
    std::vector<double> B_exact;  // the exact constants (B differs under a sparse map)
    ProjFrame *d_frames = nullptr;
    int2 *d_sp = nullptr;       // [S][Up][sparse_k] sparse map (basis index, constant bits)
    int *d_gtab = nullptr;      // [S][sparse_ng (Up + 1)] channel list and constants of the fused staging
    float *d_Bu = nullptr;      // [bu_rows][Cp]: row s*Up + u, zero padded
    float *d_Bsw = nullptr;     // Bu in MFMA lane order (16-row tiles), for the forward map
    uint16_t *d_Bsw16 = nullptr; // bf16 Bu in MFMA lane order (16-row tiles, 32-coefficient steps), forward
    uint16_t *d_BuT16 = nullptr; // bf16 [S][Cp][16]: B^T with u padded to 16, adjoint
    int pb = 0;                 // projections per forward batch (0: no workspace attached)
    long long vol_pad = 0;
    size_t per_proj = 0;        // bytes of one projection's mapped volume M
    int n_part = 0;             // float64 reduction partials
    // Caller-owned workspace (tt_set_workspace): partials, folded residual
    // yf, a data-sized residual scratch and the mapped volumes of one batch.
    char *ws = nullptr;
    size_t ws_bytes = 0;
    double *d_part = nullptr;   // [n_part]
    float *d_yf = nullptr;      // [S][nj][nk][Up]
    float *d_resid = nullptr;   // [S][nj][nk][n_seg]
    float *d_M = nullptr;       // [pb][vol_pad][Up], zero border
    float *d_cT = nullptr;      // [C][V] channel-major copy of c (fused sparse forward only)
    size_t table_bytes = 0;
    bool timing = false;
    struct Mark {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
};

namespace {

// Brackets the launches of one kernel class with events when timing is on.
struct KTimer {
    tt_ctx *c;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    KTimer(tt_ctx *ctx, int k, bool allowed = true) : c(ctx), kind(k)
    {
        if (allowed && c->timing && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            hipEventRecord(a, c->stream);
    }
    ~KTimer()
    {
        if (b) {
            hipEventRecord(b, c->stream);
            c->marks.push_back({kind, a, b});
        }
    }
};

}  // namespace

struct tt_lbfgs {
    tt_ctx *ctx = nullptr;
    int m = 0;
    std::vector<float *> s, y;  // m + 1 slots each
    float *g[2] = {nullptr, nullptr};
    float *d = nullptr;
    float *r = nullptr, *q = nullptr;
    double *st = nullptr;
    int *ist = nullptr;
    double *part = nullptr;
    int gcur = 0;
    float *c = nullptr;
    const float *data = nullptr, *w = nullptr;
    double mu = 0.0;
    bool inited = false;
};

static uint16_t to_bf16(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}

// Basis tables in the layouts the kernels read, built from the constants in use (c->B).
struct Tables {
    std::vector<float> bu;         // [bu_rows][Cp]: row s*Up + u, zero padded
    std::vector<float> bsw;        // bu in MFMA lane order: tile rt, k-step ks, lane l
    std::vector<uint16_t> bsw16;   // bf16 bu in MFMA lane order (16-row tiles, k blocks of 16)
    std::vector<uint16_t> but16;   // bf16 [S][Cp][16]: B^T with u padded to 16
};
static void build_tables(const tt_ctx *c, Tables &t)
{
    const Dims &d = c->d;
    const int S = d.S;
    const int bu_rows = round_up(S * d.Up, 256) + 256;
    t.bu.assign((size_t)bu_rows * d.Cp, 0.0f);
    for (int s = 0; s < S; ++s)
        for (int u = 0; u < d.U; ++u)
            for (int i = 0; i < d.C; ++i)
                t.bu[((size_t)s * d.Up + u) * d.Cp + i] = (float)c->B[((size_t)s * d.nseg + u) * d.C + i];
    // row tile rt (16 Cp values): 32-coefficient steps kp, lane l, eight values
    // bu[16 rt + l % 16][32 kp + 8 (l / 16) + q]; then, for Cp / 16 odd, the last
    // 16 coefficients as four values bu[16 rt + l % 16][32 KP + 4 (l / 16) + q]
    const int KP = d.Cp / 32;
    t.bsw16.assign(t.bu.size(), 0);
    t.but16.assign((size_t)S * d.Cp * 16, 0);
    for (int rt = 0; rt < bu_rows / 16; ++rt) {
        const size_t base = (size_t)rt * 16 * d.Cp;
        for (int l = 0; l < 64; ++l) {
            const float *row = &t.bu[((size_t)rt * 16 + l % 16) * d.Cp];
            for (int kp = 0; kp < KP; ++kp)
                for (int q = 0; q < 8; ++q)
                    t.bsw16[base + ((size_t)kp * 64 + l) * 8 + q] = to_bf16(row[32 * kp + 8 * (l / 16) + q]);
            if (d.Cp & 16)
                for (int q = 0; q < 4; ++q)
                    t.bsw16[base + (size_t)KP * 512 + l * 4 + q] = to_bf16(row[32 * KP + 4 * (l / 16) + q]);
        }
    }
    for (int s = 0; s < S; ++s)
        for (int i = 0; i < d.Cp; ++i)
            for (int u = 0; u < d.Up; ++u)
                t.but16[((size_t)s * d.Cp + i) * 16 + u] = to_bf16(t.bu[((size_t)s * d.Up + u) * d.Cp + i]);
    // MFMA-ordered copy of bu: tile rt, k-step ks, lane l -> bu[16 rt + l % 16][4 ks + l / 16]
    t.bsw.assign(t.bu.size(), 0.0f);
    const int KS = d.Cp / 4;
    for (int rt = 0; rt < bu_rows / 16; ++rt)
        for (int ks = 0; ks < KS; ++ks)
            for (int l = 0; l < 64; ++l)
                t.bsw[((size_t)rt * KS + ks) * 64 + l] = t.bu[((size_t)rt * 16 + l % 16) * d.Cp + 4 * ks + l / 16];
}

// Kept entries of one row of basis constants under the sparse map: taken one
// at a time, the largest remaining magnitude m first, and among the remaining
// entries with |B| >= m - 1e-9 max|row| the lowest index.
static void sparse_select(const double *row, int C, int k, std::vector<int> &keep)
{
    double scale = 0.0;
    for (int i = 0; i < C; ++i) scale = std::max(scale, std::fabs(row[i]));
    std::vector<char> used(C, 0);
    keep.clear();
    for (int n = 0; n < std::min(k, C); ++n) {
        double m = -1.0;
        for (int i = 0; i < C; ++i)
            if (!used[i]) m = std::max(m, std::fabs(row[i]));
        for (int i = 0; i < C; ++i)
            if (!used[i] && std::fabs(row[i]) >= m - 1e-9 * scale) {
                used[i] = 1;
                keep.push_back(i);
                break;
            }
    }
}

static long long n_coef(const tt_ctx *c) { return (long long)c->d.nx * c->d.ny * c->d.nz * c->d.C; }
static long long n_data(const tt_ctx *c) { return (long long)c->d.S * c->d.nj * c->d.nk * c->d.nseg; }

extern "C" {

const char *tt_last_error(void) { return g_last_error.c_str(); }

const char *tt_error_string(int code)
{
    switch (code) {
    case TT_OK: return "ok";
    case TT_EINVAL: return "invalid argument";
    case TT_ESHAPE: return "inconsistent shape";
    case TT_ENOMEM: return "out of memory";
    case TT_EHIP: return "HIP runtime error";
    case TT_ENONFINITE: return "non-finite value";
    case TT_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown error";
    }
}

int tt_num_coeffs(int ell_max)
{
    if (ell_max < 0 || ell_max % 2) return fail(TT_EINVAL, "ell_max must be even and >= 0");
    return num_coeffs(ell_max);
}

int tt_sh_eval(int ell_max, int64_t n, const double *dirs, double *out)
{
    if (ell_max < 0 || ell_max % 2 || ell_max > 16) return fail(TT_EINVAL, "ell_max must be even, 0..16");
    if (n < 0 || (n > 0 && (!dirs || !out))) return fail(TT_EINVAL, "null pointer");
    const int C = num_coeffs(ell_max);
    for (int64_t t = 0; t < n; ++t) {
        const double *v = dirs + 3 * t;
        if (!(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] > 0.0)) return fail(TT_EINVAL, "zero direction");
        sh_eval_one(ell_max, v, out + C * t);
    }
    return TT_OK;
}

static bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

static int read_geometry(const tt_geometry *geom, Geometry &g)
{
    if (!geom) return fail(TT_EINVAL, "geometry is null");
    const tt_geometry &G = *geom;
    if (G.nx < 1 || G.ny < 1 || G.nz < 1 || G.nj < 1 || G.nk < 1 || G.n_proj < 1)
        return fail(TT_ESHAPE, "volume, detector and projection counts must be >= 1");
    if ((long long)G.nx * G.ny * G.nz > (1LL << 31) - 1) return fail(TT_EUNSUPPORTED, "volume above 2^31 voxels");
    if (G.ell_max < 0 || G.ell_max % 2) return fail(TT_EINVAL, "ell_max must be even and >= 0");
    if (G.ell_max > 16) return fail(TT_EUNSUPPORTED, "ell_max above 16");
    if (G.n_seg < 1 || G.n_seg > 64) return fail(TT_EINVAL, "n_seg must be 1..64");
    if (G.n_sub < 1) return fail(TT_EINVAL, "n_sub must be >= 1");
    if (!(G.step > 0.0) || !std::isfinite(G.step)) return fail(TT_EINVAL, "step must be > 0");
    if (!(G.seg_span > 0.0) || !std::isfinite(G.seg_span)) return fail(TT_EINVAL, "seg_span must be > 0");
    if (G.map_precision != TT_MAP_FP32 && G.map_precision != TT_MAP_BF16)
        return fail(TT_EINVAL, "map_precision must be TT_MAP_FP32 or TT_MAP_BF16");
    if (!G.inner_angle || !G.outer_angle) return fail(TT_EINVAL, "angle arrays are null");
    const double *vecs[7] = {G.p, G.j, G.k, G.q0, G.q90, G.alpha_axis, G.beta_axis};
    for (auto v : vecs) {
        if (!finite3(v) || !(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] > 0.0))
            return fail(TT_EINVAL, "geometry vectors must be finite and nonzero");
    }
    // the raster directions and the beam must form an orthonormal frame
    auto dot = [](const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
    if (std::fabs(dot(G.p, G.j)) > 1e-9 || std::fabs(dot(G.p, G.k)) > 1e-9 || std::fabs(dot(G.j, G.k)) > 1e-9 ||
        std::fabs(dot(G.p, G.p) - 1) > 1e-9 || std::fabs(dot(G.j, G.j) - 1) > 1e-9 || std::fabs(dot(G.k, G.k) - 1) > 1e-9)
        return fail(TT_EINVAL, "p, j, k must be orthonormal");
    g.nx = G.nx; g.ny = G.ny; g.nz = G.nz; g.ell_max = G.ell_max; g.n_proj = G.n_proj;
    g.nj = G.nj; g.nk = G.nk; g.n_seg = G.n_seg; g.n_sub = G.n_sub;
    g.step = G.step; g.seg_span = G.seg_span;
    g.inner.assign(G.inner_angle, G.inner_angle + G.n_proj);
    g.outer.assign(G.outer_angle, G.outer_angle + G.n_proj);
    g.joff.assign(G.n_proj, 0.0);
    g.koff.assign(G.n_proj, 0.0);
    if (G.j_offset) g.joff.assign(G.j_offset, G.j_offset + G.n_proj);
    if (G.k_offset) g.koff.assign(G.k_offset, G.k_offset + G.n_proj);
    for (int s = 0; s < G.n_proj; ++s)
        if (!std::isfinite(g.inner[s]) || !std::isfinite(g.outer[s]) || !std::isfinite(g.joff[s]) ||
            !std::isfinite(g.koff[s]))
            return fail(TT_EINVAL, "non-finite angle or offset");
    std::memcpy(g.p, G.p, sizeof g.p); std::memcpy(g.j, G.j, sizeof g.j); std::memcpy(g.k, G.k, sizeof g.k);
    std::memcpy(g.q0, G.q0, sizeof g.q0); std::memcpy(g.q90, G.q90, sizeof g.q90);
    std::memcpy(g.alpha_axis, G.alpha_axis, sizeof g.alpha_axis);
    std::memcpy(g.beta_axis, G.beta_axis, sizeof g.beta_axis);
    g.basis = G.basis;
    g.dirs.clear();
    g.kernel_width = 0.0;
    if (G.basis != TT_BASIS_SH) {
        if (G.basis != TT_BASIS_GK && G.basis != TT_BASIS_NN) return fail(TT_EINVAL, "unknown basis");
        if (G.n_dirs < 1 || !G.dirs) return fail(TT_EINVAL, "kernel bases need n_dirs >= 1 grid directions");
        if (G.n_dirs > 96) return fail(TT_EUNSUPPORTED, "at most 96 grid directions");
        if (G.basis == TT_BASIS_GK && (!(G.kernel_width > 0.0) || !std::isfinite(G.kernel_width)))
            return fail(TT_EINVAL, "kernel_width must be > 0");
        g.kernel_width = G.kernel_width;
        g.dirs.resize(3 * (size_t)G.n_dirs);
        for (int i = 0; i < G.n_dirs; ++i) {
            const double *d = G.dirs + 3 * i;
            const double n = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (!finite3(d) || !(n > 0.0)) return fail(TT_EINVAL, "grid directions must be finite and nonzero");
            for (int a = 0; a < 3; ++a) g.dirs[3 * i + a] = d[a] / n;
        }
    }
    return TT_OK;
}

int tt_geometry_basis(const tt_geometry *geom, double *B_host)
{
    if (!B_host) return fail(TT_EINVAL, "B_host is null");
    Geometry g;
    int rc = read_geometry(geom, g);
    if (rc) return rc;
    std::vector<ProjFrame> frames;
    std::vector<double> B;
    build_frames(g, frames, B);
    std::memcpy(B_host, B.data(), B.size() * sizeof(double));
    return TT_OK;
}

int tt_create(const tt_geometry *geom, tt_ctx **out)
{
    if (!out) return fail(TT_EINVAL, "out is null");
    *out = nullptr;
    tt_ctx *c = new (std::nothrow) tt_ctx();
    if (!c) return fail(TT_ENOMEM, "host allocation failed");
    Geometry &g = c->g;
    int rc0 = read_geometry(geom, g);
    if (rc0) {
        delete c;
        return rc0;
    }
    c->precision = geom->map_precision;

    build_frames(g, c->frames, c->B);

    Dims &d = c->d;
    d.nx = g.nx; d.ny = g.ny; d.nz = g.nz;
    d.C = basis_count(g);
    d.Cp = round_up(d.C, 16);
    if (d.Cp > 96) {  // the adjoint keeps Cp/16 <= 6 accumulator tiles per wave
        delete c;
        return fail(TT_EUNSUPPORTED, "projector supports ell_max <= 12 / 96 basis functions (96 padded coefficients)");
    }
    d.S = g.n_proj; d.nj = g.nj; d.nk = g.nk; d.nseg = g.n_seg;
    d.step = (float)g.step;
    d.joseph = 0;
    // the sample lattice of every projection is symmetric under x -> -x when
    // the detector is centred (no offsets); with even nx the lower and upper
    // x-halves then pair voxel by voxel
    bool centred = true;
    for (int s = 0; s < g.n_proj; ++s) centred = centred && g.joff[s] == 0.0 && g.koff[s] == 0.0;
    d.inv_pair = centred && g.nx % 2 == 0 ? 1 : 0;
    // Even orders: Y(-q) = Y(q) (and the Gaussian kernels are symmetric too), and
    // with segments over the full circle segment c + n_seg/2 probes exactly the
    // antipodes of segment c.
    // (The nearest-neighbour basis is excluded: a node nearly equidistant from
    // two grid directions may pick different ones for q and for the computed
    // -q, so its antipodal segments agree only up to such ties.)
    const bool antipodal = std::fabs(g.seg_span - 2.0 * M_PI) < 1e-12 && g.n_seg % 2 == 0 && g.basis != TT_BASIS_NN;
    d.U = antipodal ? g.n_seg / 2 : g.n_seg;
    if (d.U > 16) {
        delete c;
        return fail(TT_EUNSUPPORTED, "more than 16 distinct segments");
    }
    d.Up = d.U <= 4 ? 4 : (d.U <= 8 ? 8 : 16);
    if ((long long)d.nj * d.nk * (d.Up / 4) >= (1LL << 24)) {  // the adjoint's 24-bit row offsets
        delete c;
        return fail(TT_EUNSUPPORTED, "detector too large: nj * nk * " + std::to_string(d.Up / 4) +
                                         " must stay below 2^24 (float4 units of one projection)");
    }
    // staged march LDS per 256-ray tile: 52 KiB for four unique segments (three
    // blocks per CU), 76 KiB for more (two blocks per CU); measured best of
    // 20-76 KiB on 100^3 x 4 and of 32-76 KiB on 128^3 and 256^3 x 8
    d.march_lds = plan_slabs(c->frames, d.Up, (d.Up == 4 ? 52 : 76) * 1024);
    d.win_ok = backproject_window_fits(c->frames) ? 1 : 0;
    d.pw_lds = backproject_pw_lds(c->frames, d.Up, false, d.pw_wr, d.pw_wc);
    d.pwj_lds = backproject_pw_lds(c->frames, d.Up, true, d.pwj_wr, d.pwj_wc);

    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(TT_EHIP, "hipGetDevice failed");
    }
    // device address of the library's static scratch (tt_loss_grad_noalloc),
    // looked up once per device while it is current
    if (hipError_t e = static_scratch_init(c->device); e != hipSuccess) {
        delete c;
        return fail(TT_EHIP, std::string("static scratch lookup: ") + hipGetErrorString(e));
    }
    const int S = d.S;
    c->B_exact = c->B;
    Tables t;
    build_tables(c, t);
    c->vol_pad = (long long)(d.nx + 2) * (d.ny + 2) * (d.nz + 2);
    c->per_proj = (size_t)c->vol_pad * d.Up * sizeof(float);
    c->n_part = 1024 + std::max(4096, backproject_blocks_max(d));
    const std::vector<float> &bu = t.bu, &bsw = t.bsw;
    const std::vector<uint16_t> &bsw16 = t.bsw16, &but16 = t.but16;
    const size_t sp_len = (size_t)S * d.Up * d.C;
    const size_t gtab_len = (size_t)S * d.C * (d.Up + 1);

    auto cleanup = [&](int code, const std::string &msg) {
        tt_destroy(c);
        return fail(code, msg);
    };
    if (hipMalloc(&c->d_frames, sizeof(ProjFrame) * S) != hipSuccess ||
        hipMalloc(&c->d_Bu, bu.size() * sizeof(float)) != hipSuccess ||
        hipMalloc(&c->d_Bsw, bsw.size() * sizeof(float)) != hipSuccess ||
        hipMalloc(&c->d_Bsw16, bsw16.size() * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc(&c->d_BuT16, but16.size() * sizeof(uint16_t)) != hipSuccess ||
        hipMalloc(&c->d_sp, sp_len * sizeof(int2)) != hipSuccess ||
        hipMalloc(&c->d_gtab, gtab_len * sizeof(int)) != hipSuccess)
        return cleanup(TT_ENOMEM, "device allocation failed");
    c->table_bytes = sizeof(ProjFrame) * S + bu.size() * 10 + but16.size() * 2 + sp_len * sizeof(int2) +
                     gtab_len * sizeof(int);
    if (hipMemcpy(c->d_frames, c->frames.data(), sizeof(ProjFrame) * S, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_Bu, bu.data(), bu.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_Bsw, bsw.data(), bsw.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_Bsw16, bsw16.data(), bsw16.size() * sizeof(uint16_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_BuT16, but16.data(), but16.size() * sizeof(uint16_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess)
        return cleanup(TT_EHIP, "device upload failed");
    *out = c;
    return TT_OK;
}

void tt_destroy(tt_ctx *c)
{
    if (!c) return;
    hipStreamSynchronize(c->stream);  // queued kernels may still read these buffers
    tt_timing_enable(c, 0);
    hipFree(c->d_frames);
    hipFree(c->d_Bu);
    hipFree(c->d_Bsw);
    hipFree(c->d_Bsw16);
    hipFree(c->d_BuT16);
    hipFree(c->d_sp);
    hipFree(c->d_gtab);
    delete c;
}

int tt_set_stream(tt_ctx *c, void *stream)
{
    if (!c) return fail(TT_EINVAL, "ctx is null");
    c->stream = (hipStream_t)stream;
    return TT_OK;
}

int tt_set_projector(tt_ctx *c, int model)
{
    if (!c) return fail(TT_EINVAL, "null context");
    if (model != TT_PROJ_TRILINEAR && model != TT_PROJ_JOSEPH)
        return fail(TT_EINVAL, "model must be TT_PROJ_TRILINEAR or TT_PROJ_JOSEPH");
    c->d.joseph = model == TT_PROJ_JOSEPH;
    // Joseph's cuts carry their own 1/|d_A| weight: no sample-spacing factor
    c->d.step = c->d.joseph ? 1.0f : (float)c->g.step;
    return TT_OK;
}

int tt_set_map_precision(tt_ctx *c, int precision)
{
    if (!c) return fail(TT_EINVAL, "ctx is null");
    if (precision != TT_MAP_FP32 && precision != TT_MAP_BF16) return fail(TT_EINVAL, "bad precision");
    if (precision == TT_MAP_BF16 && c->d.sparse_k > 0)
        return fail(TT_EUNSUPPORTED, "the sparse fused map runs in float32 only");
    c->precision = precision;
    return TT_OK;
}

int tt_set_sparse_map(tt_ctx *c, int k)
{
    if (!c) return fail(TT_EINVAL, "ctx is null");
    if (k < 0) return fail(TT_EINVAL, "k must be >= 0");
    const Dims &d = c->d;
    if (k > 0 && c->precision == TT_MAP_BF16) return fail(TT_EUNSUPPORTED, "the sparse fused map runs in float32 only");
    const int kk = std::min(k, d.C);
    std::vector<int2> sp;
    std::vector<int> gtab;
    int ng = 0;
    if (k == 0) {
        c->B = c->B_exact;
    } else {
        // rows u < U; with an antipodal fold the rows c = u + U (same constants) copy row u
        sp.assign((size_t)d.S * d.Up * kk, int2{0, 0});
        std::vector<int> keep;
        for (int s = 0; s < d.S; ++s)
            for (int u = 0; u < d.U; ++u) {
                const double *row = &c->B_exact[((size_t)s * d.nseg + u) * d.C];
                sparse_select(row, d.C, kk, keep);
                std::vector<double> sparse(d.C, 0.0);
                for (size_t t = 0; t < keep.size(); ++t) {
                    sparse[keep[t]] = row[keep[t]];
                    const float w = (float)row[keep[t]];
                    int wb;
                    std::memcpy(&wb, &w, 4);
                    sp[((size_t)s * d.Up + u) * kk + t] = int2{keep[t], wb};
                }
                for (int cs = u; cs < d.nseg; cs += d.U)
                    std::memcpy(&c->B[((size_t)s * d.nseg + cs) * d.C], sparse.data(), sizeof(double) * d.C);
            }
        // channel lists of the fused staging: the basis functions any unique
        // segment of the projection keeps, in increasing order, with their
        // constants per segment (zero where a segment does not keep them)
        std::vector<std::vector<int>> lists(d.S);
        for (int s = 0; s < d.S; ++s) {
            std::vector<char> used(d.C, 0);
            for (int u = 0; u < d.U; ++u)
                for (int t = 0; t < kk; ++t) used[sp[((size_t)s * d.Up + u) * kk + t].x] = 1;
            for (int i = 0; i < d.C; ++i)
                if (used[i]) lists[s].push_back(i);
            ng = std::max(ng, (int)lists[s].size());
        }
        gtab.assign((size_t)d.S * ng * (d.Up + 1), 0);
        for (int s = 0; s < d.S; ++s) {
            int *row = &gtab[(size_t)s * ng * (d.Up + 1)];
            for (size_t g = 0; g < lists[s].size(); ++g) {
                row[g] = lists[s][g];
                for (int u = 0; u < d.U; ++u) {
                    const float w = (float)c->B[((size_t)s * d.nseg + u) * d.C + lists[s][g]];
                    std::memcpy(&row[ng + g * d.Up + u], &w, 4);
                }
            }
            // unused list slots keep channel 0 with zero constants
        }
    }
    Tables t;
    build_tables(c, t);
    TT_HIP(hipStreamSynchronize(c->stream));  // queued kernels may still read the tables
    TT_HIP(hipMemcpy(c->d_Bu, t.bu.data(), t.bu.size() * sizeof(float), hipMemcpyHostToDevice));
    TT_HIP(hipMemcpy(c->d_Bsw, t.bsw.data(), t.bsw.size() * sizeof(float), hipMemcpyHostToDevice));
    TT_HIP(hipMemcpy(c->d_Bsw16, t.bsw16.data(), t.bsw16.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
    TT_HIP(hipMemcpy(c->d_BuT16, t.but16.data(), t.but16.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
    if (!sp.empty()) TT_HIP(hipMemcpy(c->d_sp, sp.data(), sp.size() * sizeof(int2), hipMemcpyHostToDevice));
    if (!gtab.empty()) TT_HIP(hipMemcpy(c->d_gtab, gtab.data(), gtab.size() * sizeof(int), hipMemcpyHostToDevice));
    const bool was_fused = c->d.sparse_k > 0;
    c->d.sparse_k = k == 0 ? 0 : kk;
    c->d.sparse_ng = ng;
    const bool cm_changed = c->d.sparse_cm != (k > 0 && ng <= kFusedCmChannels ? 1 : 0);
    c->d.sparse_cm = k > 0 && ng <= kFusedCmChannels ? 1 : 0;
    if (was_fused != (k > 0) || cm_changed) {  // the workspace layout changes: the caller attaches a new one
        c->ws = nullptr;
        c->ws_bytes = 0;
        c->pb = 0;
    }
    return TT_OK;
}

int tt_timing_enable(tt_ctx *c, int on)
{
    if (!c) return fail(TT_EINVAL, "ctx is null");
    for (auto &mk : c->marks) {
        hipEventDestroy(mk.a);
        hipEventDestroy(mk.b);
    }
    c->marks.clear();
    c->timing = on != 0;
    return TT_OK;
}

int tt_timing_read(tt_ctx *c, double *ms_total, int64_t *launches)
{
    if (!c || !ms_total || !launches) return fail(TT_EINVAL, "null pointer");
    TT_HIP(hipStreamSynchronize(c->stream));
    for (int k = 0; k < TT_K_COUNT; ++k) {
        ms_total[k] = 0.0;
        launches[k] = 0;
    }
    for (auto &mk : c->marks) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, mk.a, mk.b) == hipSuccess) {
            ms_total[mk.kind] += ms;
            launches[mk.kind] += 1;
        }
        hipEventDestroy(mk.a);
        hipEventDestroy(mk.b);
    }
    c->marks.clear();
    return TT_OK;
}

int tt_sizes(const tt_ctx *c, int64_t *out8)
{
    if (!c || !out8) return fail(TT_EINVAL, "null pointer");
    out8[0] = n_coef(c);
    out8[1] = n_data(c);
    out8[2] = c->d.C;
    out8[3] = c->d.U;
    out8[4] = c->pb;
    out8[5] = (int64_t)c->ws_bytes;
    out8[6] = (int64_t)c->table_bytes;
    out8[7] = (int64_t)c->per_proj;
    return TT_OK;
}

// Workspace layout for a forward batch of pb projections (pb = 0: no mapped volumes).
struct WsLayout {
    size_t part, yf, resid, cT, M, total;
};
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
static WsLayout ws_layout(const tt_ctx *c, int pb)
{
    WsLayout L;
    size_t off = 0;
    L.part = off;
    off += align256(sizeof(double) * c->n_part);
    L.yf = off;
    off += align256(sizeof(float) * (size_t)c->d.S * c->d.nj * c->d.nk * c->d.Up);
    L.resid = off;
    off += align256(sizeof(float) * (size_t)n_data(c));
    L.cT = off;  // channel-major copy of c for the fused sparse forward
    if (c->d.sparse_k > 0 && c->d.sparse_cm) off += align256(sizeof(float) * (size_t)n_coef(c));
    L.M = off;
    off += align256(c->per_proj * (size_t)pb);
    L.total = off;
    return L;
}
// Largest valid forward batch not above pb: every batch but the last must
// start on a 16-row map tile (pb a multiple of 16 / Up) and batches of 256 /
// Up or more are kept whole multiples of the 256-row map block.  0 if none.
static int batch_round_down(const tt_ctx *c, long long pb)
{
    const int S = c->d.S, align = 16 / c->d.Up, full = 256 / c->d.Up;
    if (pb >= S) return S;
    if (pb >= full) return (int)(pb / full * full);
    return (int)(pb / align * align);
}
static int batch_min(const tt_ctx *c) { return std::min(c->d.S, 16 / c->d.Up); }

static int need_ws(const tt_ctx *c)
{
    if (!c->ws) return fail(TT_EINVAL, "no workspace attached to the context (tt_set_workspace)");
    return TT_OK;
}

// Scratch of one forward / adjoint / loss evaluation: the attached workspace,
// or the library's static array (tt_loss_grad_noalloc, untimed: no events).
struct Scratch {
    double *part;
    float *yf, *resid, *M, *cT;
    int pb;
    bool timed;
};
static Scratch attached(const tt_ctx *c) { return {c->d_part, c->d_yf, c->d_resid, c->d_M, c->d_cT, c->pb, true}; }

int64_t tt_workspace_bytes(const tt_ctx *c, int forward_batch)
{
    if (!c) return fail(TT_EINVAL, "ctx is null");
    if (forward_batch <= 0) return (int64_t)ws_layout(c, 0).total;  // no mapped volumes (fused forward only)
    int pb = batch_round_down(c, std::min(forward_batch, c->d.S));
    pb = std::max(pb, batch_min(c));
    return (int64_t)ws_layout(c, pb).total;
}

int tt_set_workspace(tt_ctx *c, void *work, size_t bytes)
{
    if (!c) return fail(TT_EINVAL, "ctx is null");
    if (!work) return fail(TT_EINVAL, "workspace is null");
    if (reinterpret_cast<uintptr_t>(work) % 256) return fail(TT_EINVAL, "workspace must be 256-byte aligned");
    const size_t base = ws_layout(c, 0).total;
    const long long fit = bytes > base ? (long long)((bytes - base) / c->per_proj) : 0;
    int pb = batch_round_down(c, fit);
    if (pb < batch_min(c)) {
        if (c->d.sparse_k == 0 || bytes < base)
            return fail(TT_EINVAL, "workspace of " + std::to_string(bytes) + " bytes is below the minimum of " +
                                       std::to_string(c->d.sparse_k ? base : (size_t)tt_workspace_bytes(c, 1)));
        pb = 0;  // the fused forward needs no mapped volumes
    }
    const WsLayout L = ws_layout(c, pb);
    c->ws = static_cast<char *>(work);
    c->ws_bytes = bytes;
    c->pb = pb;
    c->d_part = reinterpret_cast<double *>(c->ws + L.part);
    c->d_yf = reinterpret_cast<float *>(c->ws + L.yf);
    c->d_resid = reinterpret_cast<float *>(c->ws + L.resid);
    c->d_M = reinterpret_cast<float *>(c->ws + L.M);
    c->d_cT = reinterpret_cast<float *>(c->ws + L.cT);
    // the map writes only interior voxels: the border of every mapped volume stays zero
    if (pb > 0) TT_HIP(hipMemsetAsync(c->d_M, 0, c->per_proj * (size_t)pb, c->stream));
    return TT_OK;
}

// Number of ray samples (trilinear model) or plane cuts (Joseph) that touch the
// volume: the ray parameter ranges the forward march visits, counted on the host
// from the float64 ray frames with the same inequalities.
int tt_ray_samples(const tt_ctx *c, int64_t *out)
{
    if (!c || !out) return fail(TT_EINVAL, "null pointer");
    const Dims &d = c->d;
    const double n3[3] = {(double)d.nx, (double)d.ny, (double)d.nz};
    long long total = 0;
    for (int s = 0; s < d.S; ++s) {
        const ProjFrame &f = c->frames[s];
        for (int j = 0; j < d.nj; ++j)
            for (int k = 0; k < d.nk; ++k) {
                double b[3];
                for (int a = 0; a < 3; ++a) b[a] = f.o[a] + j * f.ej[a] + k * f.ek[a] + 0.5 * (n3[a] + 1.0);
                if (!d.joseph) {
                    double tlo = -1e300, thi = 1e300;
                    for (int a = 0; a < 3; ++a) {
                        if (f.inv_d[a] != 0.0) {
                            const double ia = f.inv_d[a] / (double)d.step;
                            const double t1 = -b[a] * ia, t2 = (n3[a] + 1.0 - b[a]) * ia;
                            tlo = std::max(tlo, std::min(t1, t2));
                            thi = std::min(thi, std::max(t1, t2));
                        } else if (!(b[a] > 0.0 && b[a] < n3[a] + 1.0)) {
                            thi = -1e300;
                        }
                    }
                    if (tlo < thi) total += std::max(0LL, (long long)std::floor(thi) - (long long)std::ceil(tlo) + 1);
                } else {
                    const int A = f.jos_a, B = (A + 1) % 3, Cc = (A + 2) % 3;
                    double plo = 1.0, phi = n3[A];
                    const int qq[2] = {B, Cc};
                    for (int i = 0; i < 2; ++i) {
                        const int q = qq[i];
                        const double r = f.d[q] * f.inv_d[A];
                        if (r != 0.0) {
                            const double t1 = b[A] - b[q] / r, t2 = b[A] + (n3[q] + 1.0 - b[q]) / r;
                            plo = std::max(plo, std::min(t1, t2));
                            phi = std::min(phi, std::max(t1, t2));
                        } else if (!(b[q] > 0.0 && b[q] < n3[q] + 1.0)) {
                            phi = -1.0;
                        }
                    }
                    const long long P0 = std::max(1LL, (long long)std::ceil(plo));
                    const long long P1 = std::min((long long)n3[A], (long long)std::floor(phi));
                    total += std::max(0LL, P1 - P0 + 1);
                }
            }
    }
    *out = total;
    return TT_OK;
}

int tt_basis_matrix(const tt_ctx *c, double *B_host)
{
    if (!c || !B_host) return fail(TT_EINVAL, "null pointer");
    std::memcpy(B_host, c->B.data(), c->B.size() * sizeof(double));
    return TT_OK;
}

static int project_sc(tt_ctx *c, const Scratch &sc, const float *cin, float *I)
{
    if (c->d.sparse_k > 0) {
        hipError_t e;
        {
            KTimer t(c, TT_K_FUSED, sc.timed);
            e = launch_march_fused(c->d, c->d_frames, cin, c->d_sp, c->d_gtab, sc.cT, I, c->stream);
        }
        if (e != hipSuccess) return fail(TT_EHIP, std::string("fused march: ") + hipGetErrorString(e));
        return TT_OK;
    }
    if (sc.pb < 1)
        return fail(TT_EINVAL, "the attached workspace holds no mapped volumes; attach one sized by "
                               "tt_workspace_bytes with a forward batch >= 1");
    for (int s0 = 0; s0 < c->d.S; s0 += sc.pb) {
        const int np = std::min(sc.pb, c->d.S - s0);
        hipError_t e;
        {
            KTimer t(c, TT_K_MAP, sc.timed);
            e = c->precision == TT_MAP_BF16 ? launch_map_bf16(c->d, cin, c->d_Bsw16, s0, np, sc.M, c->stream)
                                            : launch_map_fp32(c->d, cin, c->d_Bsw, s0, np, sc.M, c->stream);
        }
        if (e != hipSuccess) return fail(e == hipErrorNotSupported ? TT_EUNSUPPORTED : TT_EHIP,
                                         std::string("map: ") + hipGetErrorString(e));
        {
            KTimer t(c, TT_K_MARCH, sc.timed);
            e = launch_march(c->d, c->d_frames, sc.M, s0, np, I, c->stream);
        }
        if (e != hipSuccess) return fail(TT_EHIP, std::string("march: ") + hipGetErrorString(e));
    }
    return TT_OK;
}

static int project_impl(tt_ctx *c, const float *cin, float *I)
{
    if (int rc = need_ws(c)) return rc;
    return project_sc(c, attached(c), cin, I);
}

int tt_project(tt_ctx *c, const float *cin, float *I)
{
    if (!c || !cin || !I) return fail(TT_EINVAL, "null pointer");
    return project_impl(c, cin, I);
}

static int backproject_sc(tt_ctx *c, const Scratch &sc, float *g, float beta, const float *cin, double *partials)
{
    hipError_t e;
    {
        KTimer t(c, TT_K_BACKPROJECT, sc.timed);
        e = launch_backproject(c->d, c->d_frames, sc.yf, c->d_Bu, c->d_BuT16, c->precision == TT_MAP_BF16, g, beta,
                               cin, partials, c->stream);
    }
    if (e != hipSuccess) return fail(e == hipErrorNotSupported ? TT_EUNSUPPORTED : TT_EHIP,
                                     std::string("backproject: ") + hipGetErrorString(e));
    return TT_OK;
}

static int backproject_impl(tt_ctx *c, float *g, float beta, const float *cin, double *partials)
{
    if (int rc = need_ws(c)) return rc;
    return backproject_sc(c, attached(c), g, beta, cin, partials);
}

int tt_adjoint(tt_ctx *c, const float *y, float *g, float beta, const float *cin)
{
    if (!c || !y || !g) return fail(TT_EINVAL, "null pointer");
    if (beta != 0.0f && !cin) return fail(TT_EINVAL, "beta != 0 needs c");
    if (int rc = need_ws(c)) return rc;
    {
        KTimer t(c, TT_K_FOLD);
        TT_HIP(launch_fold(c->d, y, c->d.step, c->d_yf, c->stream));
    }
    return backproject_impl(c, g, beta, beta != 0.0f ? cin : nullptr, nullptr);
}

static int loss_grad_sc(tt_ctx *c, const Scratch &sc, const float *cin, const float *data, const float *w,
                        double mu, double *loss, float *grad, float *resid)
{
    float *r = resid ? resid : sc.resid;
    int rc = project_sc(c, sc, cin, r);
    if (rc) return rc;
    const int nb = 1024;
    {
        KTimer t(c, TT_K_RESIDUAL, sc.timed);
        TT_HIP(launch_residual_fold(c->d, r, data, w, r, sc.yf, sc.part, nb, c->stream));
        TT_HIP(launch_sum_partials(sc.part, nb, loss, 1.0, 0, c->stream));
    }
    double *p2 = sc.part + nb;
    rc = backproject_sc(c, sc, grad, (float)(2.0 * mu), cin, p2);
    if (rc) return rc;
    TT_HIP(launch_sum_partials(p2, backproject_blocks(c->d), loss, mu, 1, c->stream));
    return TT_OK;
}

int tt_loss_grad(tt_ctx *c, const float *cin, const float *data, const float *w, double mu, double *loss,
                 float *grad, float *resid)
{
    if (!c || !cin || !data || !loss || !grad) return fail(TT_EINVAL, "null pointer");
    if (!(mu >= 0.0) || !std::isfinite(mu)) return fail(TT_EINVAL, "mu must be finite and >= 0");
    if (int rc = need_ws(c)) return rc;
    return loss_grad_sc(c, attached(c), cin, data, w, mu, loss, grad, resid);
}

int tt_loss_grad_noalloc(tt_ctx *c, const float *cin, const float *data, const float *w, double mu, double *loss,
                         float *grad, float *resid)
{
    if (!c || !cin || !data || !loss || !grad) return fail(TT_EINVAL, "null pointer");
    if (!(mu >= 0.0) || !std::isfinite(mu)) return fail(TT_EINVAL, "mu must be finite and >= 0");
    char *base = static_cast<char *>(static_scratch(c->device));
    if (!base) return fail(TT_EHIP, "the library's static scratch is not available on device " +
                                        std::to_string(c->device));
    // same layout as an attached workspace, the batch as large as the array allows
    WsLayout L = ws_layout(c, 0);
    if (resid) {  // the residual goes to the caller's buffer: no data-sized scratch
        const size_t shift = L.cT - L.resid;
        L.cT -= shift;
        L.M -= shift;
        L.total -= shift;
    }
    const size_t cap = kStaticScratchBytes;
    const long long fit = cap > L.total ? (long long)((cap - L.total) / c->per_proj) : 0;
    const bool fused = c->d.sparse_k > 0;  // the fused forward maps nothing
    const int pb = fused ? 0 : batch_round_down(c, fit);
    if (fused ? L.total > cap : pb < batch_min(c))
        return fail(TT_ENOMEM, "problem needs " +
                                   std::to_string(L.total + (fused ? 0 : c->per_proj * (size_t)batch_min(c))) +
                                   " bytes of scratch, above the static limit of " + std::to_string(cap) +
                                   " bytes; use tt_loss_grad with a workspace");
    Scratch sc;
    sc.part = reinterpret_cast<double *>(base + L.part);
    sc.yf = reinterpret_cast<float *>(base + L.yf);
    sc.resid = resid ? nullptr : reinterpret_cast<float *>(base + L.resid);
    sc.M = reinterpret_cast<float *>(base + L.M);
    sc.cT = reinterpret_cast<float *>(base + L.cT);
    sc.pb = pb;
    sc.timed = false;
    // the map writes interior voxels only; the array holds whatever the last
    // call on this device left there, so the zero border is restored each time
    if (pb > 0) TT_HIP(launch_zero(sc.M, c->per_proj * (size_t)pb, c->stream));
    return loss_grad_sc(c, sc, cin, data, w, mu, loss, grad, resid);
}

// ---------------------------------------------------------------------------
// Normal-operator diagonal of the isotropic field: d = (A^T A u)_{v,0}
// ---------------------------------------------------------------------------
struct NormalWork {
    float *u, *I, *g;
    char *red;
    size_t total;
};
static NormalWork normal_layout(const tt_ctx *c, char *base)
{
    NormalWork L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    L.u = reinterpret_cast<float *>(take(sizeof(float) * n_coef(c)));
    L.I = reinterpret_cast<float *>(take(sizeof(float) * n_data(c)));
    L.g = reinterpret_cast<float *>(take(sizeof(float) * n_coef(c)));
    L.red = take(std::max<size_t>(ball_median_work_bytes(), 1024 * sizeof(float)) + 256);
    L.total = off;
    return L;
}

int64_t tt_normal_work_bytes(const tt_ctx *c)
{
    if (!c) return fail(TT_EINVAL, "ctx is null");
    return (int64_t)normal_layout(c, nullptr).total;
}

// g = A^T A u for the unit isotropic field u (g may alias nothing in the work area).
static int normal_iso(tt_ctx *c, const NormalWork &L, float *g)
{
    const long long nvox = (long long)c->d.nx * c->d.ny * c->d.nz;
    TT_HIP(launch_fill_iso(L.u, nvox, c->d.C, c->stream));
    int rc = project_impl(c, L.u, L.I);
    if (rc) return rc;
    return tt_adjoint(c, L.I, g, 0.0f, nullptr);
}

static int check_work(const tt_ctx *c, void *work, size_t bytes)
{
    if (!work) return fail(TT_EINVAL, "work buffer is null");
    if (reinterpret_cast<uintptr_t>(work) % 256) return fail(TT_EINVAL, "work buffer must be 256-byte aligned");
    if (bytes < normal_layout(c, nullptr).total) return fail(TT_EINVAL, "work buffer below tt_normal_work_bytes");
    return TT_OK;
}

int tt_kappa(tt_ctx *c, double radius, void *work, size_t work_bytes, double *kappa)
{
    if (!c || !kappa) return fail(TT_EINVAL, "null pointer");
    if (!(radius >= 0.0) || !std::isfinite(radius)) return fail(TT_EINVAL, "radius must be finite and >= 0");
    if (int rc = check_work(c, work, work_bytes)) return rc;
    const NormalWork L = normal_layout(c, static_cast<char *>(work));
    int rc = normal_iso(c, L, L.g);
    if (rc) return rc;
    float *med = reinterpret_cast<float *>(L.red + ball_median_work_bytes());
    TT_HIP(launch_ball_median(L.g, c->d.nx, c->d.ny, c->d.nz, c->d.C, 0, radius, L.red, med, c->stream));
    float h = 0.0f;
    TT_HIP(hipMemcpyAsync(&h, med, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    TT_HIP(hipStreamSynchronize(c->stream));
    if (!std::isfinite(h)) return fail(TT_ENONFINITE, "no voxel centre inside the support ball");
    *kappa = h;
    return TT_OK;
}

int tt_voxel_preconditioner(tt_ctx *c, double floor_frac, float *p, void *work, size_t work_bytes)
{
    if (!c || !p) return fail(TT_EINVAL, "null pointer");
    if (!(floor_frac > 0.0) || !std::isfinite(floor_frac)) return fail(TT_EINVAL, "floor_frac must be > 0");
    if (int rc = check_work(c, work, work_bytes)) return rc;
    const NormalWork L = normal_layout(c, static_cast<char *>(work));
    int rc = normal_iso(c, L, p);
    if (rc) return rc;
    TT_HIP(launch_voxel_precond(p, (long long)c->d.nx * c->d.ny * c->d.nz, c->d.C, (float)floor_frac,
                                reinterpret_cast<float *>(L.red), c->stream));
    return TT_OK;
}

int64_t tt_channel_stats_work_len(void) { return (int64_t)chstats_work_doubles(); }

int tt_channel_stats(const float *x, int64_t nvox, int cstride, int nch, float pre_scale, float *shift, float *scale,
                     double *work, int64_t work_len, void *stream)
{
    if (!x || !shift || !scale || !work) return fail(TT_EINVAL, "null pointer");
    if (nvox < 1 || nch < 1 || nch > 64 || cstride < nch) return fail(TT_ESHAPE, "need nvox >= 1, 1 <= nch <= 64 and cstride >= nch");
    if (!std::isfinite(pre_scale)) return fail(TT_EINVAL, "pre_scale must be finite");
    if (work_len < (int64_t)chstats_work_doubles()) return fail(TT_EINVAL, "work below tt_channel_stats_work_len()");
    TT_HIP(launch_channel_stats(x, nvox, cstride, nch, pre_scale, shift, scale, work, (hipStream_t)stream));
    return TT_OK;
}

// ---------------------------------------------------------------------------
// L-BFGS
// ---------------------------------------------------------------------------
void tt_lbfgs_destroy(tt_lbfgs *st)
{
    if (!st) return;
    if (st->ctx) hipStreamSynchronize(st->ctx->stream);  // queued kernels may still use the workspace
    delete st;
}

// Solver workspace: m + 1 slots each for s and y, two gradients and the
// direction (coefficient-sized), residual and A d (data-sized), the float64 /
// int state and the reduction partials, each 256-byte aligned.
static size_t lbfgs_layout(const tt_ctx *c, int m, tt_lbfgs *st, char *base)
{
    const size_t vb = align256(sizeof(float) * n_coef(c)), db = align256(sizeof(float) * n_data(c));
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    for (int i = 0; i <= m; ++i) {
        char *ps = take(vb), *py = take(vb);
        if (st) {
            st->s[i] = reinterpret_cast<float *>(ps);
            st->y[i] = reinterpret_cast<float *>(py);
        }
    }
    char *g0 = take(vb), *g1 = take(vb), *d = take(vb), *r = take(db), *q = take(db);
    char *sd = take(sizeof(double) * kStateDoubles), *si = take(sizeof(int) * kStateInts);
    char *part = take(sizeof(double) * (kMaxBasis + 1) * lbfgs_blocks());
    if (st) {
        st->g[0] = reinterpret_cast<float *>(g0);
        st->g[1] = reinterpret_cast<float *>(g1);
        st->d = reinterpret_cast<float *>(d);
        st->r = reinterpret_cast<float *>(r);
        st->q = reinterpret_cast<float *>(q);
        st->st = reinterpret_cast<double *>(sd);
        st->ist = reinterpret_cast<int *>(si);
        st->part = reinterpret_cast<double *>(part);
    }
    return off;
}

int64_t tt_lbfgs_workspace_bytes(const tt_ctx *c, int m)
{
    if (!c) return fail(TT_EINVAL, "ctx is null");
    if (m < 1 || m > kMaxM) return fail(TT_EUNSUPPORTED, "history m must be 1.." + std::to_string(kMaxM));
    return (int64_t)lbfgs_layout(c, m, nullptr, nullptr);
}

int tt_lbfgs_create(tt_ctx *c, int m, void *work, size_t bytes, tt_lbfgs **out)
{
    if (!out) return fail(TT_EINVAL, "out is null");
    *out = nullptr;
    if (!c) return fail(TT_EINVAL, "ctx is null");
    if (m < 1 || m > kMaxM) return fail(TT_EUNSUPPORTED, "history m must be 1.." + std::to_string(kMaxM));
    if (!work) return fail(TT_EINVAL, "workspace is null");
    if (reinterpret_cast<uintptr_t>(work) % 256) return fail(TT_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = lbfgs_layout(c, m, nullptr, nullptr);
    if (bytes < need)
        return fail(TT_EINVAL, "L-BFGS workspace of " + std::to_string(bytes) + " bytes is below the " +
                                   std::to_string(need) + " needed");
    tt_lbfgs *st = new (std::nothrow) tt_lbfgs();
    if (!st) return fail(TT_ENOMEM, "host allocation failed");
    st->ctx = c;
    st->m = m;
    st->s.assign(m + 1, nullptr);
    st->y.assign(m + 1, nullptr);
    lbfgs_layout(c, m, st, static_cast<char *>(work));
    // history slots start at zero (masked out until filled, but never read uninitialised)
    const size_t vb = sizeof(float) * n_coef(c);
    for (int i = 0; i <= m; ++i) {
        if (hipMemsetAsync(st->s[i], 0, vb, c->stream) != hipSuccess ||
            hipMemsetAsync(st->y[i], 0, vb, c->stream) != hipSuccess) {
            delete st;
            return fail(TT_EHIP, "clearing the L-BFGS history failed");
        }
    }
    *out = st;
    return TT_OK;
}

int tt_lbfgs_init(tt_lbfgs *st, float *cin, const float *data, const float *w, double mu)
{
    if (!st || !cin || !data) return fail(TT_EINVAL, "null pointer");
    if (!(mu >= 0.0) || !std::isfinite(mu)) return fail(TT_EINVAL, "mu must be finite and >= 0");
    tt_ctx *c = st->ctx;
    hipStream_t s = c->stream;
    st->c = cin;
    st->data = data;
    st->w = w;
    st->mu = mu;
    st->gcur = 0;
    const int m = st->m, ns = m + 1, gi = 2 * ns;
    const long long n = n_coef(c), nd = n_data(c);
    // host-prepared initial state: empty ring, gamma = 1
    std::vector<double> h(kStateDoubles, 0.0);
    std::vector<int> hi(kStateInts, 0);
    h[kGamma] = 1.0;
    hi[kMask2] = 1;  // first list entry (the gradient) for the initial dot product
    TT_HIP(hipMemcpyAsync(st->st, h.data(), sizeof(double) * kStateDoubles, hipMemcpyHostToDevice, s));
    TT_HIP(hipMemcpyAsync(st->ist, hi.data(), sizeof(int) * kStateInts, hipMemcpyHostToDevice, s));
    int rc = project_impl(c, cin, st->r);
    if (rc) return rc;
    TT_HIP(launch_residual_fold(c->d, st->r, data, w, st->r, c->d_yf, c->d_part, 1024, s));
    TT_HIP(launch_sum_partials(c->d_part, 1024, st->st + kLossR, 1.0, 0, s));
    TT_HIP(lbfgs_wnorm2(st->r, nullptr, nd, st->part, st->st + kRR, s));
    TT_HIP(lbfgs_wnorm2(data, nullptr, nd, st->part, st->st + kDataNorm2, s));
    double *p2 = c->d_part + 1024;
    rc = backproject_impl(c, st->g[0], (float)(2.0 * mu), cin, p2);
    if (rc) return rc;
    TT_HIP(launch_sum_partials(p2, backproject_blocks(c->d), st->st + kCC, 1.0, 0, s));
    const float *gl[1] = {st->g[0]};
    TT_HIP(lbfgs_multidot(st->g[0], gl, 1, st->ist + kMask2, n, st->part, st->st + kDotsG, s));
    // G[g][g] = g . g  (copied on the device)
    TT_HIP(hipMemcpyAsync(st->st + kGram + gi * kMaxBasis + gi, st->st + kDotsG, sizeof(double),
                          hipMemcpyDeviceToDevice, s));
    st->inited = true;
    return TT_OK;
}

static int lbfgs_step_impl(tt_lbfgs *st, const float *user_d)
{
    if (!st || !st->inited) return fail(TT_EINVAL, "solver not initialised");
    tt_ctx *c = st->ctx;
    hipStream_t s = c->stream;
    const int m = st->m, ns = m + 1;
    const long long n = n_coef(c);
    float *gold = st->g[st->gcur], *gnew = st->g[1 - st->gcur];
    std::vector<const float *> basis(2 * ns + 2);
    for (int i = 0; i < ns; ++i) {
        basis[i] = st->s[i];
        basis[ns + i] = st->y[i];
    }
    basis[2 * ns] = gold;
    basis[2 * ns + 1] = gnew;
    if (user_d) {
        // caller's direction: d . b_a for the valid history and the gradient, and d . d
        {
            KTimer t(c, TT_K_PLAN);
            TT_HIP(lbfgs_plan_user_direction(st->st, st->ist, m, s));
        }
        KTimer t(c, TT_K_VECTOR);
        TT_HIP(hipMemcpyAsync(st->d, user_d, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
        TT_HIP(lbfgs_multidot(st->d, basis.data(), 2 * ns + 1, st->ist + kMask, n, st->part, st->st + kDotsD, s));
        TT_HIP(lbfgs_wnorm2(st->d, nullptr, n, st->part, st->st + kDotsD + kMaxBasis, s));
    } else {
        {
            KTimer t(c, TT_K_PLAN);
            TT_HIP(lbfgs_plan_direction(st->st, st->ist, m, s));
        }
        KTimer t(c, TT_K_VECTOR);
        TT_HIP(lbfgs_combine(basis.data(), 2 * ns + 1, st->st + kCoef, st->ist + kMask, n, st->d, st->part,
                             st->st + kDotsD, s));
    }
    int rc = project_impl(c, st->d, st->q);
    if (rc) return rc;
    {
        KTimer t(c, TT_K_VECTOR);
        TT_HIP(lbfgs_wnorm2(st->q, st->w, n_data(c), st->part, st->st + kQQ, s));
    }
    {
        KTimer t(c, TT_K_PLAN);
        TT_HIP(lbfgs_plan_alpha(st->st, st->ist, m, st->mu, s));
    }
    {
        KTimer t(c, TT_K_VECTOR);
        TT_HIP(lbfgs_update_c(st->c, st->d, basis.data(), ns, st->st, st->ist, n, s));
    }
    {
        KTimer t(c, TT_K_RESIDUAL);
        TT_HIP(lbfgs_resid_update(c->d, st->r, st->q, st->w, st->st, c->d_yf, st->part, st->st + kLossR, s));
    }
    double *p2 = c->d_part + 1024;
    rc = backproject_impl(c, gnew, (float)(2.0 * st->mu), st->c, p2);
    if (rc) return rc;
    {
        KTimer t(c, TT_K_VECTOR);
        TT_HIP(launch_sum_partials(p2, backproject_blocks(c->d), st->st + kCC, 1.0, 0, s));
        // dots of the new gradient with the history, and y[cand] = g_new - g_old in the same pass
        TT_HIP(lbfgs_multidot(gnew, basis.data(), 2 * ns + 2, st->ist + kMask2, n, st->part, st->st + kDotsG, s,
                              basis.data() + ns, ns, st->ist, 2 * ns));
    }
    {
        KTimer t(c, TT_K_PLAN);
        TT_HIP(lbfgs_plan_update(st->st, st->ist, m, st->mu, s));
    }
    st->gcur = 1 - st->gcur;
    return TT_OK;
}

int tt_lbfgs_step(tt_lbfgs *st) { return lbfgs_step_impl(st, nullptr); }

int tt_lbfgs_step_direction(tt_lbfgs *st, const float *d_dev)
{
    if (!d_dev) return fail(TT_EINVAL, "direction is null");
    return lbfgs_step_impl(st, d_dev);
}

int tt_lbfgs_query(tt_lbfgs *st, double *out4)
{
    if (!st || !out4) return fail(TT_EINVAL, "null pointer");
    if (!st->inited) return fail(TT_EINVAL, "solver not initialised");
    TT_HIP(hipStreamSynchronize(st->ctx->stream));
    double h[kStateDoubles];
    int hi[kStateInts];
    TT_HIP(hipMemcpy(h, st->st, sizeof h, hipMemcpyDeviceToHost));
    TT_HIP(hipMemcpy(hi, st->ist, sizeof hi, hipMemcpyDeviceToHost));
    out4[0] = h[kLossR] + st->mu * h[kCC];
    out4[1] = std::sqrt(h[kRR]);
    out4[2] = std::sqrt(h[kDataNorm2]);
    out4[3] = hi[kAccepted];
    if (!std::isfinite(out4[0]) || !std::isfinite(out4[1])) return fail(TT_ENONFINITE, "non-finite loss or residual");
    return TT_OK;
}

int tt_lbfgs_refresh(tt_lbfgs *st)
{
    if (!st || !st->inited) return fail(TT_EINVAL, "solver not initialised");
    tt_ctx *c = st->ctx;
    hipStream_t s = c->stream;
    int rc = project_impl(c, st->c, st->r);
    if (rc) return rc;
    {
        KTimer t(c, TT_K_RESIDUAL);
        TT_HIP(launch_residual_fold(c->d, st->r, st->data, st->w, st->r, c->d_yf, c->d_part, 1024, s));
        TT_HIP(launch_sum_partials(c->d_part, 1024, st->st + kLossR, 1.0, 0, s));
    }
    KTimer t(c, TT_K_VECTOR);
    TT_HIP(lbfgs_wnorm2(st->r, nullptr, n_data(c), st->part, st->st + kRR, s));
    return TT_OK;
}

int tt_lbfgs_run(tt_lbfgs *st, int max_iter, double rel_tol, double *hist, int *iters_out)
{
    if (!st) return fail(TT_EINVAL, "null pointer");
    if (max_iter < 0) return fail(TT_EINVAL, "max_iter must be >= 0");
    int it = 0;
    double q[4];
    int rc = tt_lbfgs_query(st, q);
    for (; rc == TT_OK && it < max_iter; ++it) {
        if (q[1] <= rel_tol * q[2]) break;
        rc = tt_lbfgs_step(st);
        if (rc == TT_OK) rc = tt_lbfgs_query(st, q);
        if (rc == TT_OK && hist) {
            hist[2 * it] = q[0];
            hist[2 * it + 1] = q[1] / q[2];
        }
    }
    if (iters_out) *iters_out = it;
    return rc;
}

// ---------------------------------------------------------------------------
// warm-start network layers
// ---------------------------------------------------------------------------
static bool net_channels_ok(int ci, int co) { return (ci == 32 || ci == 64) && (co == 32 || co == 64); }

int64_t tt_conv3d_weight_elems(int ci, int co)
{
    if (!net_channels_ok(ci, co)) return fail(TT_EUNSUPPORTED, "channels must be 32 or 64");
    return (int64_t)27 * ci * co;
}

int tt_conv3d_swizzle(const float *w, int ci, int co, uint16_t *wf, uint16_t *wd, void *stream)
{
    if (!w || !wf || !wd) return fail(TT_EINVAL, "null pointer");
    if (!net_channels_ok(ci, co)) return fail(TT_EUNSUPPORTED, "channels must be 32 or 64");
    TT_HIP(net_swizzle(w, ci, co, wf, wd, (hipStream_t)stream));
    return TT_OK;
}

int tt_conv3d(int epi, int ci, int co, const uint16_t *x, const uint16_t *wsw, const float *bias, const uint16_t *mask,
              void *y, int n, int X, int Y, int Z, void *stream)
{
    if (!x || !wsw || !y) return fail(TT_EINVAL, "null pointer");
    if (epi < 0 || epi > 2) return fail(TT_EINVAL, "bad epilogue");
    if (epi != TT_CONV_MASK_BF16 && !bias) return fail(TT_EINVAL, "bias is null");
    if (epi == TT_CONV_MASK_BF16 && !mask) return fail(TT_EINVAL, "mask is null");
    if (!net_channels_ok(ci, co)) return fail(TT_EUNSUPPORTED, "channels must be 32 or 64");
    if (n < 1 || X < 1 || Y < 1 || Z < 1) return fail(TT_ESHAPE, "empty volume");
    TT_HIP(net_conv(epi, ci, co, x, wsw, bias, mask, y, n, X, Y, Z, (hipStream_t)stream));
    return TT_OK;
}

size_t tt_conv3d_wgrad_work_bytes(int ci, int co, int n, int X, int Y, int Z)
{
    if (!net_channels_ok(ci, co) || n < 1 || X < 1 || Y < 1 || Z < 1) return 0;
    return net_wgrad_work_bytes(ci, co, n, X, Y, Z);
}

int tt_conv3d_wgrad(int ci, int co, const uint16_t *x, const uint16_t *gy, int n, int X, int Y, int Z, float *work,
                    size_t work_bytes, float *gw, float *gb, void *stream)
{
    if (!x || !gy || !work || !gw) return fail(TT_EINVAL, "null pointer");
    if (!net_channels_ok(ci, co)) return fail(TT_EUNSUPPORTED, "channels must be 32 or 64");
    if (n < 1 || X < 1 || Y < 1 || Z < 1) return fail(TT_ESHAPE, "empty volume");
    if (work_bytes < net_wgrad_work_bytes(ci, co, n, X, Y, Z)) return fail(TT_EINVAL, "work buffer too small");
    TT_HIP(net_wgrad(ci, co, x, gy, n, X, Y, Z, work, gw, gb, (hipStream_t)stream));
    return TT_OK;
}

int tt_adam(float *w, const float *g, float *m, float *v, int64_t n, int t, float lr, float b1, float b2, float eps,
            void *stream)
{
    if (!w || !g || !m || !v) return fail(TT_EINVAL, "null pointer");
    if (n < 0 || t < 1) return fail(TT_EINVAL, "n >= 0 and t >= 1 required");
    if (n == 0) return TT_OK;
    TT_HIP(net_adam(w, g, m, v, n, t, lr, b1, b2, eps, (hipStream_t)stream));
    return TT_OK;
}

int tt_mse(const float *y, const float *t, int64_t nvox, int cpad, int creal, float scale, uint16_t *gy, double *loss,
           double *work, int64_t work_len, void *stream)
{
    if (!y || !t || !loss || !work) return fail(TT_EINVAL, "null pointer");
    if (nvox < 1 || creal < 1 || cpad < creal) return fail(TT_ESHAPE, "bad sizes");
    if (work_len < 1024) return fail(TT_EINVAL, "work must hold 1024 doubles");
    TT_HIP(net_mse(y, t, nvox, cpad, creal, scale, gy, work, 1024, loss, (hipStream_t)stream));
    return TT_OK;
}

int tt_pack_bf16(const float *x, int64_t nvox, int cin, int cpad, float pre_scale, const float *shift,
                 const float *scale, uint16_t *out, void *stream)
{
    if (!x || !out) return fail(TT_EINVAL, "null pointer");
    if (nvox < 0 || cin < 1 || cpad < cin) return fail(TT_ESHAPE, "bad sizes");
    if (!std::isfinite(pre_scale)) return fail(TT_EINVAL, "pre_scale must be finite");
    if (nvox == 0) return TT_OK;
    TT_HIP(net_pack(x, nvox, cin, cpad, pre_scale, shift, scale, out, (hipStream_t)stream));
    return TT_OK;
}

int tt_tile_gather(const float *vol, int X, int Y, int Z, int cv, int cin, int cpad, const int *ox, int ntx,
                   const int *oy, int nty, const int *oz, int ntz, int T, float pre_scale, const float *shift,
                   const float *scale, int t0, int nt, uint16_t *out, void *stream)
{
    if (!vol || !ox || !oy || !oz || !out) return fail(TT_EINVAL, "null pointer");
    if (X < 1 || Y < 1 || Z < 1 || cin < 1 || cv < cin || cpad < cin || T < 1 || ntx < 1 || nty < 1 || ntz < 1)
        return fail(TT_ESHAPE, "bad sizes");
    if (t0 < 0 || nt < 0 || t0 + nt > ntx * nty * ntz) return fail(TT_EINVAL, "tile range out of bounds");
    if (!std::isfinite(pre_scale)) return fail(TT_EINVAL, "pre_scale must be finite");
    if (nt == 0) return TT_OK;
    TT_HIP(net_tile_gather(vol, X, Y, Z, cv, cin, cpad, ox, ntx, oy, nty, oz, ntz, T, pre_scale, shift, scale, t0, nt,
                           out, (hipStream_t)stream));
    return TT_OK;
}

int tt_tile_blend(const float *y, int cy, int creal, int X, int Y, int Z, const int *ox, int ntx, const int *oy,
                  int nty, const int *oz, int ntz, int T, int ramp, int cout, float *out, void *stream)
{
    if (!y || !ox || !oy || !oz || !out) return fail(TT_EINVAL, "null pointer");
    if (X < 1 || Y < 1 || Z < 1 || creal < 1 || cy < creal || cout < creal || T < 1 || ramp < 1 || ntx < 1 ||
        nty < 1 || ntz < 1)
        return fail(TT_ESHAPE, "bad sizes");
    TT_HIP(net_tile_blend(y, cy, creal, X, Y, Z, ox, ntx, oy, nty, oz, ntz, T, ramp, cout, out, (hipStream_t)stream));
    return TT_OK;
}

static int check_partials(const double *partials, int64_t len)
{
    if (!partials) return fail(TT_EINVAL, "partials is null (a value needs TT_REDUCE_WORK doubles)");
    if (len < kReduceBlocks) return fail(TT_EINVAL, "partials must hold TT_REDUCE_WORK doubles");
    return TT_OK;
}

int tt_laplacian_reg(const float *c, int nx, int ny, int nz, int C, double lambda, float *work, float *grad,
                     double *value, double *partials, int64_t partials_len, void *stream)
{
    static_assert(TT_REDUCE_WORK == kReduceBlocks, "partials length");
    if (!c || !work || !grad) return fail(TT_EINVAL, "null pointer");
    if (value)
        if (int rc = check_partials(partials, partials_len)) return rc;
    if (nx < 1 || ny < 1 || nz < 1 || C < 1) return fail(TT_ESHAPE, "sizes must be >= 1");
    if (C > kLapMaxC || (long long)nx * ny * nz > 0x7fffffffLL)
        return fail(TT_EUNSUPPORTED, "C above " + std::to_string(kLapMaxC) + " or nx * ny * nz above 2^31");
    if (!std::isfinite(lambda)) return fail(TT_EINVAL, "lambda must be finite");
    TT_HIP(launch_laplacian_reg(c, nx, ny, nz, C, lambda, work, grad, value, partials, (hipStream_t)stream));
    return TT_OK;
}

int tt_huber_reg(const float *c, int64_t n, double delta, double lambda, float *grad, double *value, double *partials,
                 int64_t partials_len, void *stream)
{
    if (n < 0) return fail(TT_ESHAPE, "n must be >= 0");
    if (value)
        if (int rc = check_partials(partials, partials_len)) return rc;
    if (!(delta > 0.0) || !std::isfinite(delta) || !std::isfinite(lambda)) return fail(TT_EINVAL, "bad delta or lambda");
    if (n == 0) return TT_OK;
    if (!c || !grad) return fail(TT_EINVAL, "null pointer");
    TT_HIP(launch_huber_reg(c, n, delta, lambda, grad, value, partials, (hipStream_t)stream));
    return TT_OK;
}

int tt_huber_loss(const float *I, const float *data, const float *w, int64_t n, double delta, float *y,
                  double *value, double *partials, int64_t partials_len, void *stream)
{
    if (n < 0) return fail(TT_ESHAPE, "n must be >= 0");
    if (value)
        if (int rc = check_partials(partials, partials_len)) return rc;
    if (!(delta > 0.0) || !std::isfinite(delta)) return fail(TT_EINVAL, "delta must be > 0");
    if (n == 0) return TT_OK;
    if (!I || !data || !y) return fail(TT_EINVAL, "null pointer");
    TT_HIP(launch_huber_loss(I, data, w, n, delta, y, value, partials, (hipStream_t)stream));
    return TT_OK;
}

int tt_sumsq(const float *x, int64_t n, double scale, double *value, double *partials, int64_t partials_len,
             void *stream)
{
    if (n < 0) return fail(TT_ESHAPE, "n must be >= 0");
    if (!value) return fail(TT_EINVAL, "null value");
    if (int rc = check_partials(partials, partials_len)) return rc;
    if (n == 0) return TT_OK;
    if (!x) return fail(TT_EINVAL, "null pointer");
    TT_HIP(launch_sumsq(x, n, scale, value, partials, (hipStream_t)stream));
    return TT_OK;
}

int tt_gd_step(float *c, float *y, const float *g, const float *precond, int64_t n, float step, float momentum,
               void *stream)
{
    if (n < 0) return fail(TT_ESHAPE, "n must be >= 0");
    if (!std::isfinite(step) || !std::isfinite(momentum)) return fail(TT_EINVAL, "bad step or momentum");
    if (n == 0) return TT_OK;
    if (!c || !y || !g) return fail(TT_EINVAL, "null pointer");
    TT_HIP(launch_nesterov(c, y, g, precond, n, step, momentum, (hipStream_t)stream));
    return TT_OK;
}

int tt_tensor_properties(const float *c, int64_t n_vox, int ell_max, float *out, void *stream)
{
    if (ell_max < 0 || ell_max % 2) return fail(TT_EINVAL, "ell_max must be even and >= 0");
    if (ell_max > 16) return fail(TT_EUNSUPPORTED, "ell_max above 16");
    if (n_vox < 0) return fail(TT_ESHAPE, "n_vox must be >= 0");
    if (n_vox == 0) return TT_OK;  // nothing to read or write: any pointers accepted
    if (!c || !out) return fail(TT_EINVAL, "null pointer");
    if ((reinterpret_cast<uintptr_t>(c) | reinterpret_cast<uintptr_t>(out)) % 16)
        return fail(TT_EINVAL, "c and out must be 16-byte aligned");
    static_assert(TT_PROP_FIELDS == kPropFields, "field count");
    TT_HIP(launch_tensor_props(c, n_vox, num_coeffs(ell_max), out, (hipStream_t)stream));
    return TT_OK;
}

}  // extern "C"
