// Host-side float64 precompute: spherical harmonics, goniometer rotations,
// ray frames and segment-averaged basis constants.
//
// Spherical harmonics (paper section 3.2): real, orthonormal, even orders.
// Evaluated with the fully normalised associated-Legendre recurrence
//   Pbar_mm     = Pbar_{m-1,m-1} s sqrt((2m+1)/(2m)),     Pbar_00 = 1/sqrt(4 pi)
//   Pbar_{m+1,m} = x sqrt(2m+3) Pbar_mm
//   Pbar_lm     = a_lm (x Pbar_{l-1,m} - Pbar_{l-2,m} / a_{l-1,m}),
//   a_lm        = sqrt((4 l^2 - 1) / (l^2 - m^2)),
// and cos(m phi), sin(m phi) by the Chebyshev recurrence from the direction's
// x/s and y/s, so no angle is ever formed.  Y_l0 = Pbar_l0,
// Y_lm = sqrt2 Pbar_lm cos(m phi), Y_l,-m = sqrt2 Pbar_lm sin(m phi) (m > 0),
// without the Condon-Shortley phase; index i(l, m) = l(l-1)/2 + l + m.
//
// Goniometer (section 2): R_s = R_beta(beta_s) R_alpha(alpha_s), composed here
// as unit quaternions.  Ray frame of projection s in sample coordinates:
// e_j = R^T j, e_k = R^T k, d = R^T p (Eq. real_space_geom), origin of pixel
// (0, 0) at -((nj-1)/2 + dj) e_j - ((nk-1)/2 + dk) e_k.
//
// Basis constants (Eq. projection_matrix): mean of Y_i(R_s^T q(phi)) over the
// n_sub midpoint nodes of segment c, q(phi) = cos(phi) q0 + sin(phi) q90
// (small-angle form of Eq. 1), segment c centred at c * span / n_seg.
#include "tt_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace tt {

int num_coeffs(int ell_max) { return (ell_max / 2 + 1) * (ell_max + 1); }

int basis_count(const Geometry &g) { return g.basis == TT_BASIS_SH ? num_coeffs(g.ell_max) : (int)(g.dirs.size() / 3); }

// Kernel basis functions at unit direction q (Gaussian kernels or nearest
// neighbour on the grid g.dirs), antipodally symmetric.
static void kernel_eval(const Geometry &g, const double *q, double *out)
{
    const int n = (int)(g.dirs.size() / 3);
    int nearest = 0;
    double best = -1.0;
    for (int i = 0; i < n; ++i) {
        const double *d = &g.dirs[3 * i];
        const double c = std::min(1.0, std::fabs(d[0] * q[0] + d[1] * q[1] + d[2] * q[2]));
        if (g.basis == TT_BASIS_GK) {
            const double w = std::acos(c);
            out[i] = std::exp(-0.5 * w * w / (g.kernel_width * g.kernel_width));
        } else {
            out[i] = 0.0;
            if (c > best) {
                best = c;
                nearest = i;
            }
        }
    }
    if (g.basis == TT_BASIS_NN) out[nearest] = 1.0;
}

void sh_eval_one(int ell_max, const double *dir, double *out)
{
    const double kFourPi = 4.0 * M_PI;
    double r = std::sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double x = dir[2] / r;
    double sx = dir[0] / r, sy = dir[1] / r;
    double s = std::sqrt(sx * sx + sy * sy);
    double cphi = 1.0, sphi = 0.0;
    if (s > 0.0) {
        cphi = sx / s;
        sphi = sy / s;
    }
    // Pbar[l][m] for m <= l <= ell_max (small, on the stack)
    double P[17][17];
    P[0][0] = 1.0 / std::sqrt(kFourPi);
    for (int m = 1; m <= ell_max; ++m) P[m][m] = P[m - 1][m - 1] * s * std::sqrt((2.0 * m + 1.0) / (2.0 * m));
    for (int m = 0; m < ell_max; ++m) P[m + 1][m] = x * std::sqrt(2.0 * m + 3.0) * P[m][m];
    for (int m = 0; m <= ell_max; ++m)
        for (int l = m + 2; l <= ell_max; ++l) {
            double a = std::sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
            double ap = std::sqrt((4.0 * (l - 1) * (l - 1) - 1.0) / ((double)(l - 1) * (l - 1) - (double)m * m));
            P[l][m] = a * (x * P[l - 1][m] - P[l - 2][m] / ap);
        }
    double cm[17], sm[17];
    cm[0] = 1.0;
    sm[0] = 0.0;
    for (int m = 1; m <= ell_max; ++m) {
        cm[m] = cm[m - 1] * cphi - sm[m - 1] * sphi;
        sm[m] = sm[m - 1] * cphi + cm[m - 1] * sphi;
    }
    const double r2 = std::sqrt(2.0);
    int i = 0;
    for (int l = 0; l <= ell_max; l += 2) {
        for (int m = l; m >= 1; --m) out[i++] = r2 * P[l][m] * sm[m];
        out[i++] = P[l][0];
        for (int m = 1; m <= l; ++m) out[i++] = r2 * P[l][m] * cm[m];
    }
}

namespace {

struct Quat {
    double w, x, y, z;
};

Quat axis_angle(const double *axis, double th)
{
    double n = std::sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
    double h = 0.5 * th, sh = std::sin(h) / n;
    return {std::cos(h), axis[0] * sh, axis[1] * sh, axis[2] * sh};
}

Quat mul(const Quat &a, const Quat &b)
{
    return {a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z,
            a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
            a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x,
            a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}

// R^T v for the rotation of unit quaternion q: rotate v by the conjugate.
void rotate_inverse(const Quat &q, const double *v, double *out)
{
    // v' = v + 2 w (u x v) + 2 u x (u x v) with u = -q.xyz, w = q.w
    double ux = -q.x, uy = -q.y, uz = -q.z;
    double tx = 2.0 * (uy * v[2] - uz * v[1]);
    double ty = 2.0 * (uz * v[0] - ux * v[2]);
    double tz = 2.0 * (ux * v[1] - uy * v[0]);
    out[0] = v[0] + q.w * tx + (uy * tz - uz * ty);
    out[1] = v[1] + q.w * ty + (uz * tx - ux * tz);
    out[2] = v[2] + q.w * tz + (ux * ty - uy * tx);
}

// Upper and lower chains of the shadow of the cube [-1, 1]^3 (the zonotope
// spanned by the three projected edges) as (slope, intercept) lines in y.
void cube_shadow(const double *ej, const double *ek, float *hull)
{
    std::vector<std::pair<double, double>> pts;
    for (int m = 0; m < 8; ++m) {
        double sx = (m & 1) ? 1 : -1, sy = (m & 2) ? 1 : -1, sz = (m & 4) ? 1 : -1;
        pts.push_back({sx * ej[0] + sy * ej[1] + sz * ej[2], sx * ek[0] + sy * ek[1] + sz * ek[2]});
    }
    std::sort(pts.begin(), pts.end());
    auto cross = [](std::pair<double, double> o, std::pair<double, double> a, std::pair<double, double> b) {
        return (a.first - o.first) * (b.second - o.second) - (a.second - o.second) * (b.first - o.first);
    };
    std::vector<std::pair<double, double>> lo, up;
    for (auto &q : pts) {
        while (lo.size() >= 2 && cross(lo[lo.size() - 2], lo.back(), q) <= 0) lo.pop_back();
        lo.push_back(q);
        while (up.size() >= 2 && cross(up[up.size() - 2], up.back(), q) >= 0) up.pop_back();
        up.push_back(q);
    }
    auto lines = [](const std::vector<std::pair<double, double>> &ch, float *out, double fallback) {
        int n = 0;
        for (size_t i = 0; i + 1 < ch.size() && n < 3; ++i) {
            double dy = ch[i + 1].first - ch[i].first;
            if (dy < 1e-9) continue;  // vertical edge: bounds y only
            double sl = (ch[i + 1].second - ch[i].second) / dy;
            out[2 * n] = (float)sl;
            out[2 * n + 1] = (float)(ch[i].second - sl * ch[i].first);
            ++n;
        }
        if (n == 0) {
            out[0] = 0.0f;
            out[1] = (float)fallback;
            n = 1;
        }
        for (int i = n; i < 3; ++i) {
            out[2 * i] = out[0];
            out[2 * i + 1] = out[1];
        }
    };
    double zmax = -1e300, zmin = 1e300;
    for (auto &q : pts) {
        zmax = std::max(zmax, q.second);
        zmin = std::min(zmin, q.second);
    }
    lines(up, hull, zmax);
    lines(lo, hull + 6, zmin);
}

}  // namespace

void build_frames(const Geometry &g, std::vector<ProjFrame> &frames, std::vector<double> &B)
{
    const int S = g.n_proj, C = basis_count(g);
    frames.resize(S);
    B.assign((size_t)S * g.n_seg * C, 0.0);
    std::vector<double> y(C);
    for (int s = 0; s < S; ++s) {
        Quat q = mul(axis_angle(g.beta_axis, g.outer[s]), axis_angle(g.alpha_axis, g.inner[s]));
        ProjFrame &f = frames[s];
        rotate_inverse(q, g.j, f.ej);
        rotate_inverse(q, g.k, f.ek);
        rotate_inverse(q, g.p, f.d);
        double cj = 0.5 * (g.nj - 1) + g.joff[s];
        double ck = 0.5 * (g.nk - 1) + g.koff[s];
        for (int a = 0; a < 3; ++a) f.o[a] = -cj * f.ej[a] - ck * f.ek[a];
        f.lj = std::fabs(f.ej[0]) + std::fabs(f.ej[1]) + std::fabs(f.ej[2]);
        f.lk = std::fabs(f.ek[0]) + std::fabs(f.ek[1]) + std::fabs(f.ek[2]);
        for (int a = 0; a < 3; ++a) f.inv_d[a] = std::fabs(f.d[a]) > 1e-12 ? 1.0 / f.d[a] : 0.0;
        cube_shadow(f.ej, f.ek, f.hull);
        {
            int A = 0;
            for (int q = 1; q < 3; ++q)
                if (std::fabs(f.d[q]) > std::fabs(f.d[A]) + 1e-9) A = q;
            const int B = (A + 1) % 3, C2 = (A + 2) % 3;
            const double rj = f.ej[A] / f.d[A], rk = f.ek[A] / f.d[A];
            const double gjB = f.ej[B] - rj * f.d[B], gjC = f.ej[C2] - rj * f.d[C2];
            const double gkB = f.ek[B] - rk * f.d[B], gkC = f.ek[C2] - rk * f.d[C2];
            const double det = gjB * gkC - gkB * gjC;  // +-1/|d_A| for an orthonormal frame
            f.jos_a = A;
            f.jos_w = (float)(1.0 / std::fabs(f.d[A]));
            f.jos_gj[0] = (float)gjB;
            f.jos_gj[1] = (float)gjC;
            f.jos_gk[0] = (float)gkB;
            f.jos_gk[1] = (float)gkC;
            f.jos_igk[0] = std::fabs(gkB) > 1e-6 ? (float)(1.0 / gkB) : kFlatInv;
            f.jos_igk[1] = std::fabs(gkC) > 1e-6 ? (float)(1.0 / gkC) : kFlatInv;
            f.jos_rj = (float)((std::fabs(gkB) + std::fabs(gkC)) / std::fabs(det));
            f.jos_rk = (float)((std::fabs(gjB) + std::fabs(gjC)) / std::fabs(det));
        }
        for (int a = 0; a < 3; ++a) {
            f.ejf[a] = (float)f.ej[a];
            f.ekf[a] = (float)f.ek[a];
            f.df[a] = (float)f.d[a];
            f.inv_df[a] = f.inv_d[a] != 0.0 ? (float)f.inv_d[a] : kFlatInv;
        }
        for (int c = 0; c < g.n_seg; ++c) {
            double *row = &B[((size_t)s * g.n_seg + c) * C];
            for (int m = 0; m < g.n_sub; ++m) {
                double phi = (c - 0.5 + (m + 0.5) / g.n_sub) * g.seg_span / g.n_seg;
                double qd[3], qs[3];
                for (int a = 0; a < 3; ++a) qd[a] = std::cos(phi) * g.q0[a] + std::sin(phi) * g.q90[a];
                rotate_inverse(q, qd, qs);
                if (g.basis == TT_BASIS_SH)
                    sh_eval_one(g.ell_max, qs, y.data());
                else
                    kernel_eval(g, qs, y.data());
                for (int i = 0; i < C; ++i) row[i] += y[i];
            }
            for (int i = 0; i < C; ++i) row[i] /= g.n_sub;
        }
    }
}

// Slab plan of the staged march.  For a tile of T x T parallel rays and a
// slab of W planes of axis A, the samples of the slab lie in the parallelepiped
// spanned by the tile's corner rays between the planes; its extent along the
// other two axes does not depend on where the tile sits, so one (eb, ez) per
// projection bounds every tile's staged box (+2 for the corner cells and
// rounding, +2 for the one-voxel margin on each side).
int plan_slabs(std::vector<ProjFrame> &frames, int up, int lds_budget)
{
    constexpr int kMaxSlab = 8;
    const double T = kMarchTile - 1;
    int most = 0;
    for (ProjFrame &f : frames) {
        const int A = std::fabs(f.d[0]) >= std::fabs(f.d[1]) ? 0 : 1, B = 1 - A;
        f.slab_a = A;
        f.slab_w = f.slab_eb = f.slab_ez = 0;
        if (std::fabs(f.d[A]) < 0.25) continue;  // steep rays: many samples per plane
        for (int W = kMaxSlab; W >= 1; --W) {
            double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
            for (int v = 0; v < 8; ++v) {
                const double J = (v & 1) ? T : 0.0, K = (v & 2) ? T : 0.0, P = (v & 4) ? W : 0.0;
                const double t = (P - J * f.ej[A] - K * f.ek[A]) / f.d[A];
                const double q[2] = {J * f.ej[B] + K * f.ek[B] + t * f.d[B], J * f.ej[2] + K * f.ek[2] + t * f.d[2]};
                for (int a = 0; a < 2; ++a) {
                    lo[a] = std::min(lo[a], q[a]);
                    hi[a] = std::max(hi[a], q[a]);
                }
            }
            const int eb = (int)std::floor(hi[0] - lo[0]) + 5, ez = (int)std::floor(hi[1] - lo[1]) + 5;
            // element arrays padded to 64 (the march copies whole waves of 64)
            const long long bytes = (((long long)(W + 1) * eb * ez + 63) & ~63LL) * up * (long long)sizeof(float);
            if (bytes <= lds_budget) {
                f.slab_w = W;
                f.slab_eb = eb;
                f.slab_ez = ez;
                most = std::max(most, (int)bytes);
                break;
            }
        }
    }
    return most;
}

}  // namespace tt
