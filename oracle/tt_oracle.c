/*
 * tt_oracle.c -- FP64 CPU oracle for the tensor-tomography forward model.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct
 * implementation written from the paper's equations (Nielsen et al.,
 * "Mumott", section 2 "Methodology" and section 3.5 "Object-oriented
 * framework").  Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.  It shares no code, header or table with the
 * GPU library.
 *
 * What it computes (section / equation of the paper in brackets):
 *   - real even-order spherical harmonics              [sect. 3.2 "SH"]
 *   - goniometer rotation R_s = R_beta(beta) R_alpha(alpha)  [sect. 2, Eq. 1 text]
 *   - segment-averaged basis constants B_{s,c,i}        [Eq. projection_matrix]
 *   - ray geometry with raster offsets                  [Eq. real_space_geom]
 *   - forward model I_sjkc = sum P_{sjk,xyz} sum_i B_{sic} c_xyzi
 *                                                       [Eqs. projection_operator,
 *                                                        forward_model]
 *   - its exact adjoint, the squared loss with L2 regularisation and its
 *     gradient                                          [Eqs. opt_prob_general_form,
 *                                                        residual]
 *   - L-BFGS with an exact line search                  [sect. 3.5 "Optimization"]
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - P_{sjk,xyz} is realised as unit-step ray sampling with trilinear (tent)
 *     weights and zero padding: samples x_n = u_jk + n*step*d_s, n integer,
 *     weight T(x_n - x_v) = prod_a max(0, 1 - |x_n,a - x_v,a|), times step.
 *   - volume and detector are centred on the rotation centre: voxel centre
 *     x_v = i - (N-1)/2 per axis, pixel (j,k) at (j - (Nj-1)/2 - dj) e_j + ...
 *   - the segment average of Eq. projection_matrix is taken with an n_sub-node
 *     midpoint rule; segment c is centred at c*span/n_seg.
 *   - small-angle scattering direction q(phi) = cos(phi) q0 + sin(phi) q90
 *     (the approximate form of Eq. 1).
 *   - loss L(c) = sum w (Ac - I)^2 + mu sum c^2, no 1/2, no normalisation.
 *   - with model = 1, P_{sjk,xyz} is Joseph's method instead (the paper's own
 *     projector, sect. 3.5): cuts with the voxel-centre planes normal to the
 *     ray's dominant axis A (ties within 1e-9 go to the lower axis), bilinear
 *     interpolation within each plane, weight 1/|d_A| per cut.
 *
 * Parity status: every function here is pinned by the CPU test-suite (closed
 * forms, invariants, library special cases, brute force); none is unpinned.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OG_PI 3.14159265358979323846

typedef struct {
    int32_t nx, ny, nz;
    int32_t ell_max;
    int32_t n_proj;
    int32_t nj, nk, n_seg, n_sub;
    int32_t model;        /* 0: unit-step trilinear samples; 1: Joseph's method */
    double step;          /* ray sample spacing, in voxels */
    double seg_span;      /* angular range covered by the segments (2 pi) */
    const double *inner;  /* alpha_s, radians, length n_proj */
    const double *outer;  /* beta_s, radians */
    const double *joff;   /* delta j_s (may be NULL) */
    const double *koff;   /* delta k_s (may be NULL) */
    double p[3], j[3], k[3], q0[3], q90[3], alpha[3], beta[3];
    int32_t basis;        /* 0: spherical harmonics; 1: Gaussian kernels; 2: nearest neighbour */
    int32_t n_dirs;       /* grid directions of the kernel bases */
    const double *dirs;   /* [n_dirs][3] */
    double width;         /* Gaussian kernel width (radians) */
} og_geom;

/* ------------------------------------------------------------------------ */
/* Spherical harmonics (sect. 3.2): real, orthonormal, even l only.         */
/* Index i(l, m) = l(l-1)/2 + l + m.  Y_l0 = N_l0 P_l(cos th);              */
/* Y_lm = sqrt2 N_lm P_l^m(cos th) cos(m ph), Y_l,-m = ... sin(m ph), m > 0; */
/* N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!); no Condon-Shortley phase.      */
/* ------------------------------------------------------------------------ */

int og_num_coeffs(int ell_max) { return (ell_max / 2 + 1) * (ell_max + 1); }

/* Associated Legendre function P_l^m(x) without the (-1)^m phase, by the
 * textbook upward recurrence in l starting from P_m^m = (2m-1)!! (1-x^2)^{m/2}. */
double og_legendre(int l, int m, double x)
{
    double s = sqrt(fmax(0.0, 1.0 - x * x));
    double pmm = 1.0;
    for (int t = 1; t <= m; ++t) pmm *= (double)(2 * t - 1) * s;
    if (l == m) return pmm;
    double pm1 = x * (double)(2 * m + 1) * pmm;
    if (l == m + 1) return pm1;
    double pl = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pl = ((double)(2 * ll - 1) * x * pm1 - (double)(ll + m - 1) * pmm) / (double)(ll - m);
        pmm = pm1;
        pm1 = pl;
    }
    return pl;
}

static double og_norm(int l, int m)
{
    double ratio = 1.0; /* (l-m)!/(l+m)! */
    for (int t = l - m + 1; t <= l + m; ++t) ratio /= (double)t;
    return sqrt((2.0 * l + 1.0) / (4.0 * OG_PI) * ratio);
}

/* Evaluate all even-order Y_i at direction dir (need not be normalised). */
void og_sh(int ell_max, const double *dir, double *out)
{
    double r = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double ct = dir[2] / r;
    double ph = atan2(dir[1], dir[0]);
    int i = 0;
    for (int l = 0; l <= ell_max; l += 2) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double v = og_norm(l, am) * og_legendre(l, am, ct);
            if (m > 0) v *= sqrt(2.0) * cos(m * ph);
            else if (m < 0) v *= sqrt(2.0) * sin(am * ph);
            out[i++] = v;
        }
    }
}

/* Batched form for the tests: dirs[n][3] -> out[n][C]. */
void og_sh_batch(int ell_max, int64_t n, const double *dirs, double *out)
{
    int C = og_num_coeffs(ell_max);
    for (int64_t t = 0; t < n; ++t) og_sh(ell_max, dirs + 3 * t, out + C * t);
}

/* ------------------------------------------------------------------------ */
/* Goniometer (sect. 2): R_s = R_beta(beta_s) R_alpha(alpha_s), each a       */
/* right-handed rotation about a unit axis (Rodrigues' formula).            */
/* ------------------------------------------------------------------------ */

static void og_axis_rotation(const double *axis, double th, double *R)
{
    double n = sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
    double u[3] = {axis[0] / n, axis[1] / n, axis[2] / n};
    double K[9] = {0.0, -u[2], u[1], u[2], 0.0, -u[0], -u[1], u[0], 0.0};
    double s = sin(th), c1 = 1.0 - cos(th);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double k2 = 0.0;
            for (int t = 0; t < 3; ++t) k2 += K[3 * a + t] * K[3 * t + b];
            R[3 * a + b] = (a == b ? 1.0 : 0.0) + s * K[3 * a + b] + c1 * k2;
        }
}

void og_rotation(const og_geom *g, int s, double *R)
{
    double Ra[9], Rb[9];
    og_axis_rotation(g->alpha, g->inner[s], Ra);
    og_axis_rotation(g->beta, g->outer[s], Rb);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double v = 0.0;
            for (int t = 0; t < 3; ++t) v += Rb[3 * a + t] * Ra[3 * t + b];
            R[3 * a + b] = v;
        }
}

/* R^T v */
static void og_rt(const double *R, const double *v, double *out)
{
    for (int a = 0; a < 3; ++a) out[a] = R[a] * v[0] + R[3 + a] * v[1] + R[6 + a] * v[2];
}

/* ------------------------------------------------------------------------ */
/* Basis constants (Eq. projection_matrix): the mean of B_i(R_s^T q(phi))   */
/* over segment c, by an n_sub-node midpoint rule.  B[s][c][i].             */
/* ------------------------------------------------------------------------ */

/* Number of basis functions: SH count for ell_max, else the grid size. */
int og_n_basis(const og_geom *g) { return g->basis == 0 ? og_num_coeffs(g->ell_max) : g->n_dirs; }

/* Kernel bases on a grid of directions n_i (sect. 3.3 "Basis sets"); both
 * are antipodally symmetric like the scattering they describe:
 *   Gaussian kernels   f_i(q) = exp(-w_i^2 / (2 width^2)),
 *                      w_i = angle between q and the nearer of +-n_i;
 *   nearest neighbour  f_i(q) = 1 if n_i is the grid direction nearest to
 *                      +-q (ties to the lowest index), else 0. */
static void og_kernel_basis(const og_geom *g, const double *q, double *out)
{
    int best = 0;
    double best_c = -1.0;
    for (int i = 0; i < g->n_dirs; ++i) {
        const double *n = g->dirs + 3 * i;
        double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        double c = fabs(n[0] * q[0] + n[1] * q[1] + n[2] * q[2]) / nn;
        if (c > 1.0) c = 1.0;
        if (g->basis == 1) {
            double w = acos(c);
            out[i] = exp(-w * w / (2.0 * g->width * g->width));
        } else {
            out[i] = 0.0;
            if (c > best_c) {
                best_c = c;
                best = i;
            }
        }
    }
    if (g->basis == 2) out[best] = 1.0;
}

void og_basis_matrix(const og_geom *g, double *B)
{
    int C = og_n_basis(g);
    double *y = (double *)malloc(sizeof(double) * C);
    for (int s = 0; s < g->n_proj; ++s) {
        double R[9];
        og_rotation(g, s, R);
        for (int c = 0; c < g->n_seg; ++c) {
            double *row = B + ((int64_t)s * g->n_seg + c) * C;
            for (int i = 0; i < C; ++i) row[i] = 0.0;
            for (int m = 0; m < g->n_sub; ++m) {
                double phi = ((double)c + ((double)m + 0.5) / g->n_sub - 0.5) * g->seg_span / g->n_seg;
                double q[3], qs[3];
                for (int a = 0; a < 3; ++a) q[a] = cos(phi) * g->q0[a] + sin(phi) * g->q90[a];
                og_rt(R, q, qs);
                if (g->basis == 0)
                    og_sh(g->ell_max, qs, y);
                else
                    og_kernel_basis(g, qs, y);
                for (int i = 0; i < C; ++i) row[i] += y[i] / g->n_sub;
            }
        }
    }
    free(y);
}

/* ------------------------------------------------------------------------ */
/* Ray geometry (Eq. real_space_geom), in sample coordinates centred on the  */
/* rotation centre: e_j = R^T j, e_k = R^T k, d = R^T p, and the ray through */
/* pixel (j,k) is o + j e_j + k e_k + t d with                               */
/* o = -((Nj-1)/2 + dj) e_j - ((Nk-1)/2 + dk) e_k.                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    double ej[3], ek[3], d[3], o[3];
} og_frame;

void og_projection_frame(const og_geom *g, int s, double *out12)
{
    double R[9];
    og_rotation(g, s, R);
    og_frame f;
    og_rt(R, g->j, f.ej);
    og_rt(R, g->k, f.ek);
    og_rt(R, g->p, f.d);
    double cj = 0.5 * (g->nj - 1) + (g->joff ? g->joff[s] : 0.0);
    double ck = 0.5 * (g->nk - 1) + (g->koff ? g->koff[s] : 0.0);
    for (int a = 0; a < 3; ++a) f.o[a] = -cj * f.ej[a] - ck * f.ek[a];
    memcpy(out12, &f, sizeof(f));
}

static void og_get_frame(const og_geom *g, int s, og_frame *f)
{
    og_projection_frame(g, s, (double *)f);
}

/* Largest |n| that can reach the tent support of the volume: a sample at
 * parameter t is at distance >= |t| from the centre, and it touches the
 * volume only within sqrt(3) of a voxel centre. */
static int og_n_limit(const og_geom *g)
{
    double h = 0.5 * sqrt((double)g->nx * g->nx + (double)g->ny * g->ny + (double)g->nz * g->nz) + 2.0;
    return (int)ceil(h / g->step) + 1;
}

/* Tent weight of sample x for voxel (ix,iy,iz). */
static double og_tent(const og_geom *g, const double *x, int ix, int iy, int iz)
{
    double dx = fabs(x[0] - (ix - 0.5 * (g->nx - 1)));
    double dy = fabs(x[1] - (iy - 0.5 * (g->ny - 1)));
    double dz = fabs(x[2] - (iz - 0.5 * (g->nz - 1)));
    if (dx >= 1.0 || dy >= 1.0 || dz >= 1.0) return 0.0;
    return (1.0 - dx) * (1.0 - dy) * (1.0 - dz);
}

/* Ray sum of every coefficient channel along ray (s,j,k):
 * J_i = step * sum_n sum_v T(x_n - x_v) c_{v,i}  (Eq. projection_operator). */
static void og_ray_sum(const og_geom *g, const og_frame *f, int j, int k, const double *c, int C,
                       double *J)
{
    for (int i = 0; i < C; ++i) J[i] = 0.0;
    int nl = og_n_limit(g);
    for (int n = -nl; n <= nl; ++n) {
        double x[3];
        for (int a = 0; a < 3; ++a) x[a] = f->o[a] + j * f->ej[a] + k * f->ek[a] + n * g->step * f->d[a];
        int bx = (int)floor(x[0] + 0.5 * (g->nx - 1));
        int by = (int)floor(x[1] + 0.5 * (g->ny - 1));
        int bz = (int)floor(x[2] + 0.5 * (g->nz - 1));
        for (int ix = bx; ix <= bx + 1; ++ix) {
            if (ix < 0 || ix >= g->nx) continue;
            for (int iy = by; iy <= by + 1; ++iy) {
                if (iy < 0 || iy >= g->ny) continue;
                for (int iz = bz; iz <= bz + 1; ++iz) {
                    if (iz < 0 || iz >= g->nz) continue;
                    double w = og_tent(g, x, ix, iy, iz);
                    if (w == 0.0) continue;
                    const double *cv = c + (((int64_t)ix * g->ny + iy) * g->nz + iz) * C;
                    for (int i = 0; i < C; ++i) J[i] += w * cv[i];
                }
            }
        }
    }
    for (int i = 0; i < C; ++i) J[i] *= g->step;
}

/* ------------------------------------------------------------------------ */
/* Joseph's method (the discretisation the paper's projector uses, sect.     */
/* 3.5): the ray is cut by every voxel-centre plane normal to its dominant   */
/* axis A; at each cut the field is interpolated bilinearly in the two other */
/* axes (zero outside the volume), and each cut is weighted by the path      */
/* length between consecutive planes, 1 / |d_A|.                             */
/* ------------------------------------------------------------------------ */

/* Dominant axis of d; ties (within 1e-9) go to the lower axis index. */
static int og_dominant_axis(const double *d)
{
    int a = 0;
    for (int q = 1; q < 3; ++q)
        if (fabs(d[q]) > fabs(d[a]) + 1e-9) a = q;
    return a;
}

static void og_dims(const og_geom *g, int *n)
{
    n[0] = g->nx;
    n[1] = g->ny;
    n[2] = g->nz;
}

/* Cut of ray (j, k) with the centre plane of voxel layer i along axis A:
 * returns the in-plane coordinates u[3] (voxel index units, u[A] = i). */
static void og_joseph_cut(const og_geom *g, const og_frame *f, int A, int j, int k, int i, double *u)
{
    int n[3];
    og_dims(g, n);
    double base[3];
    for (int q = 0; q < 3; ++q) base[q] = f->o[q] + j * f->ej[q] + k * f->ek[q];
    double xA = i - 0.5 * (n[A] - 1);           /* centred coordinate of the plane */
    double t = (xA - base[A]) / f->d[A];
    for (int q = 0; q < 3; ++q) u[q] = base[q] + t * f->d[q] + 0.5 * (n[q] - 1);
    u[A] = i;
}

/* J_i = (1 / |d_A|) sum over layers of the bilinear interpolation of c_i. */
static void og_ray_sum_joseph(const og_geom *g, const og_frame *f, int j, int k, const double *c, int C,
                              double *J)
{
    int n[3];
    og_dims(g, n);
    int A = og_dominant_axis(f->d), B = (A + 1) % 3, Cx = (A + 2) % 3;
    for (int q = 0; q < C; ++q) J[q] = 0.0;
    for (int i = 0; i < n[A]; ++i) {
        double u[3];
        og_joseph_cut(g, f, A, j, k, i, u);
        int b0 = (int)floor(u[B]), c0 = (int)floor(u[Cx]);
        for (int bb = b0; bb <= b0 + 1; ++bb) {
            if (bb < 0 || bb >= n[B]) continue;
            double wb = 1.0 - fabs(u[B] - bb);
            for (int cc = c0; cc <= c0 + 1; ++cc) {
                if (cc < 0 || cc >= n[Cx]) continue;
                double w = wb * (1.0 - fabs(u[Cx] - cc));
                if (w <= 0.0) continue;
                int v[3];
                v[A] = i;
                v[B] = bb;
                v[Cx] = cc;
                const double *cv = c + (((int64_t)v[0] * g->ny + v[1]) * g->nz + v[2]) * C;
                for (int q = 0; q < C; ++q) J[q] += w * cv[q];
            }
        }
    }
    for (int q = 0; q < C; ++q) J[q] /= fabs(f->d[A]);
}

/* Transpose of og_ray_sum_joseph: add (w / |d_A|) ybar to the interpolated voxels. */
static void og_ray_splat_joseph(const og_geom *g, const og_frame *f, int j, int k, const double *ybar, int C,
                                double *acc)
{
    int n[3];
    og_dims(g, n);
    int A = og_dominant_axis(f->d), B = (A + 1) % 3, Cx = (A + 2) % 3;
    double inv = 1.0 / fabs(f->d[A]);
    for (int i = 0; i < n[A]; ++i) {
        double u[3];
        og_joseph_cut(g, f, A, j, k, i, u);
        int b0 = (int)floor(u[B]), c0 = (int)floor(u[Cx]);
        for (int bb = b0; bb <= b0 + 1; ++bb) {
            if (bb < 0 || bb >= n[B]) continue;
            double wb = 1.0 - fabs(u[B] - bb);
            for (int cc = c0; cc <= c0 + 1; ++cc) {
                if (cc < 0 || cc >= n[Cx]) continue;
                double w = wb * (1.0 - fabs(u[Cx] - cc));
                if (w <= 0.0) continue;
                int v[3];
                v[A] = i;
                v[B] = bb;
                v[Cx] = cc;
                double *av = acc + (((int64_t)v[0] * g->ny + v[1]) * g->nz + v[2]) * C;
                for (int q = 0; q < C; ++q) av[q] += w * inv * ybar[q];
            }
        }
    }
}

/* Joseph weight of voxel v for ray (j, k): (1/|d_A|) times the bilinear
 * weight of v at the ray's cut with v's own layer along A. */
static double og_joseph_weight(const og_geom *g, const og_frame *f, int j, int k, const int *v)
{
    int A = og_dominant_axis(f->d), B = (A + 1) % 3, Cx = (A + 2) % 3;
    double u[3];
    og_joseph_cut(g, f, A, j, k, v[A], u);
    double db = fabs(u[B] - v[B]), dc = fabs(u[Cx] - v[Cx]);
    if (db >= 1.0 || dc >= 1.0) return 0.0;
    return (1.0 - db) * (1.0 - dc) / fabs(f->d[A]);
}

/* Forward model (Eq. forward_model): I[s][j][k][c] = sum_i B[s][c][i] J_i. */
void og_project(const og_geom *g, const double *B, const double *c, double *I)
{
    int C = og_n_basis(g);
    int64_t rows = (int64_t)g->n_proj * g->nj;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t sj = 0; sj < rows; ++sj) {
        int s = (int)(sj / g->nj), j = (int)(sj % g->nj);
        og_frame f;
        og_get_frame(g, s, &f);
        double *J = (double *)malloc(sizeof(double) * C);
        for (int k = 0; k < g->nk; ++k) {
            if (g->model == 1)
                og_ray_sum_joseph(g, &f, j, k, c, C, J);
            else
                og_ray_sum(g, &f, j, k, c, C, J);
            double *out = I + (((int64_t)s * g->nj + j) * g->nk + k) * g->n_seg;
            for (int cc = 0; cc < g->n_seg; ++cc) {
                const double *b = B + ((int64_t)s * g->n_seg + cc) * C;
                double v = 0.0;
                for (int i = 0; i < C; ++i) v += b[i] * J[i];
                out[cc] = v;
            }
        }
        free(J);
    }
}

/* Forward model on a list of rays (s,j,k) only: out[r][n_seg]. */
void og_project_rays(const og_geom *g, const double *B, const double *c, int64_t n_rays,
                     const int32_t *sjk, double *out)
{
    int C = og_n_basis(g);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < n_rays; ++r) {
        int s = sjk[3 * r], j = sjk[3 * r + 1], k = sjk[3 * r + 2];
        og_frame f;
        og_get_frame(g, s, &f);
        double *J = (double *)malloc(sizeof(double) * C);
        if (g->model == 1)
            og_ray_sum_joseph(g, &f, j, k, c, C, J);
        else
            og_ray_sum(g, &f, j, k, c, C, J);
        for (int cc = 0; cc < g->n_seg; ++cc) {
            const double *b = B + ((int64_t)s * g->n_seg + cc) * C;
            double v = 0.0;
            for (int i = 0; i < C; ++i) v += b[i] * J[i];
            out[r * g->n_seg + cc] = v;
        }
        free(J);
    }
}

/* Splat step * T(x_n - x_v) * ybar into every voxel touched by ray (s,j,k). */
static void og_ray_splat(const og_geom *g, const og_frame *f, int j, int k, const double *ybar, int C,
                         double *acc)
{
    int nl = og_n_limit(g);
    for (int n = -nl; n <= nl; ++n) {
        double x[3];
        for (int a = 0; a < 3; ++a) x[a] = f->o[a] + j * f->ej[a] + k * f->ek[a] + n * g->step * f->d[a];
        int bx = (int)floor(x[0] + 0.5 * (g->nx - 1));
        int by = (int)floor(x[1] + 0.5 * (g->ny - 1));
        int bz = (int)floor(x[2] + 0.5 * (g->nz - 1));
        for (int ix = bx; ix <= bx + 1; ++ix) {
            if (ix < 0 || ix >= g->nx) continue;
            for (int iy = by; iy <= by + 1; ++iy) {
                if (iy < 0 || iy >= g->ny) continue;
                for (int iz = bz; iz <= bz + 1; ++iz) {
                    if (iz < 0 || iz >= g->nz) continue;
                    double w = og_tent(g, x, ix, iy, iz);
                    if (w == 0.0) continue;
                    double *av = acc + (((int64_t)ix * g->ny + iy) * g->nz + iz) * C;
                    for (int i = 0; i < C; ++i) av[i] += w * g->step * ybar[i];
                }
            }
        }
    }
}

/* Adjoint (transpose of Eq. forward_model):
 * out[v][i] = sum_{s,j,k} sum_n step T(x_n - x_v) sum_c B[s][c][i] y[s][j][k][c].
 * Threads splat into private volumes that are summed in thread order; the
 * thread count is capped so the private volumes fit in mem_budget bytes. */
void og_adjoint(const og_geom *g, const double *B, const double *y, double *out, double mem_budget)
{
    int C = og_n_basis(g);
    int64_t nv = (int64_t)g->nx * g->ny * g->nz * C;
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double per = (double)nv * sizeof(double);
    int cap = (int)(mem_budget / per);
    if (cap < 1) cap = 1;
    if (nt > cap) nt = cap;
    double **priv = (double **)malloc(sizeof(double *) * nt);
    priv[0] = out;
    memset(out, 0, sizeof(double) * nv);
    for (int t = 1; t < nt; ++t) priv[t] = (double *)calloc(nv, sizeof(double));
    int64_t rows = (int64_t)g->n_proj * g->nj;
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *ybar = (double *)malloc(sizeof(double) * C);
#pragma omp for schedule(static)
        for (int64_t sj = 0; sj < rows; ++sj) {
            int s = (int)(sj / g->nj), j = (int)(sj % g->nj);
            og_frame f;
            og_get_frame(g, s, &f);
            for (int k = 0; k < g->nk; ++k) {
                const double *yr = y + (((int64_t)s * g->nj + j) * g->nk + k) * g->n_seg;
                for (int i = 0; i < C; ++i) {
                    double v = 0.0;
                    for (int cc = 0; cc < g->n_seg; ++cc) v += B[((int64_t)s * g->n_seg + cc) * C + i] * yr[cc];
                    ybar[i] = v;
                }
                if (g->model == 1)
                    og_ray_splat_joseph(g, &f, j, k, ybar, C, priv[tid]);
                else
                    og_ray_splat(g, &f, j, k, ybar, C, priv[tid]);
            }
        }
        free(ybar);
    }
    for (int t = 1; t < nt; ++t) {
        for (int64_t e = 0; e < nv; ++e) out[e] += priv[t][e];
        free(priv[t]);
    }
    free(priv);
}

/* Adjoint at a list of voxels only (index triples), out[v][C].  For each
 * projection it visits every pixel within 2 of the voxel's detector position
 * and every sample within 2 of its depth along the beam: a nonzero tent weight
 * needs all three offsets below sqrt(3). */
void og_adjoint_voxels(const og_geom *g, const double *B, const double *y, int64_t n_vox,
                       const int32_t *xyz, double *out)
{
    int C = og_n_basis(g);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t v = 0; v < n_vox; ++v) {
        int ix = xyz[3 * v], iy = xyz[3 * v + 1], iz = xyz[3 * v + 2];
        double xv[3] = {ix - 0.5 * (g->nx - 1), iy - 0.5 * (g->ny - 1), iz - 0.5 * (g->nz - 1)};
        double *o = out + v * C;
        for (int i = 0; i < C; ++i) o[i] = 0.0;
        for (int s = 0; s < g->n_proj; ++s) {
            og_frame f;
            og_get_frame(g, s, &f);
            double w[3] = {xv[0] - f.o[0], xv[1] - f.o[1], xv[2] - f.o[2]};
            double a = w[0] * f.ej[0] + w[1] * f.ej[1] + w[2] * f.ej[2];
            double b = w[0] * f.ek[0] + w[1] * f.ek[1] + w[2] * f.ek[2];
            double t = w[0] * f.d[0] + w[1] * f.d[1] + w[2] * f.d[2];
            if (g->model == 1) {
                /* every pixel within 4 of the voxel's detector position */
                const int vv[3] = {ix, iy, iz};
                for (int j = (int)floor(a) - 4; j <= (int)floor(a) + 5; ++j) {
                    if (j < 0 || j >= g->nj) continue;
                    for (int k = (int)floor(b) - 4; k <= (int)floor(b) + 5; ++k) {
                        if (k < 0 || k >= g->nk) continue;
                        double wj = og_joseph_weight(g, &f, j, k, vv);
                        if (wj == 0.0) continue;
                        const double *yr = y + (((int64_t)s * g->nj + j) * g->nk + k) * g->n_seg;
                        for (int i = 0; i < C; ++i) {
                            double v2 = 0.0;
                            for (int cc = 0; cc < g->n_seg; ++cc) v2 += B[((int64_t)s * g->n_seg + cc) * C + i] * yr[cc];
                            o[i] += wj * v2;
                        }
                    }
                }
                continue;
            }
            int j0 = (int)floor(a) - 2, k0 = (int)floor(b) - 2;
            int n0 = (int)floor((t - 2.0) / g->step) - 1, n1 = (int)ceil((t + 2.0) / g->step) + 1;
            for (int j = j0; j <= j0 + 5; ++j) {
                if (j < 0 || j >= g->nj) continue;
                for (int k = k0; k <= k0 + 5; ++k) {
                    if (k < 0 || k >= g->nk) continue;
                    const double *yr = y + (((int64_t)s * g->nj + j) * g->nk + k) * g->n_seg;
                    double wsum = 0.0;
                    for (int n = n0; n <= n1; ++n) {
                        double x[3];
                        for (int q = 0; q < 3; ++q)
                            x[q] = f.o[q] + j * f.ej[q] + k * f.ek[q] + n * g->step * f.d[q];
                        wsum += og_tent(g, x, ix, iy, iz);
                    }
                    if (wsum == 0.0) continue;
                    for (int i = 0; i < C; ++i) {
                        double v2 = 0.0;
                        for (int cc = 0; cc < g->n_seg; ++cc) v2 += B[((int64_t)s * g->n_seg + cc) * C + i] * yr[cc];
                        o[i] += g->step * wsum * v2;
                    }
                }
            }
        }
    }
}

/* Transpose of the ray sums of one projection on an arbitrary number of
 * channels: Q[v][u] = sum_{j,k} sum_n step T(x_n - x_v) yf[j][k][u].  With
 * yf the segment-folded residual this is the adjoint before the map by
 * B_s^T; the precision-tier tests round Q at this point. */
void og_splat_projection(const og_geom *g, int s, const double *yf, int nu, double *Q)
{
    og_frame f;
    og_get_frame(g, s, &f);
    int64_t nv = (int64_t)g->nx * g->ny * g->nz * nu;
    memset(Q, 0, sizeof(double) * nv);
    for (int j = 0; j < g->nj; ++j)
        for (int k = 0; k < g->nk; ++k)
            if (g->model == 1)
                og_ray_splat_joseph(g, &f, j, k, yf + ((int64_t)j * g->nk + k) * nu, nu, Q);
            else
                og_ray_splat(g, &f, j, k, yf + ((int64_t)j * g->nk + k) * nu, nu, Q);
}

/* ------------------------------------------------------------------------ */
/* Loss and gradient (Eqs. opt_prob_general_form and residual with a = b = 2,*/
/* D = identity): r = A c - I, L = sum w r^2 + mu sum c^2,                   */
/* grad L = 2 A^T (w r) + 2 mu c.  w may be NULL (all ones).                 */
/* ------------------------------------------------------------------------ */

double og_loss_grad(const og_geom *g, const double *B, const double *c, const double *data,
                    const double *w, double mu, double *grad, double *resid, double mem_budget)
{
    int C = og_n_basis(g);
    int64_t nd = (int64_t)g->n_proj * g->nj * g->nk * g->n_seg;
    int64_t nc = (int64_t)g->nx * g->ny * g->nz * C;
    double *r = resid ? resid : (double *)malloc(sizeof(double) * nd);
    og_project(g, B, c, r);
    double loss = 0.0;
    for (int64_t e = 0; e < nd; ++e) {
        r[e] -= data[e];
        double we = w ? w[e] : 1.0;
        loss += we * r[e] * r[e];
    }
    for (int64_t e = 0; e < nc; ++e) loss += mu * c[e] * c[e];
    if (grad) {
        double *y = (double *)malloc(sizeof(double) * nd);
        for (int64_t e = 0; e < nd; ++e) y[e] = 2.0 * (w ? w[e] : 1.0) * r[e];
        og_adjoint(g, B, y, grad, mem_budget);
        for (int64_t e = 0; e < nc; ++e) grad[e] += 2.0 * mu * c[e];
        free(y);
    }
    if (!resid) free(r);
    return loss;
}

/* ------------------------------------------------------------------------ */
/* L-BFGS (sect. 3.5 "Optimization"; two-loop recursion of Nocedal & Wright, */
/* algorithm 7.4) with initial scaling gamma = s^T y / y^T y of the newest   */
/* accepted pair (1 before any pair), and the exact line search of the       */
/* quadratic loss: alpha = -g^T d / (2 (||A d||_w^2 + mu ||d||^2)).          */
/* A pair is skipped when s^T y <= 1e-12 ||s|| ||y||.  Stops after max_iter  */
/* iterations or when ||r|| / ||I|| <= tol.  hist[2*it] = loss after        */
/* iteration it, hist[2*it+1] = ||r||/||I||.  Returns iterations done; the   */
/* final relative residual is recomputed by an explicit forward.            */
/* ------------------------------------------------------------------------ */

static double og_dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t e = 0; e < n; ++e) s += a[e] * b[e];
    return s;
}

int og_lbfgs(const og_geom *g, const double *B, double *c, const double *data, const double *w,
             double mu, int m, int max_iter, double tol, double *hist, double *final_rel,
             double mem_budget)
{
    int C = og_n_basis(g);
    int64_t nd = (int64_t)g->n_proj * g->nj * g->nk * g->n_seg;
    int64_t n = (int64_t)g->nx * g->ny * g->nz * C;
    double *r = (double *)malloc(sizeof(double) * nd);
    double *q = (double *)malloc(sizeof(double) * nd);
    double *gr = (double *)malloc(sizeof(double) * n);
    double *gn = (double *)malloc(sizeof(double) * n);
    double *d = (double *)malloc(sizeof(double) * n);
    double *yb = (double *)malloc(sizeof(double) * nd);
    double *S = (double *)malloc(sizeof(double) * n * m);
    double *Y = (double *)malloc(sizeof(double) * n * m);
    double *rho = (double *)malloc(sizeof(double) * m);
    double *al = (double *)malloc(sizeof(double) * m);
    int stored = 0, head = 0; /* ring buffer: newest pair at (head-1) mod m */
    double gamma = 1.0;
    double normI = sqrt(og_dot(nd, data, data));

    og_loss_grad(g, B, c, data, w, mu, gr, r, mem_budget);
    int it = 0;
    for (; it < max_iter; ++it) {
        if (sqrt(og_dot(nd, r, r)) / normI <= tol) break;
        /* two-loop recursion: d = -H g */
        for (int64_t e = 0; e < n; ++e) d[e] = gr[e];
        for (int t = 0; t < stored; ++t) {
            int idx = ((head - 1 - t) % m + m) % m;
            al[idx] = rho[idx] * og_dot(n, S + idx * n, d);
            for (int64_t e = 0; e < n; ++e) d[e] -= al[idx] * Y[idx * n + e];
        }
        for (int64_t e = 0; e < n; ++e) d[e] *= gamma;
        for (int t = stored - 1; t >= 0; --t) {
            int idx = ((head - 1 - t) % m + m) % m;
            double be = rho[idx] * og_dot(n, Y + idx * n, d);
            for (int64_t e = 0; e < n; ++e) d[e] += S[idx * n + e] * (al[idx] - be);
        }
        for (int64_t e = 0; e < n; ++e) d[e] = -d[e];
        /* exact line search on the quadratic loss */
        og_project(g, B, d, q);
        double qq = 0.0;
        for (int64_t e = 0; e < nd; ++e) qq += (w ? w[e] : 1.0) * q[e] * q[e];
        double denom = 2.0 * (qq + mu * og_dot(n, d, d));
        if (!(denom > 0.0)) break;
        double alpha = -og_dot(n, gr, d) / denom;
        for (int64_t e = 0; e < n; ++e) c[e] += alpha * d[e];
        for (int64_t e = 0; e < nd; ++e) r[e] += alpha * q[e];
        /* new gradient 2 A^T (w r) + 2 mu c */
        for (int64_t e = 0; e < nd; ++e) yb[e] = 2.0 * (w ? w[e] : 1.0) * r[e];
        og_adjoint(g, B, yb, gn, mem_budget);
        for (int64_t e = 0; e < n; ++e) gn[e] += 2.0 * mu * c[e];
        /* curvature pair s = alpha d, y = g_new - g */
        double *Sh = S + (int64_t)head * n, *Yh = Y + (int64_t)head * n;
        double sy = 0.0, ss = 0.0, yy = 0.0;
        for (int64_t e = 0; e < n; ++e) {
            double se = alpha * d[e], ye = gn[e] - gr[e];
            sy += se * ye;
            ss += se * se;
            yy += ye * ye;
        }
        if (sy > 1e-12 * sqrt(ss) * sqrt(yy)) {
            for (int64_t e = 0; e < n; ++e) {
                Sh[e] = alpha * d[e];
                Yh[e] = gn[e] - gr[e];
            }
            rho[head] = 1.0 / sy;
            gamma = sy / yy;
            head = (head + 1) % m;
            if (stored < m) ++stored;
        }
        memcpy(gr, gn, sizeof(double) * n);
        if (hist) {
            double loss = 0.0;
            for (int64_t e = 0; e < nd; ++e) loss += (w ? w[e] : 1.0) * r[e] * r[e];
            loss += mu * og_dot(n, c, c);
            hist[2 * it] = loss;
            hist[2 * it + 1] = sqrt(og_dot(nd, r, r)) / normI;
        }
    }
    og_project(g, B, c, r);
    for (int64_t e = 0; e < nd; ++e) r[e] -= data[e];
    if (final_rel) *final_rel = sqrt(og_dot(nd, r, r)) / normI;
    free(r); free(q); free(gr); free(gn); free(d); free(yb);
    free(S); free(Y); free(rho); free(al);
    return it;
}

int og_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
