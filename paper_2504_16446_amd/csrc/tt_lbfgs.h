// Device-resident L-BFGS state: float64 scalars and the Gram matrix of the
// history, and int bookkeeping of the pair ring.  Offsets into two arrays.
#pragma once

#include <hip/hip_runtime.h>

namespace tt {

constexpr int kMaxM = 10;                      // longest supported history
constexpr int kMaxBasis = 2 * (kMaxM + 1) + 1;  // s slots, y slots, gradient

// float64 state
constexpr int kGram = 0;                                   // [kMaxBasis][kMaxBasis]
constexpr int kRho = kGram + kMaxBasis * kMaxBasis;        // [kMaxM + 1]
constexpr int kAlphaTmp = kRho + kMaxM + 1;                // [kMaxM + 1]
constexpr int kCoef = kAlphaTmp + kMaxM + 1;               // [kMaxBasis]
constexpr int kGamma = kCoef + kMaxBasis;
constexpr int kAlpha = kGamma + 1;
constexpr int kQQ = kAlpha + 1;        // ||A d||_w^2
constexpr int kLoss = kQQ + 1;         // sum w r^2 + mu sum c^2
constexpr int kLossR = kLoss + 1;      // sum w r^2
constexpr int kRR = kLossR + 1;        // sum r^2 (must follow kLossR)
constexpr int kCC = kRR + 1;           // sum c^2
constexpr int kDataNorm2 = kCC + 1;    // sum I^2
constexpr int kDotsD = kDataNorm2 + 1; // [kMaxBasis + 1]: d . b_a, d . d at kMaxBasis
constexpr int kDotsG = kDotsD + kMaxBasis + 1;  // [kMaxBasis + 1]: g_new . list
constexpr int kStateDoubles = kDotsG + kMaxBasis + 1;

// int state
constexpr int kOrder = 0;               // [kMaxM] slots, oldest first
constexpr int kCount = kOrder + kMaxM;  // valid pairs
constexpr int kCand = kCount + 1;       // slot receiving the next pair
constexpr int kAccepted = kCand + 1;
constexpr int kIter = kAccepted + 1;
constexpr int kMask = kIter + 1;              // [kMaxBasis + 1] combine mask
constexpr int kMask2 = kMask + kMaxBasis + 1;  // [kMaxBasis + 1] multidot mask
constexpr int kStateInts = kMask2 + kMaxBasis + 1;

struct Dims;
hipError_t lbfgs_plan_direction(double *st, int *ist, int m, hipStream_t s);
hipError_t lbfgs_plan_alpha(double *st, int *ist, int m, double mu, hipStream_t s);
hipError_t lbfgs_plan_user_direction(double *st, int *ist, int m, hipStream_t s);
hipError_t lbfgs_plan_update(double *st, int *ist, int m, double mu, hipStream_t s);
hipError_t lbfgs_combine(const float *const *basis, int nb, const double *coef, const int *mask, long long n,
                         float *d, double *partials, double *out, hipStream_t s);
// Dot products x . vecs[a] (masked).  With y_slots, also y[cand] = x - vecs[gold].
hipError_t lbfgs_multidot(const float *x, const float *const *vecs, int nv, const int *mask, long long n,
                          double *partials, double *out, hipStream_t s, const float *const *y_slots = nullptr,
                          int ns = 0, const int *ist = nullptr, int gold = 0);
hipError_t lbfgs_wnorm2(const float *q, const float *w, long long n, double *partials, double *out, hipStream_t s);
hipError_t lbfgs_update_c(float *c, const float *d, const float *const *s_slots, int ns, const double *st,
                          const int *ist, long long n, hipStream_t s);
hipError_t lbfgs_make_y(const float *const *y_slots, int ns, const int *ist, const float *gn, const float *go,
                        long long n, hipStream_t s);
hipError_t lbfgs_resid_update(const Dims &d, float *r, const float *q, const float *w, const double *st, float *yf,
                              double *partials, double *out, hipStream_t s);
int lbfgs_blocks();

}  // namespace tt
