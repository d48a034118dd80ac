// Learned level-1 smoother blocks: network inference that writes the blocks,
// and the training kernels (backward pass, parameter-gradient reduction,
// Adam).  The definitions are in include/saamg.h next to
// amg_smoother_set_weights.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace saamg {

constexpr int kFeat = 90;
constexpr int kHid = 64;
constexpr int kOut = 6;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kFeat * kHid;   // 5760
constexpr int kOffW2 = kOffB1 + kHid;           // 5824
constexpr int kOffB2 = kOffW2 + kHid * kHid;    // 9920
constexpr int kOffW3 = kOffB2 + kHid;           // 9984
constexpr int kOffB3 = kOffW3 + kHid * kOut;    // 10368
constexpr int kParams = kOffB3 + kOut;          // 10374
constexpr int kGradChunk = 512;                 // nodes per partial sum of the parameter gradient

// g = network(phi) for nb nodes (phi: nb x 90, g: nb x 6, row-major).  z1 and
// z2 (nb x 64 pre-activations) are stored when non-null (training).
// FP32 copy of n BF16 values (network parameters stored in BF16)
void launch_bf16_widen(int n, const uint16_t *bits, float *out, hipStream_t s);
void launch_mlp_forward(int nb, const float *phi, const float *theta, float *z1, float *z2, float *g,
                        hipStream_t s);
// S_i = L_i (I + sym(c tanh g_i)) L_i^T into the planar block array M (same
// layout as the smoother blocks).  t (nb x 6, may be null) receives tanh(g).
// check: non-finite blocks are replaced by the block of Mbj and counted in
// *nbad (device int, zeroed by the caller).
template <typename T>
void launch_assemble_blocks(int nb, const float *g, const double *L, T *M, const T *Mbj, float *t, int check,
                            int *nbad, hipStream_t s);
// w = e - S r (S planar FP64 blocks)
void launch_block_resid(int nb, const double *S, const double *e, const double *r, double *w, hipStream_t s);
// partial dot products of a . b (grid = returned value), then out = sum
int launch_dot_out(int64_t n, const double *a, const double *b, double *partials, int max_grid, double *out,
                   hipStream_t s);
// loss bookkeeping: scal[2] += scal[1] / scal[0]; scal[3] = -2 / scal[0]
void launch_loss_acc(double *scal, hipStream_t s);
// U_i += (*coef) q_i r_i^T (U: nb x 9 FP64)
void launch_outer_acc(int nb, double *U, const double *q, const double *r, const double *coef, hipStream_t s);
// dg = c (1 - t^2) sym^T(L^T (inv_k U) L)
void launch_block_grad(int nb, const double *U, const double *L, const float *t, double inv_k, float *dg,
                       hipStream_t s);
// backward through the two hidden layers: dz2, dz1 (nb x 64)
void launch_mlp_backward(int nb, const float *theta, const float *z1, const float *z2, const float *dg,
                         float *dz1, float *dz2, hipStream_t s);
// grad = [accumulate ? grad : 0] + scale * dl/dtheta, through per-chunk FP64
// partial sums (partials: ceil(nb / kGradChunk) x kParams doubles)
void launch_param_grad(int nb, const float *phi, const float *z1, const float *z2, const float *dg,
                       const float *dz1, const float *dz2, double *partials, float *grad, float scale,
                       int accumulate, hipStream_t s);
void launch_adam(int n, float *theta, const float *grad, float *m, float *v, float lr, float beta1, float beta2,
                 float eps, float bc1, float bc2, hipStream_t s);
// e - z for the training errors: e -= z
void launch_sub_from(int64_t n, const double *z, double *e, hipStream_t s);

}  // namespace saamg
