// Kernels of the learned level-1 smoother blocks (gfx950).
//
// Inference runs once per weight update, not per iteration: one thread per
// node evaluates the 90 -> 64 -> 64 -> 6 network in FP32 with the parameters
// staged in LDS (every lane reads the same weight, so each LDS read is a
// broadcast), and a second kernel turns the 6 outputs into the symmetric
// block S_i = L_i (I + X_i) L_i^T written straight into the planar smoother
// array the V-cycle kernels read (the level-1 fused post-sweep operator
// G = P - S (A P) is then formed again before the next V-cycle).  The solve
// therefore pays nothing per iteration for the learned blocks.  Training adds the backward pass per node and a
// deterministic parameter-gradient reduction (per-chunk FP64 partial sums,
// added in a fixed order).
#include <algorithm>
#include <cmath>

#include "learned.hpp"

namespace saamg {

namespace {

__device__ __forceinline__ double lsum_wave(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// sum over the workgroup, valid in thread 0
__device__ __forceinline__ double lsum_block(double v, double *lds) {
    v = lsum_wave(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; ++i) s += lds[i];
    __syncthreads();
    return s;
}

__device__ __forceinline__ int64_t planar(int64_t row, int e) {
    return (row / kMSlice) * (9 * kMSlice) + e * kMSlice + (row % kMSlice);
}

__constant__ double kSpread[kOut] = {0.25, 0.25, 0.25, 0.05, 0.05, 0.05};

}  // namespace

__global__ __launch_bounds__(kBlock) void k_mlp_forward(int nb, const float *__restrict__ phi,
                                                        const float *__restrict__ theta,
                                                        float *__restrict__ z1o, float *__restrict__ z2o,
                                                        float *__restrict__ g) {
    __shared__ float w[kParams];
    for (int i = threadIdx.x; i < kParams; i += kBlock) w[i] = theta[i];
    __syncthreads();
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= nb) return;
    float h1[kHid];
#pragma unroll
    for (int b = 0; b < kHid; ++b) h1[b] = w[kOffB1 + b];
    const float *x = phi + (size_t)n * kFeat;
    for (int a = 0; a < kFeat; ++a) {
        const float xa = x[a];
        const float *wr = w + kOffW1 + a * kHid;
#pragma unroll
        for (int b = 0; b < kHid; ++b) h1[b] = fmaf(xa, wr[b], h1[b]);
    }
    if (z1o) {
        float *o = z1o + (size_t)n * kHid;
#pragma unroll
        for (int b = 0; b < kHid; ++b) o[b] = h1[b];
    }
#pragma unroll
    for (int b = 0; b < kHid; ++b) h1[b] = fmaxf(h1[b], 0.0f);
    float h2[kHid];
#pragma unroll
    for (int b = 0; b < kHid; ++b) h2[b] = w[kOffB2 + b];
#pragma unroll
    for (int a = 0; a < kHid; ++a) {
        const float *wr = w + kOffW2 + a * kHid;
#pragma unroll
        for (int b = 0; b < kHid; ++b) h2[b] = fmaf(h1[a], wr[b], h2[b]);
    }
    if (z2o) {
        float *o = z2o + (size_t)n * kHid;
#pragma unroll
        for (int b = 0; b < kHid; ++b) o[b] = h2[b];
    }
    float out[kOut];
#pragma unroll
    for (int c = 0; c < kOut; ++c) out[c] = w[kOffB3 + c];
#pragma unroll
    for (int a = 0; a < kHid; ++a) {
        const float ha = fmaxf(h2[a], 0.0f);
#pragma unroll
        for (int c = 0; c < kOut; ++c) out[c] = fmaf(ha, w[kOffW3 + a * kOut + c], out[c]);
    }
#pragma unroll
    for (int c = 0; c < kOut; ++c) g[(size_t)n * kOut + c] = out[c];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_assemble_blocks(int nb, const float *__restrict__ g,
                                                            const double *__restrict__ L, T *__restrict__ M,
                                                            const T *__restrict__ Mbj, float *__restrict__ tout,
                                                            int check, int *nbad) {
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= nb) return;
    double t[kOut];
#pragma unroll
    for (int c = 0; c < kOut; ++c) {
        t[c] = tanh((double)g[(size_t)n * kOut + c]);
        if (tout) tout[(size_t)n * kOut + c] = (float)t[c];
    }
    // T = I + sym(c t)
    const double T00 = 1.0 + kSpread[0] * t[0], T11 = 1.0 + kSpread[1] * t[1], T22 = 1.0 + kSpread[2] * t[2];
    const double T01 = kSpread[3] * t[3], T02 = kSpread[4] * t[4], T12 = kSpread[5] * t[5];
    const double *l = L + (size_t)n * 6;
    const double l00 = l[0], l10 = l[1], l11 = l[2], l20 = l[3], l21 = l[4], l22 = l[5];
    // W = L T (L lower triangular)
    const double W00 = l00 * T00, W01 = l00 * T01, W02 = l00 * T02;
    const double W10 = l10 * T00 + l11 * T01, W11 = l10 * T01 + l11 * T11, W12 = l10 * T02 + l11 * T12;
    const double W20 = l20 * T00 + l21 * T01 + l22 * T02, W21 = l20 * T01 + l21 * T11 + l22 * T12,
                 W22 = l20 * T02 + l21 * T12 + l22 * T22;
    // S = W L^T
    double S[9];
    S[0] = W00 * l00;
    S[1] = W00 * l10 + W01 * l11;
    S[2] = W00 * l20 + W01 * l21 + W02 * l22;
    S[3] = W10 * l00;
    S[4] = W10 * l10 + W11 * l11;
    S[5] = W10 * l20 + W11 * l21 + W12 * l22;
    S[6] = W20 * l00;
    S[7] = W20 * l10 + W21 * l11;
    S[8] = W20 * l20 + W21 * l21 + W22 * l22;
    bool finite = true;
#pragma unroll
    for (int e = 0; e < 9; ++e) finite = finite && isfinite(S[e]);
    if (check && !finite) {
#pragma unroll
        for (int e = 0; e < 9; ++e) M[planar(n, e)] = Mbj[planar(n, e)];
        atomicAdd(nbad, 1);
        return;
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) M[planar(n, e)] = (T)S[e];
}

__global__ __launch_bounds__(kBlock) void k_block_resid(int nb, const double *__restrict__ S,
                                                        const double *__restrict__ e,
                                                        const double *__restrict__ r, double *__restrict__ w) {
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= nb) return;
    const double r0 = r[3 * (size_t)n], r1 = r[3 * (size_t)n + 1], r2 = r[3 * (size_t)n + 2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double v = S[planar(n, 3 * a)] * r0 + S[planar(n, 3 * a + 1)] * r1 + S[planar(n, 3 * a + 2)] * r2;
        w[3 * (size_t)n + a] = e[3 * (size_t)n + a] - v;
    }
}

__global__ __launch_bounds__(kBlock) void k_dot_partial(int64_t n, const double *__restrict__ a,
                                                        const double *__restrict__ b, double *partials) {
    __shared__ double lds[kBlock / 64];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        s += a[i] * b[i];
    s = lsum_block(s, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_sum_out(const double *__restrict__ partials, int nblk, double *out) {
    __shared__ double lds[kBlock / 64];
    double s = 0.0;
    for (int j = threadIdx.x; j < nblk; j += kBlock) s += partials[j];
    s = lsum_block(s, lds);
    if (threadIdx.x == 0) *out = s;
}

__global__ void k_loss_acc(double *scal) {
    if (threadIdx.x == 0) {
        scal[2] += scal[1] / scal[0];
        scal[3] = -2.0 / scal[0];
    }
}

__global__ __launch_bounds__(kBlock) void k_outer_acc(int nb, double *__restrict__ U, const double *__restrict__ q,
                                                      const double *__restrict__ r, const double *coef) {
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= nb) return;
    const double c = *coef;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double qa = c * q[3 * (size_t)n + a];
#pragma unroll
        for (int b = 0; b < 3; ++b) U[9 * (size_t)n + 3 * a + b] += qa * r[3 * (size_t)n + b];
    }
}

__global__ __launch_bounds__(kBlock) void k_block_grad(int nb, const double *__restrict__ U,
                                                       const double *__restrict__ L, const float *__restrict__ t,
                                                       double inv_k, float *__restrict__ dg) {
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= nb) return;
    double u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = inv_k * U[9 * (size_t)n + e];
    const double *l = L + (size_t)n * 6;
    // L as a full lower-triangular 3x3
    const double Lm[9] = {l[0], 0.0, 0.0, l[1], l[2], 0.0, l[3], l[4], l[5]};
    // dX = L^T U L:  (L^T U)_{ab} = sum_c L_{ca} U_{cb}
    double LU[9], dX[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            LU[3 * a + b] = Lm[a] * u[b] + Lm[3 + a] * u[3 + b] + Lm[6 + a] * u[6 + b];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            dX[3 * a + b] = LU[3 * a] * Lm[b] + LU[3 * a + 1] * Lm[3 + b] + LU[3 * a + 2] * Lm[6 + b];
    const double adj[kOut] = {dX[0], dX[4], dX[8], dX[1] + dX[3], dX[2] + dX[6], dX[5] + dX[7]};
#pragma unroll
    for (int c = 0; c < kOut; ++c) {
        const double tc = t[(size_t)n * kOut + c];
        dg[(size_t)n * kOut + c] = (float)(kSpread[c] * (1.0 - tc * tc) * adj[c]);
    }
}

__global__ __launch_bounds__(kBlock) void k_mlp_backward(int nb, const float *__restrict__ theta,
                                                         const float *__restrict__ z1, const float *__restrict__ z2,
                                                         const float *__restrict__ dg, float *__restrict__ dz1,
                                                         float *__restrict__ dz2) {
    __shared__ float w[kParams];
    for (int i = threadIdx.x; i < kParams; i += kBlock) w[i] = theta[i];
    __syncthreads();
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= nb) return;
    float d[kOut];
#pragma unroll
    for (int c = 0; c < kOut; ++c) d[c] = dg[(size_t)n * kOut + c];
    float e2[kHid];
    const float *zz2 = z2 + (size_t)n * kHid;
#pragma unroll
    for (int a = 0; a < kHid; ++a) {
        float s = 0.0f;
#pragma unroll
        for (int c = 0; c < kOut; ++c) s = fmaf(w[kOffW3 + a * kOut + c], d[c], s);
        e2[a] = zz2[a] > 0.0f ? s : 0.0f;
        dz2[(size_t)n * kHid + a] = e2[a];
    }
    const float *zz1 = z1 + (size_t)n * kHid;
#pragma unroll
    for (int a = 0; a < kHid; ++a) {
        const float *wr = w + kOffW2 + a * kHid;
        float s = 0.0f;
#pragma unroll
        for (int b = 0; b < kHid; ++b) s = fmaf(wr[b], e2[b], s);
        dz1[(size_t)n * kHid + a] = zz1[a] > 0.0f ? s : 0.0f;
    }
}

// One thread per parameter and node chunk.
__global__ __launch_bounds__(kBlock) void k_param_partial(int nb, const float *__restrict__ phi,
                                                          const float *__restrict__ z1,
                                                          const float *__restrict__ z2,
                                                          const float *__restrict__ dg,
                                                          const float *__restrict__ dz1,
                                                          const float *__restrict__ dz2, double *partials) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= kParams) return;
    const int chunk = blockIdx.y;
    const int n0 = chunk * kGradChunk, n1 = min(nb, n0 + kGradChunk);
    double acc = 0.0;
    if (p < kOffB1) {
        const int a = p / kHid, b = p % kHid;
        for (int n = n0; n < n1; ++n) acc += (double)phi[(size_t)n * kFeat + a] * (double)dz1[(size_t)n * kHid + b];
    } else if (p < kOffW2) {
        const int b = p - kOffB1;
        for (int n = n0; n < n1; ++n) acc += (double)dz1[(size_t)n * kHid + b];
    } else if (p < kOffB2) {
        const int q = p - kOffW2, a = q / kHid, b = q % kHid;
        for (int n = n0; n < n1; ++n)
            acc += (double)fmaxf(z1[(size_t)n * kHid + a], 0.0f) * (double)dz2[(size_t)n * kHid + b];
    } else if (p < kOffW3) {
        const int b = p - kOffB2;
        for (int n = n0; n < n1; ++n) acc += (double)dz2[(size_t)n * kHid + b];
    } else if (p < kOffB3) {
        const int q = p - kOffW3, a = q / kOut, c = q % kOut;
        for (int n = n0; n < n1; ++n)
            acc += (double)fmaxf(z2[(size_t)n * kHid + a], 0.0f) * (double)dg[(size_t)n * kOut + c];
    } else {
        const int c = p - kOffB3;
        for (int n = n0; n < n1; ++n) acc += (double)dg[(size_t)n * kOut + c];
    }
    partials[(size_t)chunk * kParams + p] = acc;
}

__global__ __launch_bounds__(kBlock) void k_param_final(int nchunks, const double *__restrict__ partials,
                                                        float *__restrict__ grad, float scale, int accumulate) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= kParams) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += partials[(size_t)c * kParams + p];
    const float v = (float)((double)scale * s);
    grad[p] = accumulate ? grad[p] + v : v;
}

__global__ __launch_bounds__(kBlock) void k_adam(int n, float *__restrict__ theta, const float *__restrict__ grad,
                                                 float *__restrict__ m, float *__restrict__ v, float lr, float b1,
                                                 float b2, float eps, float bc1, float bc2) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

__global__ __launch_bounds__(kBlock) void k_sub_from(int64_t n, const double *__restrict__ z, double *__restrict__ e) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) e[i] -= z[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline int nodes_grid(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

// theta32[i] = the BF16 value bits[i] widened to FP32 (exact: the 16 bits
// are the upper half of the FP32 pattern)
__global__ __launch_bounds__(kBlock) void k_bf16_widen(int n, const uint16_t *__restrict__ bits,
                                                       float *__restrict__ out) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = __uint_as_float(((uint32_t)bits[i]) << 16);
}

void launch_bf16_widen(int n, const uint16_t *bits, float *out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_bf16_widen, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, bits, out);
}

void launch_mlp_forward(int nb, const float *phi, const float *theta, float *z1, float *z2, float *g,
                        hipStream_t s) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_mlp_forward, dim3(nodes_grid(nb)), dim3(kBlock), 0, s, nb, phi, theta, z1, z2, g);
}

template <typename T>
void launch_assemble_blocks(int nb, const float *g, const double *L, T *M, const T *Mbj, float *t, int check,
                            int *nbad, hipStream_t s) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_assemble_blocks<T>, dim3(nodes_grid(nb)), dim3(kBlock), 0, s, nb, g, L, M, Mbj, t,
                       check, nbad);
}
template void launch_assemble_blocks<double>(int, const float *, const double *, double *, const double *,
                                             float *, int, int *, hipStream_t);
template void launch_assemble_blocks<float>(int, const float *, const double *, float *, const float *,
                                            float *, int, int *, hipStream_t);

void launch_block_resid(int nb, const double *S, const double *e, const double *r, double *w, hipStream_t s) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_block_resid, dim3(nodes_grid(nb)), dim3(kBlock), 0, s, nb, S, e, r, w);
}

int launch_dot_out(int64_t n, const double *a, const double *b, double *partials, int max_grid, double *out,
                   hipStream_t s) {
    int grid = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, max_grid);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_dot_partial, dim3(grid), dim3(kBlock), 0, s, n, a, b, partials);
    hipLaunchKernelGGL(k_sum_out, dim3(1), dim3(kBlock), 0, s, partials, grid, out);
    return grid;
}

void launch_loss_acc(double *scal, hipStream_t s) { hipLaunchKernelGGL(k_loss_acc, dim3(1), dim3(64), 0, s, scal); }

void launch_outer_acc(int nb, double *U, const double *q, const double *r, const double *coef, hipStream_t s) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_outer_acc, dim3(nodes_grid(nb)), dim3(kBlock), 0, s, nb, U, q, r, coef);
}

void launch_block_grad(int nb, const double *U, const double *L, const float *t, double inv_k, float *dg,
                       hipStream_t s) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_block_grad, dim3(nodes_grid(nb)), dim3(kBlock), 0, s, nb, U, L, t, inv_k, dg);
}

void launch_mlp_backward(int nb, const float *theta, const float *z1, const float *z2, const float *dg,
                         float *dz1, float *dz2, hipStream_t s) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_mlp_backward, dim3(nodes_grid(nb)), dim3(kBlock), 0, s, nb, theta, z1, z2, dg, dz1, dz2);
}

void launch_param_grad(int nb, const float *phi, const float *z1, const float *z2, const float *dg,
                       const float *dz1, const float *dz2, double *partials, float *grad, float scale,
                       int accumulate, hipStream_t s) {
    const int nchunks = std::max(1, (nb + kGradChunk - 1) / kGradChunk);
    const int pblocks = (kParams + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_param_partial, dim3(pblocks, nchunks), dim3(kBlock), 0, s, nb, phi, z1, z2, dg, dz1, dz2,
                       partials);
    hipLaunchKernelGGL(k_param_final, dim3(pblocks), dim3(kBlock), 0, s, nchunks, partials, grad, scale, accumulate);
}

void launch_adam(int n, float *theta, const float *grad, float *m, float *v, float lr, float beta1, float beta2,
                 float eps, float bc1, float bc2, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_adam, dim3(nodes_grid(n)), dim3(kBlock), 0, s, n, theta, grad, m, v, lr, beta1, beta2, eps,
                       bc1, bc2);
}

void launch_sub_from(int64_t n, const double *z, double *e, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_sub_from, dim3(nodes_grid(n)), dim3(kBlock), 0, s, n, z, e);
}

}  // namespace saamg
