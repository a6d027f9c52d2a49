// Learned warm start: per-cell network kernels (forward, backward, Adam) and
// the seed sampler.
//
// Network: 16 inputs -> 128 -> 128 -> 128 outputs (one logit per step), ReLU
// between layers, softmax over the steps 1..m of the instance.  Weights are
// used in bfloat16 (fp32 master copy for Adam); every product is
// bf16(A) * bf16(B) accumulated in fp32 on v_mfma_f32_16x16x16bf16_1k.
//
// Sampler: from quantised marginals q[c][t] (uint16, > 0) it draws one
// permutation per replica, step by step: W = sum of q[., t] over unvisited
// cells, u = word 0 of Philox(counter {t, r, instance id, 0}, key {seed, 4}),
// target = floor(u W / 2^32), and the step goes to the first unvisited cell
// (in free-list order) whose running sum exceeds the target.  Integer only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "uavq_device.h"
#include "uavq_internal.h"

namespace uavq {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// fp32 -> bf16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// C[M x N] = op(A)[M x K] op(B)[K x N] (+ bias[n]) with optional ReLU applied to
// A on load, output ReLU-mask by Zmask > 0, and accumulation into C.
// op(A)[i][k] = A[i * a_si + k * a_sk], op(B)[k][n] = B[k * b_sk + n * b_sn].
struct GemmArgs {
    const float *A;
    int64_t a_si, a_sk;
    const float *B;
    int64_t b_sk, b_sn;
    float *C;
    int64_t ldc;
    const float *bias;      // [N] or NULL
    const float *zmask;     // [M x ldz]: C *= (zmask > 0), or NULL
    int64_t ldz;
    int32_t M, N, K;
    int32_t relu_a;         // apply max(0, .) to A on load
    int32_t accumulate;     // C += result
    int32_t kchunk;         // > 0: split K into chunks of this length; chunk q's partial product goes to
    int64_t c_chunk;        //      C + q * c_chunk (no bias, mask or accumulation)
};

__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
    const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
    const int tilesM = (g.M + 15) >> 4, tilesN = (g.N + 15) >> 4;
    const int nchunk = g.kchunk > 0 ? (g.K + g.kchunk - 1) / g.kchunk : 1;
    const int64_t tile = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (tile >= (int64_t)tilesM * tilesN * nchunk) return;
    const int64_t tmn = tile % ((int64_t)tilesM * tilesN);
    const int q = (int)(tile / ((int64_t)tilesM * tilesN));
    const int tm = (int)(tmn % tilesM), tn = (int)(tmn / tilesM);
    const int ai = 16 * tm + li, bn = 16 * tn + li;
    const int kbeg = g.kchunk > 0 ? q * g.kchunk : 0;
    const int kend = g.kchunk > 0 ? min(g.K, kbeg + g.kchunk) : g.K;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = kbeg; k0 < kend; k0 += 16) {
        v4s av, bv;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int k = k0 + 4 * lg + j;
            float a = 0.f, b = 0.f;
            if (ai < g.M && k < kend) {
                a = g.A[ai * g.a_si + k * g.a_sk];
                if (g.relu_a) a = fmaxf(a, 0.f);
            }
            if (bn < g.N && k < kend) b = g.B[k * g.b_sk + bn * g.b_sn];
            av[j] = (short)bf16_bits(a);
            bv[j] = (short)bf16_bits(b);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; v++) {
        const int i = 16 * tm + 4 * lg + v;
        if (i < g.M && bn < g.N) {
            float c = acc[v];
            if (g.kchunk > 0) {
                g.C[q * g.c_chunk + i * g.ldc + bn] = c;
                continue;
            }
            if (g.bias) c += g.bias[bn];
            if (g.zmask && !(g.zmask[i * g.ldz + bn] > 0.f)) c = 0.f;
            float *dst = g.C + i * g.ldc + bn;
            *dst = g.accumulate ? *dst + c : c;
        }
    }
}

// Masked softmax over the first m[row] of 128 logits; writes probabilities,
// the per-row loss -log p[label] and the logit gradient (p - onehot) * scale.
__global__ __launch_bounds__(256) void k_softmax_ce(const float *Z, const int32_t *msteps, const int32_t *label,
                                                    int rows, float scale, float *P, float *G, float *row_loss) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= rows) return;
    const int m = msteps[row];
    const float *z = Z + (int64_t)row * 128;
    const float z0 = lane < m ? z[lane] : -INFINITY, z1 = lane + 64 < m ? z[lane + 64] : -INFINITY;
    float mx = fmaxf(z0, z1);
    for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    const float e0 = lane < m ? __expf(z0 - mx) : 0.f, e1 = lane + 64 < m ? __expf(z1 - mx) : 0.f;
    float s = e0 + e1;
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    const float p0 = e0 / s, p1 = e1 / s;
    if (P) {
        P[(int64_t)row * 128 + lane] = p0;
        P[(int64_t)row * 128 + lane + 64] = p1;
    }
    if (label) {
        const int lb = label[row];
        if (G) {
            G[(int64_t)row * 128 + lane] = (p0 - (lane == lb ? 1.f : 0.f)) * scale * (lane < m ? 1.f : 0.f);
            G[(int64_t)row * 128 + lane + 64] = (p1 - (lane + 64 == lb ? 1.f : 0.f)) * scale * (lane + 64 < m ? 1.f : 0.f);
        }
        if (lane == 0 && row_loss) row_loss[row] = logf(s) + mx - z[lb];
    }
}

// column sums of G [rows x n] (bias gradients); one thread per column
// Column sums of G[rows][n] in chunks of rchunk rows: block q writes the sums
// of its rows to part[q][n].
__global__ void k_colsum(const float *G, int rows, int n, int rchunk, float *part) {
    const int j = threadIdx.x, q = blockIdx.x;
    if (j >= n) return;
    const int i1 = min(rows, (q + 1) * rchunk);
    float s = 0.f;
    for (int i = q * rchunk; i < i1; i++) s += G[(int64_t)i * n + j];
    part[(int64_t)q * n + j] = s;
}

// out[j] = sum over q = 0..nq-1 (in this order) of part[q * stride + j]
__global__ void k_sum_parts(const float *part, int nq, int64_t stride, int64_t n, float *out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float s = 0.f;
    for (int q = 0; q < nq; q++) s += part[q * stride + j];
    out[j] = s;
}

__global__ void k_sum(const float *v, int n, float *out) {
    __shared__ float sh[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += v[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// Adam with bias correction on the fp32 master parameters
__global__ void k_adam(float *w, float *m1, float *m2, const float *g, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    w[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

// q[c][t] = floor(p[c][t] * 65534) + 1 (1..65535) for t < m (fp32 decision)
__global__ void k_quantize(const float *P, const int32_t *msteps, int rows, uint16_t *Q) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)rows * 128) return;
    const int row = (int)(i >> 7), t = (int)(i & 127);
    Q[i] = t < msteps[row] ? (uint16_t)(floorf(P[i] * 65534.0f) + 1.0f) : (uint16_t)0;
}

// One wavefront per (instance, seeded replica); lanes hold cells c and c + 64.
struct SampleArgs {
    const uint16_t *Q;          // per instance: m rows (cells) of 128 steps, at q_off[i]
    const int64_t *q_off;       // row offset (in rows of 128) of instance i
    const int32_t *m;           // per instance
    const uint32_t *inst_id;    // per instance
    const int64_t *state_off;   // word offset of replica 0 of instance i
    const int32_t *n_seeded;    // replicas 0 .. n_seeded[i]-1 are sampled
    int32_t n_inst, max_seeded;
    uint32_t seed;
    uint32_t *states;           // packed states (plan layout)
};

__global__ __launch_bounds__(256) void k_sample_seeds(SampleArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int inst = (int)(wid / a.max_seeded), r = (int)(wid % a.max_seeded);
    if (inst >= a.n_inst || r >= a.n_seeded[inst]) return;
    const int m = a.m[inst], W = (m + 31) >> 5;
    const uint16_t *q = a.Q + a.q_off[inst] * 128;
    uint32_t *st = a.states + a.state_off[inst] + (int64_t)r * m * W;
    bool used0 = lane >= m, used1 = lane + 64 >= m;
    for (int t = 1; t <= m; t++) {
        const uint32_t w0 = used0 ? 0u : q[lane * 128 + (t - 1)];
        const uint32_t w1 = used1 ? 0u : q[(lane + 64) * 128 + (t - 1)];
        // inclusive prefix sums in cell order: lanes 0..63 then 64..127
        uint64_t p0 = w0, p1 = w1;
        for (int off = 1; off < 64; off <<= 1) {
            const uint64_t y0 = __shfl_up(p0, off, 64), y1 = __shfl_up(p1, off, 64);
            if (lane >= off) {
                p0 += y0;
                p1 += y1;
            }
        }
        const uint64_t tot0 = __shfl(p0, 63, 64);
        p1 += tot0;
        const uint64_t Wt = __shfl(p1, 63, 64);
        const uint4 v = philox(make_uint4((uint32_t)t, (uint32_t)r, a.inst_id[inst], 0u), a.seed, 4u);
        const uint64_t target = ((uint64_t)v.x * Wt) >> 32;
        const uint64_t b0 = __ballot(!used0 && p0 > target), b1 = __ballot(!used1 && p1 > target);
        const int c = b0 ? __builtin_ctzll(b0) : 64 + __builtin_ctzll(b1);
        if (lane == (c & 63)) {
            if (c < 64) used0 = true;
            else used1 = true;
        }
        // row t-1 of the packed state: a single set bit at cell c
        for (int wd = lane; wd < W; wd += 64) st[(int64_t)(t - 1) * W + wd] = (wd == (c >> 5)) ? (1u << (c & 31)) : 0u;
    }
}

}  // namespace uavq

using namespace uavq;

extern "C" {

int uavq_mlp_param_count(void) { return 16 * 128 + 128 + 128 * 128 + 128 + 128 * 128 + 128; }

int uavq_mlp_workspace_bytes(int32_t rows, size_t *bytes) {
    if (rows < 0 || !bytes) return set_error(UAVQ_EINVAL, "mlp_workspace_bytes: bad argument");
    // Z1, Z2, Z3, P, G3, G2, G1 (rows x 128 each) + per-row loss + partial products of
    // the row-split gradient reductions (chunks of 128 rows)
    const size_t nq = ((size_t)rows + 127) / 128;
    *bytes = (size_t)rows * 128 * 4 * 7 + (size_t)rows * 4 + 256 + nq * 128 * 128 * 4 + nq * 128 * 4 + 256;
    return UAVQ_OK;
}

static int gemm(hipStream_t st, const float *A, int64_t a_si, int64_t a_sk, const float *B, int64_t b_sk, int64_t b_sn,
                float *C, int64_t ldc, int M, int N, int K, const float *bias, const float *zmask, int64_t ldz,
                int relu_a, int accumulate) {
    if (M <= 0 || N <= 0) return UAVQ_OK;
    GemmArgs g{A, a_si, a_sk, B, b_sk, b_sn, C, ldc, bias, zmask, ldz, M, N, K, relu_a, accumulate, 0, 0};
    const int64_t tiles = (int64_t)((M + 15) / 16) * ((N + 15) / 16);
    hipLaunchKernelGGL(k_gemm_bf16, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, st, g);
    UAVQ_HIP(hipGetLastError());
    return UAVQ_OK;
}

// C[M][N] = A^T-style product over a long K (the rows of a batch), split into
// chunks of 128 whose partial tiles are summed in chunk order: deterministic,
// and enough waves for the weight gradients.
static int gemm_rows(hipStream_t st, const float *A, int64_t a_si, int64_t a_sk, const float *B, int64_t b_sk,
                     int64_t b_sn, float *C, int M, int N, int K, int relu_a, float *part) {
    if (M <= 0 || N <= 0) return UAVQ_OK;
    const int nq = (K + 127) / 128;
    GemmArgs g{A, a_si, a_sk, B, b_sk, b_sn, part, N, nullptr, nullptr, 0, M, N, K, relu_a, 0, 128,
               (int64_t)M * N};
    const int64_t tiles = (int64_t)((M + 15) / 16) * ((N + 15) / 16) * nq;
    hipLaunchKernelGGL(k_gemm_bf16, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, st, g);
    UAVQ_HIP(hipGetLastError());
    const int64_t n = (int64_t)M * N;
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, nq, n, n, C);
    UAVQ_HIP(hipGetLastError());
    return UAVQ_OK;
}

static int colsum_rows(hipStream_t st, const float *G, int rows, float *out, float *part) {
    const int nq = (rows + 127) / 128;
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)nq), dim3(128), 0, st, G, rows, 128, 128, part);
    UAVQ_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(128), 0, st, part, nq, (int64_t)128, (int64_t)128, out);
    UAVQ_HIP(hipGetLastError());
    return UAVQ_OK;
}

struct MlpView {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
};
static MlpView view(const float *p) {
    MlpView v;
    v.W1 = p;
    v.b1 = v.W1 + 16 * 128;
    v.W2 = v.b1 + 128;
    v.b2 = v.W2 + 128 * 128;
    v.W3 = v.b2 + 128;
    v.b3 = v.W3 + 128 * 128;
    return v;
}

static int forward(const float *params, const float *X, int rows, float *Z1, float *Z2, float *Z3, hipStream_t st) {
    const MlpView w = view(params);
    int rc;
    if ((rc = gemm(st, X, 16, 1, w.W1, 128, 1, Z1, 128, rows, 128, 16, w.b1, nullptr, 0, 0, 0))) return rc;
    if ((rc = gemm(st, Z1, 128, 1, w.W2, 128, 1, Z2, 128, rows, 128, 128, w.b2, nullptr, 0, 1, 0))) return rc;
    return gemm(st, Z2, 128, 1, w.W3, 128, 1, Z3, 128, rows, 128, 128, w.b3, nullptr, 0, 1, 0);
}

int uavq_mlp_forward(const float *d_params, const float *d_X, const int32_t *d_m, int32_t rows, float *d_probs,
                     void *d_ws, size_t ws_bytes, void *stream) {
    size_t need = 0;
    if (!d_params || !d_X || !d_m || !d_probs || rows < 0 || uavq_mlp_workspace_bytes(rows, &need) ||
        ws_bytes < need || (rows > 0 && !d_ws))
        return set_error(UAVQ_EINVAL, "mlp_forward: bad argument");
    if (rows == 0) return UAVQ_OK;
    hipStream_t st = (hipStream_t)stream;
    float *Z1 = (float *)d_ws, *Z2 = Z1 + (size_t)rows * 128, *Z3 = Z2 + (size_t)rows * 128;
    int rc = forward(d_params, d_X, rows, Z1, Z2, Z3, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_softmax_ce, dim3((rows + 3) / 4), dim3(256), 0, st, Z3, d_m, nullptr, rows, 0.f, d_probs,
                       nullptr, nullptr);
    UAVQ_HIP(hipGetLastError());
    return UAVQ_OK;
}

int uavq_mlp_loss_grad(const float *d_params, const float *d_X, const int32_t *d_m, const int32_t *d_label,
                       int32_t rows, float *d_grad, float *d_loss, void *d_ws, size_t ws_bytes, void *stream) {
    size_t need = 0;
    if (!d_params || !d_X || !d_m || !d_label || !d_grad || !d_loss || rows < 1 ||
        uavq_mlp_workspace_bytes(rows, &need) || ws_bytes < need || !d_ws)
        return set_error(UAVQ_EINVAL, "mlp_loss_grad: bad argument");
    hipStream_t st = (hipStream_t)stream;
    const size_t L = (size_t)rows * 128;
    float *Z1 = (float *)d_ws, *Z2 = Z1 + L, *Z3 = Z2 + L, *P = Z3 + L, *G3 = P + L, *G2 = G3 + L, *G1 = G2 + L;
    float *rl = G1 + L;
    const size_t nq = ((size_t)rows + 127) / 128;
    float *gpart = (float *)(((uintptr_t)(rl + rows) + 255) & ~(uintptr_t)255);   // nq x 128 x 128
    float *cpart = gpart + nq * 128 * 128;                                          // nq x 128
    int rc = forward(d_params, d_X, rows, Z1, Z2, Z3, st);
    if (rc) return rc;
    const float scale = 1.0f / (float)rows;
    hipLaunchKernelGGL(k_softmax_ce, dim3((rows + 3) / 4), dim3(256), 0, st, Z3, d_m, d_label, rows, scale, P, G3, rl);
    UAVQ_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, rl, rows, d_loss);
    UAVQ_HIP(hipGetLastError());
    const MlpView w = view(d_params);
    float *gW1 = d_grad, *gb1 = gW1 + 16 * 128, *gW2 = gb1 + 128, *gb2 = gW2 + 128 * 128, *gW3 = gb2 + 128,
          *gb3 = gW3 + 128 * 128;
    // layer 3: dW3 = relu(Z2)^T G3, db3 = colsum G3, G2 = (G3 W3^T) * [Z2 > 0]
    if ((rc = gemm_rows(st, Z2, 1, 128, G3, 128, 1, gW3, 128, 128, rows, 1, gpart))) return rc;
    if ((rc = colsum_rows(st, G3, rows, gb3, cpart))) return rc;
    if ((rc = gemm(st, G3, 128, 1, w.W3, 1, 128, G2, 128, rows, 128, 128, nullptr, Z2, 128, 0, 0))) return rc;
    // layer 2
    if ((rc = gemm_rows(st, Z1, 1, 128, G2, 128, 1, gW2, 128, 128, rows, 1, gpart))) return rc;
    if ((rc = colsum_rows(st, G2, rows, gb2, cpart))) return rc;
    if ((rc = gemm(st, G2, 128, 1, w.W2, 1, 128, G1, 128, rows, 128, 128, nullptr, Z1, 128, 0, 0))) return rc;
    // layer 1
    if ((rc = gemm_rows(st, d_X, 1, 16, G1, 128, 1, gW1, 16, 128, rows, 0, gpart))) return rc;
    if ((rc = colsum_rows(st, G1, rows, gb1, cpart))) return rc;
    return UAVQ_OK;
}

int uavq_mlp_adam(float *d_params, float *d_m1, float *d_m2, const float *d_grad, int32_t step, float lr,
                  void *stream) {
    if (!d_params || !d_m1 || !d_m2 || !d_grad || step < 1 || !(lr > 0.f))
        return set_error(UAVQ_EINVAL, "mlp_adam: bad argument");
    const int n = uavq_mlp_param_count();
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_params, d_m1, d_m2, d_grad,
                       n, lr, b1, b2, 1e-8f, c1, c2);
    UAVQ_HIP(hipGetLastError());
    return UAVQ_OK;
}

int uavq_quantize_marginals(const float *d_probs, const int32_t *d_m, int32_t rows, uint16_t *d_q, void *stream) {
    if (rows < 0 || (rows > 0 && (!d_probs || !d_m || !d_q))) return set_error(UAVQ_EINVAL, "quantize: bad argument");
    if (rows == 0) return UAVQ_OK;
    const int64_t n = (int64_t)rows * 128;
    hipLaunchKernelGGL(k_quantize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, d_probs, d_m,
                       rows, d_q);
    UAVQ_HIP(hipGetLastError());
    return UAVQ_OK;
}

int uavq_sample_seeds(const uavq_plan *pl, const uint16_t *d_q, const int64_t *q_row_off, const int32_t *n_seeded,
                      uint32_t *d_states, void *d_scratch, size_t scratch_bytes, void *stream) {
    if (!pl || !d_q || !q_row_off || !n_seeded || !d_states) return set_error(UAVQ_EINVAL, "sample_seeds: bad argument");
    const int n = pl->n_inst;
    if (n == 0) return UAVQ_OK;
    int maxs = 0;
    for (int i = 0; i < n; i++) {
        if (n_seeded[i] < 0 || n_seeded[i] > pl->desc[i].nrep)
            return set_error(UAVQ_EINVAL, "sample_seeds: n_seeded[%d] out of range", i);
        if (pl->desc[i].m > 128) return set_error(UAVQ_ETOOBIG, "sample_seeds: m > 128");
        maxs = std::max(maxs, n_seeded[i]);
    }
    if (maxs == 0) return UAVQ_OK;
    // small per-instance tables staged in the caller's scratch buffer
    const size_t need = (size_t)n * (8 + 4 + 4 + 8 + 4) + 64;
    if (!d_scratch || scratch_bytes < need) return set_error(UAVQ_EINVAL, "sample_seeds: scratch needs %zu bytes", need);
    std::vector<int64_t> qo(q_row_off, q_row_off + n), so(n);
    std::vector<int32_t> mm(n), ns(n_seeded, n_seeded + n);
    std::vector<uint32_t> ids(n);
    for (int i = 0; i < n; i++) {
        mm[i] = pl->desc[i].m;
        ids[i] = pl->desc[i].inst_id;
        so[i] = pl->desc[i].state_off;
    }
    uint8_t *s = (uint8_t *)d_scratch;
    int64_t *dqo = (int64_t *)s;            s += 8 * (size_t)n;
    int64_t *dso = (int64_t *)s;            s += 8 * (size_t)n;
    int32_t *dm = (int32_t *)s;             s += 4 * (size_t)n;
    int32_t *dns = (int32_t *)s;            s += 4 * (size_t)n;
    uint32_t *did = (uint32_t *)s;
    hipStream_t st = (hipStream_t)stream;
    UAVQ_HIP(hipMemcpyAsync(dqo, qo.data(), 8 * (size_t)n, hipMemcpyHostToDevice, st));
    UAVQ_HIP(hipMemcpyAsync(dso, so.data(), 8 * (size_t)n, hipMemcpyHostToDevice, st));
    UAVQ_HIP(hipMemcpyAsync(dm, mm.data(), 4 * (size_t)n, hipMemcpyHostToDevice, st));
    UAVQ_HIP(hipMemcpyAsync(dns, ns.data(), 4 * (size_t)n, hipMemcpyHostToDevice, st));
    UAVQ_HIP(hipMemcpyAsync(did, ids.data(), 4 * (size_t)n, hipMemcpyHostToDevice, st));
    SampleArgs a{d_q, dqo, dm, did, dso, dns, n, maxs, pl->p.seed, d_states};
    const int64_t waves = (int64_t)n * maxs;
    hipLaunchKernelGGL(k_sample_seeds, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, a);
    UAVQ_HIP(hipGetLastError());
    // pageable copies above are complete once the stream reaches the kernel; keep the host vectors alive until then
    UAVQ_HIP(hipStreamSynchronize(st));
    return UAVQ_OK;
}

}  // extern "C"
