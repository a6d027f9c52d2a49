// MFMA field/energy refresh and the dense-field Metropolis sweep (gfx950).
//
// The one dense contraction of the method is the local-field / energy
// refresh.  Couplings and costs are non-negative integers; they are split
// into int8 limbs (v = lo + 128 hi, lo = v & 127, hi = v >> 7) and contracted
// against the 0/1 state with v_mfma_i32_16x16x32_i8, accumulating in int32:
// the result is exact.
//
//   energy refresh (any packed states):  Z = X D per state (X: steps x cells,
//     D: cell costs, symmetric), travel = sum_t <Z_t, x_{t+1}> plus the
//     start-cell legs; penalties from the step/cell occupation counts.
//   dense refresh (dense kernel):        H = b + J X across replicas.
//
// MFMA operand layout (16x16x32, 64-bit A/B per lane): lane l holds
// A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16] in byte j, and the
// result D[4 (l / 16) + v][l % 16] in accumulator v.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <mutex>

#include "uavq_device.h"
#include "uavq_internal.h"

namespace uavq {

typedef int v4i __attribute__((ext_vector_type(4)));

// 8 bits -> 8 bytes of 0/1 (byte j = bit j)
__device__ __forceinline__ uint64_t spread8(uint32_t b) {
    uint64_t v = 0;
#pragma unroll
    for (int j = 0; j < 8; j++) v |= (uint64_t)((b >> j) & 1u) << (8 * j);
    return v;
}

// ------------------------------------------------------- energy refresh --
// One wavefront per state.  LDS holds the cost matrix as two byte limbs
// (row-major, rows padded to Kp = 32-multiple) and the start-cell costs.
struct EnergyArgs {
    const uint32_t *states;     // n states, state_words apart
    int64_t n;
    int64_t *E;
    const uint8_t *D;           // m*m
    const uint8_t *ddep;        // m
    int32_t m, W, P, closed, Kp;
    int64_t c0;
};

__global__ __launch_bounds__(256) void k_energy_refresh(EnergyArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int m = a.m, W = a.W, Kp = a.Kp;
    uint8_t *lo = smem;                       // [m][Kp]
    uint8_t *hi = smem + (size_t)m * Kp;      // [m][Kp]
    uint8_t *dep = hi + (size_t)m * Kp;       // [m]
    for (int i = threadIdx.x; i < m * Kp; i += blockDim.x) {
        const int c = i / Kp, k = i % Kp;
        const int v = k < m ? a.D[c * m + k] : 0;
        lo[i] = (uint8_t)(v & 127);
        hi[i] = (uint8_t)(v >> 7);
    }
    for (int i = threadIdx.x; i < m; i += blockDim.x) dep[i] = a.ddep[i];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int64_t st = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (st >= a.n) return;
    const uint32_t *x = a.states + st * (int64_t)(m * W);
    const int li = lane & 15, lg = lane >> 4;
    const int tiles = (m + 15) >> 4;

    int64_t travel = 0;
    // Z = X D, tile by tile; the epilogue multiplies by the next step's bits
    for (int tt = 0; tt < tiles; tt++) {
        const int trow = 16 * tt + li;   // 0-based step of the A row held by this lane
        for (int tc = 0; tc < tiles; tc++) {
            const int ccol = 16 * tc + li;   // cell of the B column held by this lane
            v4i acc_lo = {0, 0, 0, 0}, acc_hi = {0, 0, 0, 0};
            for (int kb = 0; kb < Kp; kb += 32) {
                const int k0 = kb + 8 * lg;
                uint64_t av = 0;
                if (trow < m && k0 < m) {
                    const uint32_t word = x[trow * W + (k0 >> 5)];
                    uint32_t bits = (word >> (k0 & 31)) & 0xFFu;
                    if (k0 + 8 > m) bits &= (1u << (m - k0)) - 1u;
                    av = spread8(bits);
                }
                uint64_t blo = 0, bhi = 0;
                if (ccol < m) {
                    blo = *reinterpret_cast<const uint64_t *>(lo + (size_t)ccol * Kp + k0);
                    bhi = *reinterpret_cast<const uint64_t *>(hi + (size_t)ccol * Kp + k0);
                }
                acc_lo = __builtin_amdgcn_mfma_i32_16x16x32_i8((long)av, (long)blo, acc_lo, 0, 0, 0);
                acc_hi = __builtin_amdgcn_mfma_i32_16x16x32_i8((long)av, (long)bhi, acc_hi, 0, 0, 0);
            }
            // lane holds Z[t = 16 tt + 4 lg + v][c = 16 tc + li]; times x_{t+1, c}
            const int c = 16 * tc + li;
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int t0 = 16 * tt + 4 * lg + v;   // 0-based step t0 (= step t0+1)
                if (c < m && t0 + 1 < m) {
                    const int z = acc_lo[v] + 128 * acc_hi[v];
                    const uint32_t nb = (x[(t0 + 1) * W + (c >> 5)] >> (c & 31)) & 1u;
                    travel += (int64_t)z * nb;
                }
            }
        }
    }
    // start-cell legs, occupation penalties and the linear -2P terms
    int64_t rest = 0;
    for (int c = lane; c < m; c += 64) {
        const uint32_t x1 = (x[0 * W + (c >> 5)] >> (c & 31)) & 1u;
        const uint32_t xm = (x[(m - 1) * W + (c >> 5)] >> (c & 31)) & 1u;
        rest += (int64_t)dep[c] * x1;
        if (a.closed) rest += (int64_t)dep[c] * xm;
        int C = 0;
        for (int t = 0; t < m; t++) C += (x[t * W + (c >> 5)] >> (c & 31)) & 1u;
        rest += (int64_t)a.P * C * (C - 1);
    }
    for (int t = lane; t < m; t += 64) {
        int R = 0;
        for (int w = 0; w < W; w++) R += __popc(x[t * W + w]);
        rest += (int64_t)a.P * R * (R - 1) - 2LL * a.P * R;
    }
    const int64_t tot = wave_sum64(travel + rest);
    if (lane == 0) a.E[st] = a.c0 + tot;
}

static size_t energy_lds(int m) {
    const int Kp = (m + 31) / 32 * 32;
    return 2 * (size_t)m * Kp + (size_t)m + 16;
}

int launch_energy_refresh(const uint32_t *d_states, int64_t n, int64_t *d_E, const uint8_t *d_D, const uint8_t *d_dep,
                          int m, int P, int closed, int64_t c0, hipStream_t st) {
    if (n <= 0) return UAVQ_OK;
    EnergyArgs a{};
    a.states = d_states;
    a.n = n;
    a.E = d_E;
    a.D = d_D;
    a.ddep = d_dep;
    a.m = m;
    a.W = (m + 31) / 32;
    a.P = P;
    a.closed = closed;
    a.Kp = (m + 31) / 32 * 32;
    a.c0 = c0;
    const size_t lds = energy_lds(m);
    if (lds > 160 * 1024) return set_error(UAVQ_ETOOBIG, "energy refresh: m = %d too large", m);
    UAVQ_HIP(hipFuncSetAttribute((const void *)k_energy_refresh, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int wpb = 4;
    const int64_t blocks = (n + wpb - 1) / wpb;
    hipLaunchKernelGGL(k_energy_refresh, dim3((unsigned)blocks), dim3(64 * wpb), lds, st, a);
    UAVQ_HIP(hipGetLastError());
    return UAVQ_OK;
}

// -------------------------------------------------------- dense refresh --
// Xb[r][l] (bytes, rows of Np) from the packed states of one instance.
__global__ __launch_bounds__(256) void k_unpack_states(const uint32_t *states, int R, int m, int W, int Np,
                                                       uint8_t *Xb) {
    const int64_t total = (int64_t)R * Np;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / Np), l = (int)(i % Np);
        uint8_t v = 0;
        if (l < m * m) {
            const int t = l / m, c = l % m;
            v = (uint8_t)((states[(int64_t)r * m * W + t * W + (c >> 5)] >> (c & 31)) & 1u);
        }
        Xb[i] = v;
    }
}

// H[r][k] = b_k + sum_l J[k][l] X[l][r]; one wavefront per 16x16 output tile.
__global__ __launch_bounds__(256) void k_refresh_dense(const int8_t *Jlo, const int8_t *Jhi, const int32_t *b,
                                                       const uint8_t *Xb, int N, int Np, int R, int32_t *H) {
    const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
    const int tilesK = Np >> 4, tilesR = (R + 15) >> 4;
    const int64_t tile = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (tile >= (int64_t)tilesK * tilesR) return;
    const int tk = (int)(tile % tilesK), tr = (int)(tile / tilesK);
    const int krow = 16 * tk + li;          // A row (output row k)
    const int rcol = 16 * tr + li;          // B column (replica)
    v4i acc_lo = {0, 0, 0, 0}, acc_hi = {0, 0, 0, 0};
    const int8_t *alo = Jlo + (int64_t)krow * Np;
    const int8_t *ahi = Jhi + (int64_t)krow * Np;
    const uint8_t *bx = Xb + (int64_t)(rcol < R ? rcol : 0) * Np;
    for (int kb = 0; kb < Np; kb += 32) {
        const int k0 = kb + 8 * lg;
        const long a_lo = *reinterpret_cast<const long *>(alo + k0);
        const long a_hi = *reinterpret_cast<const long *>(ahi + k0);
        const long bv = rcol < R ? *reinterpret_cast<const long *>(bx + k0) : 0;
        acc_lo = __builtin_amdgcn_mfma_i32_16x16x32_i8(a_lo, bv, acc_lo, 0, 0, 0);
        acc_hi = __builtin_amdgcn_mfma_i32_16x16x32_i8(a_hi, bv, acc_hi, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; v++) {
        const int k = 16 * tk + 4 * lg + v;
        if (k < N && rcol < R) H[(int64_t)rcol * N + k] = b[k] + acc_lo[v] + 128 * acc_hi[v];
    }
}

// ---------------------------------------------------------- dense sweep --
// One replica per wavefront; h (N int32) in LDS, state bits in registers
// (lane L holds x_{L + 64 i} in bit i), 64-site windows in site order.  On an
// accept the J row (int16, global memory) is added to h.
struct DenseArgs {
    KArgs k;
    const int32_t *H;            // refreshed fields of this instance, [R][N]
    const int16_t *J;            // N*N
    const int32_t *b;            // N
    int32_t inst;                // instance index
};

__global__ __launch_bounds__(1024) void k_sweep_dense(DenseArgs da) {
    extern __shared__ __align__(16) uint8_t smem[];
    const KArgs &a = da.k;
    const InstDesc d = a.desc[da.inst];
    const int m = d.m, N = m * m, W = d.row_words;
    const int wave = threadIdx.x >> 6, L = threadIdx.x & 63;
    const int nthr = blockDim.x, nw = nthr >> 6;
    const int Ts = a.thr_stride;
    // this instance's schedule: sweep s reads table row sched_row + s * sched_step
    const int srow = d.sched_row, dstep = d.sched_step;
    uint32_t *sthr = reinterpret_cast<uint32_t *>(smem);
    int32_t *h = reinterpret_cast<int32_t *>(smem + 8 * (size_t)Ts) + (size_t)wave * N;
    __shared__ int s_first_sh;

    const int r = blockIdx.x * nw + wave;
    const bool active = r < d.nrep;
    const int64_t grep = d.rep_base + r;
    const int s0 = active ? max(a.start_sweep ? a.start_sweep[grep] : 0, a.s_begin) : a.s_end;
    if (threadIdx.x == 0) s_first_sh = a.s_end;
    __syncthreads();
    if (L == 0) atomicMin(&s_first_sh, s0);
    __syncthreads();
    const int s_first = s_first_sh;
    if (s_first < a.s_end) {
        const int n = a.dcut[srow + s_first * dstep];
        for (int i = threadIdx.x; i < n; i += nthr) sthr[(s_first & 1) * Ts + i] = a.thr[(size_t)(srow + s_first * dstep) * Ts + i];
    }

    uint32_t *st = a.states + d.state_off + (int64_t)r * d.state_words;
    uint64_t xb = 0;   // bit i: x_{L + 64 i}
    int64_t E = 0;
    const int nwin = (N + 63) >> 6;
    if (active) {
        int64_t part = 0;
        for (int i = 0; i < nwin; i++) {
            const int k = 64 * i + L;
            if (k < N) {
                const int t = k / m, c = k % m;
                const uint32_t x = (st[t * W + (c >> 5)] >> (c & 31)) & 1u;
                xb |= (uint64_t)x << i;
                const int hk = da.H[(int64_t)r * N + k];
                h[k] = hk;
                if (x) part += (int64_t)hk + da.b[k];
            }
        }
        // E = c0 + (1/2) sum_k x_k (h_k + b_k)
        E = d.c0 + wave_sum64(part) / 2;
        if (!a.resume) {   // the best state starts as the initial state
            uint32_t *bs = a.best_states + d.state_off + (int64_t)r * d.state_words;
            for (int i = L; i < d.state_words; i += 64) bs[i] = st[i];
        }
    }
    __syncthreads();

    // best so far and counters: fresh, or those of the previous segment
    int64_t bestE = LLONG_MAX;
    int bestS = -1;
    bool improved = false;   // the best state changed in this launch
    uint64_t bestxb = xb, nacc = 0, ndraw = 0;
    if (active && a.resume) {
        bestE = a.best_E[grep];
        bestS = a.best_sweep[grep];
        nacc = a.accepts[grep];
        ndraw = a.draws[grep];
    }
    for (int s = s_first; s < a.s_end; s++) {
        const uint32_t *thr = sthr + (s & 1) * Ts;
        const int dcut = a.dcut[srow + s * dstep];
        if (active && s >= s0) {
            for (int i = 0; i < nwin; i++) {
                const int k = 64 * i + L;
                const bool in = k < N;
                const int t = k / m + 1, c = k % m;
                uint64_t open = __ballot(in);
                bool have_u = false;
                uint32_t u = 0;
                while (open) {
                    const int hk = in ? h[k] : 0;
                    const int xk = (int)((xb >> i) & 1ull);
                    const int dE = xk ? -hk : hk;
                    const bool mine = (open >> L) & 1ull;
                    uint64_t accm = __ballot(mine && dE <= 0);
                    const bool need = mine && dE > 0 && dE < dcut;
                    const uint64_t needm = __ballot(need);
                    if (needm) {
                        if (need && !have_u) {
                            uint32_t cb = (uint32_t)c + 65536u * (uint32_t)((t - 1) >> 2);
                            asm volatile("" : "+v"(cb));
                            const uint4 v = philox(make_uint4(cb, (uint32_t)s, (uint32_t)r, d.inst_id), a.seed, 0u);
                            const int w = (t - 1) & 3;
                            u = w == 0 ? v.x : (w == 1 ? v.y : (w == 2 ? v.z : v.w));
                            have_u = true;
                        }
                        const uint32_t thv = need ? thr[dE] : 0u;
                        accm |= __ballot(need && u < thv);
                    }
                    if (!accm) {
                        ndraw += __popcll(needm);
                        break;
                    }
                    const int Ls = __builtin_ctzll(accm);
                    const uint64_t upto = Ls == 63 ? ~0ull : ((2ull << Ls) - 1ull);
                    ndraw += __popcll(needm & upto);
                    const int dEs = __builtin_amdgcn_readlane(dE, Ls);
                    const int xs = __builtin_amdgcn_readlane(xk, Ls);
                    E += dEs;
                    nacc++;
                    const int ks = 64 * i + Ls;
                    if (L == Ls) xb ^= 1ull << i;
                    const int sign = xs ? -1 : 1;
                    const int16_t *jr = da.J + (int64_t)ks * N;
                    for (int l = L; l < N; l += 64) h[l] += sign * (int)jr[l];
                    open &= ~upto;
                }
            }
            if (E < bestE) {
                bestE = E;
                bestS = s;
                bestxb = xb;
                improved = true;
            }
        }
        if (s + 1 < a.s_end) {
            const int n = a.dcut[srow + (s + 1) * dstep];
            uint32_t *dst = sthr + ((s + 1) & 1) * Ts;
            const uint32_t *src = a.thr + (size_t)(srow + (s + 1) * dstep) * Ts;
            for (int i2 = threadIdx.x; i2 < n; i2 += nthr) dst[i2] = src[i2];
        }
        __syncthreads();
    }
    if (active) {
        // site bits -> packed rows (each row word assembled by ballots)
        uint32_t *bs = a.best_states + d.state_off + (int64_t)r * d.state_words;
        for (int w = 0; w < d.state_words; w++) {
            const int t = w / W, c0 = 32 * (w % W);
            uint32_t fw = 0u, bw = 0u;
            for (int j = 0; j < 32 && c0 + j < m; j++) {
                const int k = t * m + c0 + j;
                const int owner = k & 63, idx = k >> 6;
                const uint32_t fb = (uint32_t)__builtin_amdgcn_readlane((int)((xb >> idx) & 1ull), owner);
                const uint32_t bb = (uint32_t)__builtin_amdgcn_readlane((int)((bestxb >> idx) & 1ull), owner);
                fw |= fb << j;
                bw |= bb << j;
            }
            if (L == 0) {
                st[w] = fw;
                if (improved) bs[w] = bw;
            }
        }
        if (L == 0) {
            a.final_E[grep] = E;
            a.best_E[grep] = bestE;
            a.best_sweep[grep] = bestS;
            a.accepts[grep] = nacc;
            a.draws[grep] = ndraw;
        }
    }
}

int launch_dense(const uavq_plan *pl, const KArgs &a, hipStream_t st) {
    const int wpb = pl->waves_per_block[1];
    for (int i = 0; i < pl->n_inst; i++) {
        const InstDesc &d = pl->desc[i];
        const int N = d.m * d.m, Np = (N + 31) / 32 * 32, R = d.nrep;
        uint8_t *Xb = (uint8_t *)a.ws + pl->dense_xb_off;
        int32_t *H = (int32_t *)((uint8_t *)a.ws + pl->dense_h_off);
        const int8_t *Jlo = (const int8_t *)(a.ws + d.Jlimb_off);
        const int8_t *Jhi = Jlo + (int64_t)Np * Np;
        hipLaunchKernelGGL(k_unpack_states, dim3(1024), dim3(256), 0, st, a.states + d.state_off, R, d.m, d.row_words,
                           Np, Xb);
        UAVQ_HIP(hipGetLastError());
        const int64_t tiles = (int64_t)(Np / 16) * ((R + 15) / 16);
        hipLaunchKernelGGL(k_refresh_dense, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, st, Jlo, Jhi,
                           (const int32_t *)(a.ws + d.b_off), Xb, N, Np, R, H);
        UAVQ_HIP(hipGetLastError());
        DenseArgs da{a, H, (const int16_t *)(a.ws + d.J_off), (const int32_t *)(a.ws + d.b_off), i};
        const size_t lds = 8 * (size_t)pl->thr_stride + (size_t)wpb * N * 4;
        if (lds > 160 * 1024) return set_error(UAVQ_ETOOBIG, "dense kernel: LDS need %zu bytes (N = %d)", lds, N);
        UAVQ_HIP(hipFuncSetAttribute((const void *)k_sweep_dense, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        if (pl->timing && i == 0) UAVQ_HIP(hipEventRecord((hipEvent_t)pl->ev[2], st));
        hipLaunchKernelGGL(k_sweep_dense, dim3((R + wpb - 1) / wpb), dim3(64 * wpb), lds, st, da);
        if (pl->timing && i == pl->n_inst - 1) UAVQ_HIP(hipEventRecord((hipEvent_t)pl->ev[3], st));
        UAVQ_HIP(hipGetLastError());
    }
    return UAVQ_OK;
}

}  // namespace uavq

// ------------------------------------------- allocation-free energy_eval --
// Staging of uavq_energy_eval_dev_noalloc: the cost matrix and the start-cell
// costs of the last call, in a file-scope device array instead of a caller
// workspace.  Every device the library runs on holds its own copy until the
// process ends; its address is looked up once per device with that device
// current and kept per device.  80 KiB covers every field the refresh kernel
// takes (its LDS tile reaches m = 283: 80,128 + 512 bytes of staging).
namespace uavq {

constexpr size_t kNoAllocScratchBytes = 80 * 1024;
constexpr int kNoAllocMaxDevices = 64;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static uint8_t *g_scratch_ptr[kNoAllocMaxDevices] = {};

static int scratch_for_current_device(uint8_t **out) {
    int dev = 0;
    UAVQ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices)
        return set_error(UAVQ_EINVAL, "energy_eval_dev_noalloc: device %d beyond the %d supported", dev,
                         kNoAllocMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(UAVQ_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<uint8_t *>(p);
    }
    *out = g_scratch_ptr[dev];
    return UAVQ_OK;
}

}  // namespace uavq

extern "C" int uavq_energy_eval_dev_noalloc(const uavq_qubo *q, const uint32_t *d_x, int64_t n, int64_t *d_E,
                                            void *stream) {
    using namespace uavq;
    if (!q || n < 0 || (n > 0 && (!d_x || !d_E)))
        return set_error(UAVQ_EINVAL, "energy_eval_dev_noalloc: bad argument");
    const size_t need = energy_ws_bytes(q);
    if (need > kNoAllocScratchBytes)
        return set_error(UAVQ_ETOOBIG, "energy_eval_dev_noalloc: m = %d needs %zu bytes of staging, the static "
                         "buffer holds %zu", q->m, need, kNoAllocScratchBytes);
    if (n == 0) return UAVQ_OK;
    uint8_t *ptr = nullptr;
    const int rc = scratch_for_current_device(&ptr);
    if (rc) return rc;
    return launch_energy(q, d_x, n, d_E, ptr, kNoAllocScratchBytes, stream);
}
