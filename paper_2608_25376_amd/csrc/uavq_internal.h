// Internal structures shared by the host code and the HIP kernels of libuavq.
#pragma once
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/uavq.h"
#include "uavq_kargs.h"

typedef struct ihipStream_t *hipStream_t_opaque;


struct uavq_qubo {
    int32_t rows, cols, depot, scale;
    int32_t m, N, P, wmax, closed, row_words;
    int64_t c0;
    std::vector<int32_t> F;      // m grid indices
    std::vector<int32_t> W;      // (m+1)^2 costs over [start, F...]
    std::vector<uint8_t> D;      // m*m costs between free cells as bytes (empty when w_max > 255)
    std::vector<uint8_t> ddep;   // m costs start -> free cell as bytes (empty when w_max > 255)
    std::vector<uint16_t> D16;   // the same costs, 16-bit (always)
    std::vector<uint16_t> ddep16;
    std::vector<int32_t> b;      // N linear terms
    std::vector<int16_t> J;      // N*N dense couplings (optional)
};

// LDS bytes of a workgroup of the m <= 64 sweep with wpb replicas: the table row, D and the start-cell costs as
// bytes, the signed cost rows (2m rows of 64 int16), and per replica the travel rows of steps 1..m plus 8 boundary
// rows (64 int16 each) and 68 step counts
inline size_t ylds_lds_bytes_for(size_t thr_stride, int m, int wpb) {
    auto a16 = [](size_t v) { return (v + 15) & ~(size_t)15; };
    return a16(4 * thr_stride + a16((size_t)m * m) + a16((size_t)m) + 256 * (size_t)m + (size_t)wpb * 64 * (m + 8) * 2) +
           (size_t)wpb * 68 * 4;
}

struct uavq_plan {
    uavq_anneal_params p;
    int32_t n_inst, S, Dmax, thr_stride;
    int32_t thr_rows;                     // rows of the table (all instances' schedules)
    std::vector<double> sched_T;          // per instance: T0_i, T1_i
    std::vector<uint8_t> blob;            // static data, uploaded verbatim at offset 0
    size_t thr_off, dcut_off, desc_off, items_off, inst_state_off_off;
    size_t blob_bytes;                    // aligned size of blob
    size_t e_init_off;                    // int64 per replica
    size_t dense_xb_off, dense_h_off;     // dense kernel: unpacked states, refreshed fields
    size_t ws_bytes;
    std::vector<uavq::InstDesc> desc;
    std::vector<uavq::WorkItem> items;    // ordered by chunk class, then LPT
    int32_t class_begin[uavq::kMaxChunks + 2];   // items of chunk class j: [class_begin[j], class_begin[j+1])
    int32_t waves_per_block[uavq::kMaxChunks + 1];
    int64_t total_rep, total_state_words;
    std::vector<int64_t> rep_offset, state_offset, inst_state_off;
    int32_t max_m, dense;
    int32_t variant;                      // UAVQ_VARIANT_* (kernel choice; never changes results)
    int32_t timing = 0;                   // record events around the sweep launches
    void *ev[2 * (uavq::kMaxChunks + 1)] = {};
    int32_t persistent = 0, graph = 0;
    // Caches filled on first use (launch shape, captured graph) are guarded by
    // mu, so that one plan may be used from several threads.
    std::mutex mu;
    int32_t prepared = 0, cu_count = 0;
    int32_t max_blocks[uavq::kMaxChunks + 2] = {};   // resident blocks per CU of each class's kernel
    size_t lds_class[uavq::kMaxChunks + 2] = {};
    int32_t pw_class[uavq::kMaxChunks + 2] = {};   // the class's block-tested sweep keeps packed draw words in LDS
    int32_t ylds_w1 = 0;         // the m <= 64 sweep runs at one wave per SIMD (launch fits the chip)
    int32_t ylds_pc = 0;         // ... with a cut-producing wave beside each replica's wave
    int32_t no_producer = 0;     // UAVQ_VARIANT_NOPRODUCER
    int32_t generic_chunk = 0;   // UAVQ_VARIANT_GENERIC
    int32_t stop_frozen = 0;     // UAVQ_STOP_FROZEN
    int32_t reduce_at_end = 0;   // UAVQ_REDUCE_AT_END
    int32_t concurrent = 0;      // UAVQ_CONCURRENT_CLASSES (and more than one class is used)
    void *side_stream[uavq::kMaxChunks + 2] = {};   // per class after the first (concurrent mode)
    void *fork_ev = nullptr, *join_ev[uavq::kMaxChunks + 2] = {};
    size_t queue_off = 0;                 // workspace: item counters (persistent mode)
    void *graph_exec = nullptr;           // cached hipGraphExec_t (graph mode)
    uint64_t graph_key = 0;
};

extern "C" void plan_destroy_events(uavq_plan *pl);   // also releases a cached graph

// Kernel launchers (uavq_kernels.hip).
namespace uavq {
// the block-tested chunked sweep for nj = 2, 3, 4 chunks (uavq_sweep_chunk.hip); NULL otherwise
const void *chunk_sweep_kernel(int nj, bool stop);
// ... for nj = 5, 6 (uavq_sweep_chunk_wide.hip); NULL otherwise
const void *chunk_sweep_wide_kernel(int nj, bool stop);
// ... for nj = 7, 8, 9 with 16-bit costs in global memory (uavq_sweep_chunk_big.hip); NULL otherwise
const void *chunk_sweep_big_kernel(int nj, bool stop);
// the 16-bit-cost sweep of classes 7..9 (uavq_sweep_big.hip); NULL otherwise
const void *big_sweep_kernel(int nj, bool stop);
int launch_anneal(const uavq_plan *plan, const KArgs &a, void *stream, int64_t *check_E);
int launch_dense(const uavq_plan *plan, const KArgs &a, hipStream_t_opaque st);
int launch_energy_refresh(const uint32_t *d_states, int64_t n, int64_t *d_E, const uint8_t *d_D, const uint8_t *d_dep,
                          int m, int P, int closed, int64_t c0, hipStream_t_opaque st);
int launch_energy(const uavq_qubo *q, const uint32_t *d_x, int64_t n, int64_t *d_E, void *d_ws,
                  size_t ws_bytes, void *stream);
size_t energy_ws_bytes(const uavq_qubo *q);
}  // namespace uavq
