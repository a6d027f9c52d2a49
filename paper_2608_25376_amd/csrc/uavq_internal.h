// Internal structures shared by the host code and the HIP kernels of libuavq.
#pragma once
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/uavq.h"

typedef struct ihipStream_t *hipStream_t_opaque;

namespace uavq {

// Largest number of 64-column chunks a replica row may span in the factored
// kernel (m <= 64 * kMaxChunks).  Classes 1..kByteChunks keep the cost matrix
// as bytes in LDS; the classes above read 16-bit costs from global memory
// (fields past 19x19, and every field with a cost above 255).
constexpr int kMaxChunks = 9;
constexpr int kByteChunks = 6;
constexpr int kMaxM = 64 * kMaxChunks;
constexpr int kWideMaxWaves = 4;   // waves per block of the kernels of classes 4..kMaxChunks

int set_error(int code, const char *fmt, ...);

// Device-side descriptor of one instance inside a plan's workspace.
struct InstDesc {
    int32_t m, P, closed, row_words;
    int32_t state_words, nrep;
    int64_t c0;
    int64_t d_off;      // byte offset of D (m*m, row-major): uint8, or uint16 for classes above kByteChunks
    int64_t ddep_off;   // byte offset of the start-cell costs (m entries, same type)
    int64_t J_off;      // byte offset of the dense J (N*N int16) or -1
    int64_t Jlimb_off;  // byte offset of the J limbs (two Np*Np int8: J & 127, J >> 7) or -1
    int64_t b_off;      // byte offset of b (N int32) or -1
    int64_t rep_base;   // global index of replica 0
    int64_t state_off;  // word offset of replica 0's state
    uint32_t inst_id;
    int32_t chunks;     // ceil(m / 64)
    // this instance's schedule: row s of its acceptance table is table row
    // sched_row + s * sched_step (step 0: a constant temperature, one row)
    int32_t sched_row, sched_step;
    float tl2_a, tl2_b; // T_s ln 2 ~= exp2(tl2_a + tl2_b s): starting guess for acceptance cuts
    int32_t wide;       // a cost exceeds 255 (no byte copy of D for the MFMA energy check)
    int32_t pad_;
};

// One workgroup's share: replicas rep0 .. rep0+nrep-1 of instance inst.
struct WorkItem {
    int32_t inst, rep0, nrep, pad;
};

// Kernel argument block (passed by value).
struct KArgs {
    const uint8_t *ws;          // workspace base
    const InstDesc *desc;
    const WorkItem *items;
    int32_t n_items;
    int32_t item_base;          // first item of this launch
    int32_t *queue;             // persistent mode: item counter of this launch (NULL = one item per block)
    int32_t queue_n;            // items in this launch (persistent mode)
    const uint32_t *thr;        // table rows of thr_stride entries (d = 0..Dmax used), per instance at its sched_row
    int32_t thr_stride;         // multiple of 4
    const int32_t *dcut;        // per table row: least d with thr[row][d] == 0
    int32_t S, Dmax;
    int32_t s_begin, s_end;     // this launch runs sweeps s_begin .. s_end-1 of the S-sweep schedule
    int32_t resume;             // continue from the outputs of a segment that ended at s_begin
    uint32_t seed;
    int32_t n_inst;
    int64_t total_rep;
    // inputs
    const uint32_t *init_states;
    const uint8_t *seeded;
    const int32_t *start_sweep;
    // working / outputs
    uint32_t *states;           // current state (final on exit)
    int64_t *E_init;            // workspace: energy of the initial state
    int64_t *final_E, *best_E;
    int32_t *best_sweep;
    uint32_t *best_states;
    uint64_t *accepts, *draws;
    int64_t *inst_best_E;
    int32_t *inst_best_replica, *inst_best_sweep;
    uint32_t *inst_best_state;
    int64_t *inst_state_off;    // per instance: word offset of its best state in inst_best_state
};

}  // namespace uavq

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
    int32_t ylds_w1 = 0;         // the m <= 64 sweep runs at one wave per SIMD (launch fits the chip)
    int32_t ylds_pc = 0;         // ... with a cut-producing wave beside each replica's wave
    int32_t no_producer = 0;     // UAVQ_VARIANT_NOPRODUCER
    int32_t generic_chunk = 0;   // UAVQ_VARIANT_GENERIC
    int32_t stop_frozen = 0;     // UAVQ_STOP_FROZEN
    int32_t reduce_at_end = 0;   // UAVQ_REDUCE_AT_END
    size_t queue_off = 0;                 // workspace: item counters (persistent mode)
    void *graph_exec = nullptr;           // cached hipGraphExec_t (graph mode)
    uint64_t graph_key = 0;
};

extern "C" void plan_destroy_events(uavq_plan *pl);   // also releases a cached graph

// Kernel launchers (uavq_kernels.hip).
namespace uavq {
// the block-tested chunked sweep for nj = 2, 3 chunks (uavq_sweep_chunk.hip); NULL otherwise
const void *chunk_sweep_kernel(int nj, bool stop);
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
