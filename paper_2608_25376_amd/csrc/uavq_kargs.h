// Kernel-side structures of libuavq: the argument block of the sweep kernels
// and the instance and work-item descriptors they read from the workspace.
#pragma once
#include <cstdint>

#include "../../include/uavq.h"

namespace uavq {

// Largest number of 64-column chunks a replica row may span in the factored
// kernel (m <= 64 * kMaxChunks).  Classes 1..kByteChunks keep the cost matrix
// as bytes in LDS; the classes above read 16-bit costs from global memory
// (fields past 19x19, and every field with a cost above 255).
constexpr int kMaxChunks = 9;
constexpr int kByteChunks = 6;
constexpr int kMaxM = 64 * kMaxChunks;
constexpr int kWideMaxWaves = 4;   // waves per block of the kernels of classes 4..kMaxChunks
constexpr int kSimdsPerChip = 1024;   // MI355X: 256 CUs x 4 SIMDs

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
    int32_t wmax;       // largest travel cost, start cell included
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
    uint64_t *attempts;         // per replica: flips attempted (N per sweep run), optional
    int32_t pw;                 // block-tested sweep: the dynamic LDS holds 1 KB per wave for packed draw words
};

}  // namespace uavq
