// The handle of a loaded system (snp_system of snp.h): its derived device
// tables, visited set, per-frontier and per-chunk buffers and launch settings.
// Shared by the runtime (snp_api.hip) and the autotuner (snp_tune.hip); not
// part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <vector>

#include "snp.h"
#include "snp_internal.hpp"

using snp::u64;

namespace snp {
// Records the message snp_last_error() returns on this thread; returns st.
snp_status set_error(snp_status st, const char* fmt, ...);
}  // namespace snp

struct snp_system {
    int m = 0, r = 0, elem_bytes = 4;
    int track = -1;  // column of the output neuron's spike train in a row (-1: none); m counts it
    int mcount = 0;  // neurons (spike-count columns); m is the row width
    bool delays = false;  // some rule has a delay: rows carry (wait, pend) per delayed neuron
    // the host description, kept for snp_run_batch (which packs the handles'
    // systems into one batched launch), and an id no other handle ever gets
    std::vector<int32_t> h_rn, h_ri, h_rj, h_rc, h_rp, h_ss, h_sd;
    int32_t count_type = SNP_COUNT_I32;
    unsigned long long uid = 0;
    long long count_max = INT_MAX;
    snp_options opt{};
    hipStream_t stream = nullptr;
    bool int8_ok = false;

    // device tables
    int* d_nrule_ptr = nullptr;
    int4* d_rules = nullptr;
    int* d_in_ptr = nullptr;
    int* d_in_src = nullptr;
    int* d_in_lane = nullptr;
    int* d_dlink = nullptr;  // with delays: neuron -> wait column, state column -> neuron
    int8_t* d_M8 = nullptr;  // r x m int8 copy of M_Pi when every entry fits (int8 path)
    u64* d_R = nullptr;      // hash weights
    u64* d_hM = nullptr;     // H of every row of M_Pi
    bool int8_ready = false; // d_M8 built and the int8 kernel's limits hold
    bool lane_form = false;  // m <= 64, in-degree <= 16: the one-neuron-per-lane expansion applies
    double pull_work = 0;      // per-child work of a pull (every neuron and in-synapse; path choice)
    double int8_row_work = 0;  // per-child work of the int8 form besides its segment's pull
    snp::DevSystem dsys{};

    // visited set
    u64* d_table = nullptr;
    u64 slots = 0;
    long long tombs = 0;
    uint32_t* d_row_slot = nullptr;
    long long max_rows = 0, max_frontier = 0, chunk_max = 0;
    // launch settings (snp_tuning): children per pass (<= chunk_max, the
    // buffers' size), int8 tiles per workgroup, sparse run length (0: automatic)
    long long chunk_eff = 0;
    int tune_tiles = 0, tune_run = 0;

    // per-frontier and per-chunk buffers
    u64 *d_psi = nullptr, *d_off = nullptr, *d_sc_sums = nullptr, *d_sc_pre = nullptr;
    u64* d_psif = nullptr;  // per parent: all children (every valid spiking vector)
    uint8_t* d_hflag = nullptr;  // per parent: 1 when no rule applies
    void* d_stage = nullptr;
    u64* d_hash = nullptr;
    int* d_cpar = nullptr;
    u64* d_ct = nullptr;
    uint32_t *d_slot = nullptr, *d_flag = nullptr, *d_pos = nullptr, *d_fsums = nullptr, *d_fpre = nullptr;
    uint32_t* d_cand = nullptr;
    // counters: a ring of slots, one per device pass, zeroed once per kRing
    // passes; a walk's start writes the slot its first pass then uses
    static constexpr int kRing = 64;
    snp::DevCounters* d_ring = nullptr;
    snp::DevCounters* d_ctr = nullptr;  // slot of the current pass
    long long pass = 0;
    u64* d_T = nullptr;                 // canonical children of the examined frontier prefix (device)
    u64* d_Tend = nullptr;              // the chunks' end under a child budget (device)
    snp::DevCounters* h_ctr = nullptr;  // the pass read last
    bool start_pending = false;         // the walk start's checks are not read yet
    bool slot_ready = false;            // the current slot was set by the walk start: reuse it

    // caller-driven walk (snp_reset / snp_expand): the handle's own row store
    void* d_store = nullptr;
    bool walk_active = false;
    long long walk_rows = 0;

    double new_ratio = 1.0;  // new / enumerated of the last chunk (chunk sizing)
    double psi_per_parent = 0.0;  // children per examined parent of the last level (0: none yet)

    // stage timing (profile option): event pairs around psi+scan, expand, insert, flags+scan, commit
    static constexpr int kStages = 5;
    hipEvent_t ev[kStages + 1] = {};

    ~snp_system() {
        void* ptrs[] = {d_nrule_ptr, d_rules, d_in_ptr, d_in_src, d_in_lane, d_M8, d_R, d_hM, d_table, d_row_slot, d_psi, d_off,
                        d_sc_sums, d_sc_pre, d_stage, d_hash, d_cpar, d_ct, d_slot, d_flag, d_pos,
                        d_fsums, d_fpre, d_ring, d_store, d_cand, d_hflag, d_T, d_psif, d_Tend, d_dlink};
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
        if (h_ctr) (void)hipHostFree(h_ctr);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};
