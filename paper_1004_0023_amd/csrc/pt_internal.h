// pt_internal.h -- launch interface between the host library and its kernels.
#pragma once

#include "pt_common.h"

namespace ptq {

struct SweepLaunch {
    DevState st;
    uint32_t key0, key1;   // flip-domain Philox key
    int32_t n_sweeps;      // whole-replica tiles: sweeps in this launch
    int32_t tile0;         // first tile of this launch
    int32_t n_tiles;
    int32_t block_threads;
    int32_t lds_bytes;
    // slice-block tiles: sweep t + sweep_off per launch
    int32_t sweep_off;
    int32_t last;          // last launch of a pt_sweep call: accumulate E_cl, C
    // a PT cycle: the tile that completes an instance's sweeps runs its exchange step
    int32_t fuse_exchange;
    uint32_t swap_key0, swap_key1;
    uint32_t t_add;        // sweeps of the call (the exchange advances t by this)
    int32_t lane_words;    // fast tiles: four-slice words per lane (2 needs G4 >= 2)
    int32_t persist;       // slice blocks: one launch of n_sweeps sweeps, all blocks resident
    // resident blocks: poll bound of a neighbour wait (0: the kernel's default) and an
    // amount added to every awaited progress count (0; a test hook sets it so that the
    // waits run into their bound)
    int32_t wait_polls, wait_extra;
    // fused whole-replica launches whose tiles each hold a whole instance: PT cycles run by
    // the launch (0 or 1: one)
    int32_t cycles;
    // resident slice blocks: every replica's ring of blocks lies in one run of the
    // workgroup-to-tile map, so on one XCD, and records and counts pass through its L2 (2:
    // the same, and the launch reports its XCDs as mismatched; a test hook)
    int32_t xcd_local;
    // fast tiles: the latency path (at most one tile per compute unit; tiles whose colour
    // classes do not fit one pass of the workgroup sweep as usual)
    int32_t lat;
};

// Lanes per 32-slot word in the bit-packed sweep (each serves 32 / kBpSweepLanes slots).
constexpr int kBpSweepLanes = 8;

// One colour class (parity p, colour g) of sweep t + sweep_off of every instance in the
// bit-packed encoding: blocks [blk0, blk0 + n_blocks) of the sweep-block list.
struct BpLaunch {
    DevState st;
    uint32_t key0, key1;
    int32_t sweep_off, p, g, blk0, n_blocks;
};

// Bit-packed encoding, octet kernels.  An octet is byte o of the 32-slot words of word group
// w: the 8 replica slots 32 w + 8 o .. 32 w + 8 o + 7.  A work item (kOctRec ints in
// DevState::otiles) is (instance, w, o, first four-slice group g0, groups ng, record
// offset, previous item, next item); the last three serve resident slice blocks: the
// offset of the block's two boundary records (N words each) and the blocks that own groups
// g0 - 1 and g0 + ng of the same octet.
//   tile launches (whole octets, ng = G4): n_sweeps sweeps with the octet resident in LDS,
//     then its E_cl and C;
//   phase launches (octet slice blocks): parity p of sweep t + sweep_off; with last, the
//     blocks add their part of E_cl and C (cleared by launch_oct_clear) at the end;
//   resident launches (octet slice blocks, all resident at once): n_sweeps sweeps, the
//     blocks exchanging boundary groups through records and progress counts, then their
//     parts of E_cl and C.
struct OctLaunch {
    DevState st;
    uint32_t key0, key1;
    int32_t tile0, n_tiles, threads, lds_bytes;
    int32_t n_sweeps, sweep_off, p, last;
    int32_t split;      // slice blocks: two lanes per (site, group), four slots each
    // whole octets: queue = each workgroup takes its octet from the device work queues
    // (DevState::oqitems, counts in oqueue) when it starts; fuse = the octet that completes
    // an instance (DevState::icount against itiles) then runs its exchange step
    int32_t queue, fuse;
    uint32_t swap_key0, swap_key1, t_add;
    int32_t rec_words;  // resident: words of the R0 record region (the R1 region follows)
    // resident: poll bound of a neighbour wait (0: the kernel's default) and an amount added
    // to every awaited progress count (0; a test hook sets it so that the waits give up)
    int32_t wait_polls, wait_extra;
    // resident: every ring of blocks lies in one run of the workgroup-to-block map, so on
    // one XCD, and records and progress counts pass through its L2 (2: the same, and the
    // launch reports its XCDs as mismatched; a test hook)
    int32_t xcd_local;
};
constexpr int kOctRec = 8;  // ints per octet work item
enum OctMode { kOctTile = 0, kOctPhase = 1, kOctResident = 2 };


// Bits of the device error word (DevState::err), read and cleared by the host after a call.
constexpr uint32_t kErrWait = 1u;     // a resident slice block gave up waiting for a neighbour
constexpr uint32_t kErrLdsBase = 2u;  // an octet kernel found its dynamic LDS away from address 0
constexpr uint32_t kErrQueue = 4u;    // a whole-octet workgroup found every work queue empty
constexpr uint32_t kErrPlace = 8u;    // a resident launch's workgroups left round-robin XCDs

// Each returns the hipError_t of the launch itself (asynchronous execution errors
// surface at the next synchronisation).
hipError_t launch_init_spins(const DevState &st, int32_t n_reps, uint32_t key0, uint32_t key1,
                             hipStream_t s);
hipError_t launch_energy(const DevState &st, int32_t rep_first, int32_t n_reps, hipStream_t s);
hipError_t launch_sweep(const SweepLaunch &L, int kind, hipStream_t s);
// Before the slice-block launches of a call: boundary records of the current spins into
// buffer (t mod 2), E_cl and C of the blocked replicas cleared.
hipError_t launch_block_prepare(const SweepLaunch &L, hipStream_t s);
hipError_t launch_exchange(const DevState &st, int32_t n_inst, uint32_t key0, uint32_t key1,
                           uint32_t t_add, hipStream_t s);
// Imaginary-time correlations of every replica added to sumCt at its current rung, with
// `chunks` workgroups per replica.
hipError_t launch_tau_corr(const DevState &st, int32_t n_reps, int32_t chunks, hipStream_t s);
hipError_t launch_advance(const DevState &st, int32_t n_inst, uint32_t t_add, hipStream_t s);
// Bit-packed encoding: initial spins, one colour class of one sweep, and E_cl, C of
// every replica (n_eblk position blocks, n_reps replica slots).
hipError_t launch_bp_init(const DevState &st, int32_t n_eblk, uint32_t key0, uint32_t key1,
                          hipStream_t s);
hipError_t launch_bp_sweep(const BpLaunch &L, hipStream_t s);
hipError_t launch_bp_energy(const DevState &st, int32_t n_eblk, int32_t n_reps, hipStream_t s);
hipError_t launch_oct_tiles(const OctLaunch &L, hipStream_t s);
hipError_t launch_oct_phase(const OctLaunch &L, hipStream_t s);
hipError_t launch_oct_resident(const OctLaunch &L, hipStream_t s);
// E_cl and C of the replicas of octet work items [tile0, tile0 + n_tiles) set to zero (the
// phase launches' last sweep and the resident launch add to them), and their progress
// counts.
hipError_t launch_oct_clear(const OctLaunch &L, hipStream_t s);
// LDS bytes of an octet work item of instance d with ng groups per parity (whole octet:
// ng = G4) in layout mode (OctMode).
int32_t oct_lds_bytes(const InstDesc &d, int32_t ng, int mode);
hipError_t oct_kernels_set_lds(int32_t tile_bytes, int32_t phase_bytes, int32_t resident_bytes);
// Resident octet slice blocks of `threads` threads and `lds_bytes` of LDS that one compute
// unit holds at once.
hipError_t oct_resident_per_cu(int32_t threads, int32_t lds_bytes, int32_t *per_cu);
// LDS bytes the whole-octet kernel adds after the largest octet (the taken list position
// and a flag).
constexpr int32_t kOctQueueLds = 16;
hipError_t launch_threshold_eval(const double *dS, uint32_t *out, int32_t n, hipStream_t s);
hipError_t sweep_kernels_set_lds(int32_t fast_bytes, int32_t generic_bytes, int32_t block_bytes);
// Slice-block workgroups of `threads` threads and `lds_bytes` of LDS that one compute unit
// holds at once in the resident (persistent) block kernel.
hipError_t block_resident_per_cu(int32_t threads, int32_t lds_bytes, int32_t *per_cu);

// Record msg as the calling thread's last error (pt_last_error) and return code.
int report_error(int code, const char *msg);

// LDS bytes a tile of P replicas of instance d needs in its sweep kernel.
int32_t sweep_tile_lds_bytes(const InstDesc &d, int32_t n_adj, int32_t P);
// LDS bytes of a slice-block tile: P replicas, ng four-slice groups per parity.
int32_t block_tile_lds_bytes(const InstDesc &d, int32_t P, int32_t ng);

}  // namespace ptq
