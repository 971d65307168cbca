// pt_common.h -- device layout and arithmetic shared by the library's host code and its
// gfx950 kernels: Philox4x32-10, the deterministic exponential, the acceptance threshold,
// and the descriptors that place every instance in the device workspace.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace ptq {

// ------------------------------------------------------------------ Philox4x32-10
// Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11): ten rounds, each two
// 32x32->64 products (multipliers 0xD2511F53, 0xCD9E8D57) whose high halves are xor-ed
// with the other two words and the round key; keys advance by 0x9E3779B9, 0xBB67AE85.
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

constexpr uint32_t kDomainSwap = 0x53574150u;  // 'SWAP'
constexpr uint32_t kDomainInit = 0x494E4954u;  // 'INIT'

struct Words4 {
    uint32_t w[4];
};

// Three-input xor: one v_bitop3_b32 (truth table 0x96) on gfx950.
__host__ __device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
    return a ^ b ^ c;
#endif
}

__host__ __device__ __forceinline__ Words4 philox10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                    uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)kPhiloxM0 * c0;
        const uint64_t pb = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = xor3((uint32_t)(pb >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(pa >> 32), c3, k1);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    Words4 o;
    o.w[0] = c0;
    o.w[1] = c1;
    o.w[2] = c2;
    o.w[3] = c3;
    return o;
}

// ------------------------------------------------------------------ exp and thresholds
// exp(x), x <= 0, from IEEE multiply/add/floor/ldexp only (every operation separately
// rounded; contraction is off for this file), so host and device agree bitwise:
// Cody-Waite reduction by ln 2 split as c1 (32 significant bits, so n*c1 is exact) plus
// c2, then the degree-12 Taylor polynomial of exp(r) in Horner form, scaled by 2^n.
// For x < -32 the value cannot affect any 32-bit threshold and 0 is returned.
__host__ __device__ __forceinline__ double exp_det(double x)
{
    const double kLog2e = 0x1.71547652b82fep+0;
    const double kLn2Hi = 0x1.62e42feep-1;           // 2977044471 / 2^32
    const double kLn2Lo = 0x1.a39ef35793c76p-33;     // ln 2 - kLn2Hi, rounded
    if (!(x >= -32.0)) return 0.0;
    const double n = floor(x * kLog2e + 0.5);
    const double r = (x - n * kLn2Hi) - n * kLn2Lo;
    // 1/j! for j = 12 down to 0, each the double nearest the exact rational
    double p = 0x1.1eed8eff8d898p-29;
    p = p * r + 0x1.ae64567f544e4p-26;
    p = p * r + 0x1.27e4fb7789f5cp-22;
    p = p * r + 0x1.71de3a556c734p-19;
    p = p * r + 0x1.a01a01a01a01ap-16;
    p = p * r + 0x1.a01a01a01a01ap-13;
    p = p * r + 0x1.6c16c16c16c17p-10;
    p = p * r + 0x1.1111111111111p-7;
    p = p * r + 0x1.5555555555555p-5;
    p = p * r + 0x1.5555555555555p-3;
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return ldexp(p, (int)n);
}

// Metropolis min(1, exp(-dS)) as a 32-bit threshold: accept iff u <= thr.
__host__ __device__ __forceinline__ uint32_t threshold(double dS)
{
    if (dS <= 0.0) return 0xFFFFFFFFu;
    double v = floor(ldexp(exp_det(-dS), 32));
    if (v > 4294967295.0) v = 4294967295.0;
    if (v < 1.0) v = 1.0;
    return (uint32_t)v - 1u;
}

// ------------------------------------------------------------------ device layout

// Table of thresholds of one rung, indexed [x][f + F][tau] with x = (s + 1)/2, f the local
// field, tau = t'/2 + 1 in {0, 1, 2}: size 2 * (2F + 1) * 3 words.
__host__ __device__ __forceinline__ int table_words(int F) { return 2 * (2 * F + 1) * 3; }

// Spin layout of one replica (device memory and LDS): bytes x = (s + 1)/2 in {0, 1},
// ordered [p][i][m] with slice k = 2m + p (parity-split, slice-minor): the Mh = M/2
// slices of one parity of one site are contiguous, so a 32-bit word holds the four
// same-parity slices that one Philox call serves.  M == 1: one parity, Mh = 1.
// Imaginary-time correlation lags per rung (PT_TAU_LAGS of the C ABI).
constexpr int kTauLags = 8;

struct InstDesc {
    int32_t N, M, R;
    int32_t Mh;        // slices per parity
    int32_t G4;        // ceil(Mh / 4): Philox calls per (site, parity)
    int32_t parities;  // 2 if M >= 2 else 1
    int32_t F;         // max |local field|
    int32_t D;         // max degree (fast-path neighbour rows are padded to D)
    int32_t n_colors;
    int32_t fast;      // 1: byte-SWAR kernels apply to this instance
    int32_t ent_sh;    // fast-path entries hold (j << ent_sh); lg(Mh) when j*Mh fits 16 bits
    int32_t rep_base;  // first global replica / rung index
    int32_t pair_base; // first global pair index (R - 1 pairs)
    int32_t adj_base;  // first generic neighbour entry
    int32_t off_base;  // first neighbour offset (N + 1 per instance)
    int32_t site_base; // first per-site entry (fields, biases, class lists)
    int32_t ent_base;  // first fast-path neighbour entry (N * D per instance)
    int32_t cls_base;  // first class offset (n_colors + 1 per instance)
    int32_t tbl_base;  // first threshold word (R tables)
    int32_t tbl_words; // words per rung table
    int32_t rep_bytes; // bytes per replica in device memory (N * M rounded up to 16)
    int64_t spin_base; // first spin byte of the instance
    // bit-packed encoding: word groups ceil(R / 32), words per (group, parity, site) row
    // (4 * G4), and the instance's first word group in the batch
    int32_t bp_W, bp_row, bp_wg_base;
    int32_t ent_mode;  // EntMode of the fast-path neighbour entries
    // bit-packed encoding, octet kernels (every |J| = 1, |h| <= 1, one degree D, fast
    // shape): 1 if they run this instance; its first 16-bit octet neighbour entry and its
    // first octet table word (kOctTableWords per rung)
    int32_t oct, oent_base, otbl_base, opad;
};

// Octet tables: per rung, the acceptance threshold indexed n + 16 sigma + 64 hz, where n is
// the number of a site's inputs (its D couplings and, when h != 0, its field) that agree with
// its spin, sigma the number of agreeing time neighbours and hz = [h != 0]; then
// a = s f = 2 n - D - hz.
constexpr int kOctTableWords = 128;

// How the byte-SWAR kernels form a site's local field from its neighbour entries.
//   kEntPerm   32-bit entries (j * Mh) << 16 | w1 << 8 | w0: a v_perm maps each neighbour
//              spin byte x to its weight w_x (any |J|, padded rows)
//   kEntXad16  16-bit entries (j * Mh) | [J < 0] << 15, every |J| = 1 and every site of
//              full degree D: a neighbour adds its spin byte x, or 1 - x when J < 0, as
//              (x ^ m) + acc with m = 0x01010101 [J < 0].  For instances whose one-replica
//              tiles would not otherwise fit two to a compute unit (it costs two operations
//              more per neighbour and lane than kEntPerm, whose v_perm lookups the compiler
//              sums with three-input adds)
enum EntMode { kEntPerm = 0, kEntXad16 = 2 };

// 32-bit words of the fast-path neighbour entries of an instance with N sites and row
// length D (two 16-bit entries per word under kEntXad16).
__host__ __device__ __forceinline__ int64_t ent_words(int64_t N, int32_t D, int32_t mode)
{
    return mode == kEntXad16 ? (N * D + 1) / 2 : N * D;
}

enum TileKind { kTileGeneric = 0, kTileFast = 1, kTileBlock = 2 };

struct Tile {
    int32_t inst;  // instance
    int32_t c0;    // first replica slot
    int32_t P;     // replicas in the tile (a power of two on the fast paths)
    int32_t kind;  // TileKind: which sweep kernel runs it
    int32_t g0;    // slice-block tiles: first four-slice group of the block
    int32_t ng;    // slice-block tiles: groups in the block (a power of two)
    int32_t hb;    // slice-block tiles: word offset of the block's boundary record
    int32_t prev;  // slice-block tiles: tile index of the block before / after it in the
    int32_t next;  //   same replica (cyclically; itself when one block covers the replica)
};

struct Counters {
    uint64_t t;      // sweeps done
    uint64_t e;      // exchange steps done
    uint64_t n_acc;  // accumulated samples
    uint64_t pad;
};

// Pointers into the workspace (all device addresses).
struct DevState {
    // immutable after init
    const InstDesc *inst;
    const int32_t *adj;       // generic neighbour entry: (j & 0xFFFF) | (J << 16)
    const int32_t *adj_off;   // per site: first entry (N + 1 per instance)
    const int16_t *hfield;    // per site
    const uint32_t *ent;      // fast neighbour entries (EntMode): (j << ent_sh) << 16 | w1 << 8 | w0,
                              // or 16-bit (j << ent_sh) | [J < 0] << 15 two to a word
    const uint32_t *bias;     // fast per-site bias (h - sum|J| + F) in every byte
    const uint16_t *csite;    // sites of each colour, colour by colour
    const int32_t *cls_off;   // per colour: first class site (n_colors + 1 per instance)
    const uint32_t *tbl;      // threshold tables
    const double *db;         // per pair: b_r - b_{r+1}
    const double *dK;         // per pair: K_r - K_{r+1}
    const Tile *tiles;
    const int32_t *rep_inst;  // global replica -> instance
    // slice-block boundary records, two buffers of halo_words words: for each block, its
    // first group of parity 0 and of parity 1 and its last group of parity 1 (N words each)
    uint32_t *halo;
    int64_t halo_words;
    // per instance: tiles of one sweep call, and tiles that finished the current call
    const int32_t *itiles;
    uint32_t *icount;
    // resident slice blocks: sweeps each block has published in the current call (one per
    // block tile), and a sticky error word (nonzero: a wait gave up)
    int32_t *prog;
    uint32_t *err;
    // bit-packed encoding: sweep blocks (instance, first item) of every colour, position
    // blocks (instance, word group, chunk, chunks) for init and energies, per word group
    // its first position block and their count, and the energy partial sums (per position
    // block, 32 slots x (2 E_cl, C))
    const int32_t *bp_sblk;
    const int32_t *bp_eblk;
    const int32_t *bp_wg;
    int64_t *bp_part;
    // bit-packed encoding, octet kernels: 16-bit neighbour entries (j | [J < 0] << 15, D per
    // site), per-site field codes (bit 0: h < 0, bit 1: h != 0), per-rung tables, the work
    // list of the octet launches (kOctRec ints per item), and for resident slice blocks
    // their boundary records (an R0 region, then an R1 region) and progress counts (two per
    // work item: parity 0, parity 1)
    const uint16_t *oent;
    const uint8_t *ohinfo;
    const uint32_t *otbl;
    const int32_t *otiles;
    uint32_t *orec;
    int32_t *oprog;
    // whole octets from the device work queues: positions taken from each XCD's queue
    // (8 counts) and workgroups that have taken theirs (the last resets all nine for the
    // next launch); oqitems: the queues' 9 offsets, then their list positions
    int32_t *oqueue;
    const int32_t *oqitems;
    // resident slice blocks (octets, bytes): the XCD offsets their workgroups found
    uint32_t *xseen;
    // mutable state
    uint8_t *spins;
    int64_t *E;       // per replica slot
    int64_t *C;
    int32_t *rung_of;
    int32_t *label;
    uint64_t *rt;
    int32_t *replica_of;  // per rung
    int64_t *sumE, *sumC, *sumE2, *sumC2;
    int64_t *sumCt;       // per rung x kTauLags: imaginary-time correlations
    uint64_t *nup, *ndown;  // per rung: exchange steps with an UP / DOWN replica there
    uint64_t *acc, *att;  // per pair
    Counters *ctr;        // per instance
};

}  // namespace ptq
