// pt_host.hip -- host side of the C ABI declared in include/ptqmc.h.
//
// One context holds a batch of instances.  All state lives in one device workspace:
// an immutable region (instance descriptors, neighbour lists, colour blocks, threshold
// tables, pair constants, tiles) followed by the mutable state region (spins, energies,
// permutation, labels, swap statistics, accumulators, counters) that pt_save/pt_load
// copy as one block.  Every sweep and exchange runs on the device; the host only
// launches, so a PT cycle never crosses PCIe (unlike the per-cycle copies of the
// paper's Figure 6).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <utility>
#include <string>
#include <vector>

#include "../../include/ptqmc.h"
#include "pt_internal.h"

using namespace ptq;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(PT_EHIP, std::string(what) + ": " + hipGetErrorString(e) + " (hip error " +
                             std::to_string((int)e) + ")");
}

#define HIP_TRY(call)                                     \
    do {                                                  \
        hipError_t e__ = (call);                          \
        if (e__ != hipSuccess) return hip_fail(e__, #call); \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

constexpr uint32_t kMagic = 0x51505450u;  // checkpoint tag
constexpr uint32_t kVersion = 3;
constexpr int kMaxField = 1023;

// Host copy of everything that is uploaded once, plus the layout of the workspace.
struct Plan {
    std::vector<InstDesc> desc;
    std::vector<int32_t> adj, adj_off, cls_off, rep_inst;
    std::vector<int16_t> hfield;
    std::vector<uint16_t> csite;
    std::vector<uint32_t> ent, bias, tbl;
    std::vector<double> db, dK;
    std::vector<int32_t> n_adj;  // per instance
    int64_t total_reps = 0, total_pairs = 0, spin_bytes = 0;
    int64_t max_tiles = 0;  // tile slots: one per (replica, four-slice group) at most
    // bit-packed encoding: sweep blocks (n, item0) colour by colour with each colour's
    // (first block, blocks); position blocks (n, w, chunk, chunks); per word group
    // (first position block, blocks)
    int32_t encoding = PT_INT8;
    std::vector<int32_t> bp_sblk, bp_eblk, bp_wg;
    std::vector<std::pair<int32_t, int32_t>> bp_colour;
    int32_t bp_n_eblk = 0;
    // bit-packed encoding, octet kernels: 16-bit entries, field codes, per-rung tables and the
    // work list (tiles first, then slice blocks; kOctRec ints each)
    std::vector<uint16_t> oent;
    std::vector<uint8_t> ohinfo;
    std::vector<uint32_t> otbl;
    std::vector<int32_t> otiles;
    int32_t n_otile = 0, n_oblock = 0;         // whole-octet tiles, octet slice blocks
    // the whole-octet work queues: offsets of the 8 per-XCD queues (9 ints), then each
    // queue's list positions, largest octet first
    std::vector<int32_t> oqitems;
    // resident octet slice blocks: every ring of blocks in one run of the launch's map
    bool oblock_xcd = false;
    int32_t otile_lds = 0, oblock_lds = 0;     // their largest LDS need
    int32_t oblock_threads = 256;
    bool oblock_split = false;                 // slice blocks: two lanes per (site, group)
    int32_t oblock_res_lds = 0;                // slice blocks, resident layout
    int64_t orec_words = 0;                    // words of each boundary-record region
    bool bp_generic = false;                   // some packed instance runs the per-class kernel
    int64_t halo_words = 0; // one buffer of slice-block boundary records, at most
    uint64_t flips_per_sweep = 0;
    // byte offsets in the workspace
    size_t o_inst, o_adj, o_off, o_h, o_ent, o_bias, o_csite, o_cls, o_tbl, o_db, o_dK, o_tiles,
        o_repinst, o_halo, o_itiles, o_icount, o_prog, o_err, o_bp_sblk, o_bp_eblk, o_bp_wg,
        o_bp_part, o_oent, o_ohinfo, o_otbl, o_otiles, o_orec, o_oprog, o_oqueue, o_oqitems,
        o_xseen;
    size_t o_state;  // start of the mutable region
    size_t o_spins, o_E, o_C, o_rung, o_label, o_rt, o_repof, o_sumE, o_sumC, o_sumE2,
        o_sumC2, o_nup, o_ndown, o_acc, o_att, o_ctr, o_sumCt;
    size_t state_bytes, total_bytes;
};

int validate(const pt_instance &in, int idx)
{
    auto bad = [&](const std::string &m) {
        return fail(PT_EINVAL, "instance " + std::to_string(idx) + ": " + m);
    };
    if (in.N < 1 || in.N > 65535) return bad("N must be in [1, 65535]");
    if (in.M < 1 || (in.M > 1 && (in.M % 2))) return bad("M must be 1 or even");
    if (in.M > 4096) return bad("M must be <= 4096");
    if (in.R < 2) return bad("R must be >= 2");
    if (in.n_edges < 0) return bad("n_edges < 0");
    if (in.n_colors < 1 || in.n_colors > 256) return bad("n_colors must be in [1, 256]");
    if (!in.h || !in.color || !in.rung_b || !in.rung_K) return bad("null array");
    if (in.n_edges > 0 && (!in.edge_i || !in.edge_j || !in.edge_J)) return bad("null edge array");
    for (int i = 0; i < in.N; ++i)
        if (in.color[i] >= in.n_colors) return bad("colour out of range");
    std::vector<int64_t> fsum(in.N);
    for (int i = 0; i < in.N; ++i) fsum[i] = std::abs((int)in.h[i]);
    std::vector<std::pair<int, int>> seen;
    seen.reserve(in.n_edges);
    for (int e = 0; e < in.n_edges; ++e) {
        const int i = in.edge_i[e], j = in.edge_j[e];
        if (i < 0 || j >= in.N || i >= j) return bad("edge " + std::to_string(e) + " needs 0 <= i < j < N");
        if (in.color[i] == in.color[j]) return bad("improper colouring at edge " + std::to_string(e));
        fsum[i] += std::abs((int)in.edge_J[e]);
        fsum[j] += std::abs((int)in.edge_J[e]);
        seen.emplace_back(i, j);
    }
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end()) return bad("duplicate edge");
    for (int i = 0; i < in.N; ++i)
        if (fsum[i] > kMaxField) return bad("local field bound exceeds 1023");
    for (int r = 0; r < in.R; ++r) {
        if (!std::isfinite(in.rung_b[r])) return bad("non-finite b");
        if (in.M >= 2 && (!std::isfinite(in.rung_K[r]) || !(in.rung_K[r] > 0.0)))
            return bad("K must be finite and > 0 when M >= 2");
    }
    return PT_OK;
}

// Threshold table of one rung: [x][f + F][tau], x = (s + 1)/2, tau = t'/2 + 1.
void build_table(uint32_t *out, int F, int M, double b, double K)
{
    const double Keff = (M >= 2) ? K : 0.0;
    for (int x = 0; x < 2; ++x) {
        const int s = x ? 1 : -1;
        for (int f = -F; f <= F; ++f) {
            for (int tau = 0; tau < 3; ++tau) {
                const int tp = 2 * (tau - 1);
                const int64_t dE = -2 * (int64_t)s * f;
                const int64_t dC = -2 * (int64_t)s * tp;
                const double dS = b * (double)dE - Keff * (double)dC;
                out[(x * (2 * F + 1) + (f + F)) * 3 + tau] = threshold(dS);
            }
        }
    }
}

// Octet table of one rung (kOctTableWords words): entry n + 16 sigma + 64 hz holds thr(dS) for
// a = s f = 2 n - D - hz agreeing-minus-disagreeing inputs and sigma agreeing time
// neighbours, i.e. dE = -2 a and dC = -4 (sigma - 1): the entry build_table holds for x = 1,
// f = a, tau = sigma, from the same operations.  Unused entries stay 0.
void build_oct_table(uint32_t *out, int D, double b, double K)
{
    for (int k = 0; k < kOctTableWords; ++k) out[k] = 0u;
    for (int hz = 0; hz < 2; ++hz)
        for (int sigma = 0; sigma < 3; ++sigma)
            for (int n = 0; n <= D + hz; ++n) {
                const int a = 2 * n - D - hz;
                const int64_t dE = -2 * (int64_t)a;
                const int64_t dC = -2 * (int64_t)(2 * (sigma - 1));
                const double dS = b * (double)dE - K * (double)dC;
                out[n + 16 * sigma + 64 * hz] = threshold(dS);
            }
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// LDS of one gfx950 workgroup; instances whose whole replicas exceed it run as slice blocks
constexpr int32_t kLdsPerWorkgroup = 163840;

// Bit-packed encoding: position blocks per word group (at most this many; each block
// passes over 64 positions at a time).
constexpr int32_t kBpMaxChunks = 1024;
constexpr int32_t kBpThreadsHost = 256;

// Whether every ring of slice blocks ([first, end) positions, consecutive) lies within one
// run of the launches' map from workgroups to tiles (runs of nb / 8 positions, each on one
// XCD; the tail past 8 runs keeps its own indices and XCDs).
bool rings_in_runs(const std::vector<std::pair<int, int>> &rings, int nb)
{
    const int q = nb / 8;
    if (q == 0 || nb % 8 != 0) return false;
    for (const auto &r : rings)
        if (r.first / q != (r.second - 1) / q) return false;
    return true;
}

int make_plan(const pt_instance *inst, int32_t n_inst, uint32_t flags, int32_t encoding, Plan &P)
{
    if (!inst || n_inst < 1) return fail(PT_EINVAL, "need at least one instance");
    if (encoding != PT_INT8 && encoding != PT_BITPACK32) return fail(PT_EINVAL, "unknown encoding");
    P = Plan();
    P.encoding = encoding;
    const bool bp = encoding == PT_BITPACK32;
    int64_t rep = 0, pair = 0, adjb = 0, offb = 0, siteb = 0, entb = 0, clsb = 0, tblb = 0,
            spinb = 0, wgb = 0;
    for (int n = 0; n < n_inst; ++n) {
        int rc = validate(inst[n], n);
        if (rc) return rc;
        const pt_instance &in = inst[n];
        InstDesc d{};
        d.N = in.N;
        d.M = in.M;
        d.R = in.R;
        d.Mh = (in.M >= 2) ? in.M / 2 : 1;
        d.G4 = (d.Mh + 3) / 4;
        d.parities = (in.M >= 2) ? 2 : 1;
        d.n_colors = in.n_colors;
        // generic neighbour lists: (j & 0xFFFF) | (J << 16)
        std::vector<int32_t> deg(in.N + 1, 0);
        for (int e = 0; e < in.n_edges; ++e) {
            deg[in.edge_i[e] + 1]++;
            deg[in.edge_j[e] + 1]++;
        }
        int D = 0;
        for (int i = 0; i < in.N; ++i) D = std::max(D, deg[i + 1]);
        for (int i = 0; i < in.N; ++i) deg[i + 1] += deg[i];
        std::vector<int32_t> fill(in.N, 0), entries(2 * (size_t)in.n_edges);
        for (int e = 0; e < in.n_edges; ++e) {
            const int i = in.edge_i[e], j = in.edge_j[e];
            const int32_t J = in.edge_J[e];
            entries[deg[i] + fill[i]++] = (j & 0xFFFF) | (int32_t)((uint32_t)J << 16);
            entries[deg[j] + fill[j]++] = (i & 0xFFFF) | (int32_t)((uint32_t)J << 16);
        }
        int F = 0;
        std::vector<int> sumabs(in.N, 0);
        for (int i = 0; i < in.N; ++i) {
            for (int e = deg[i]; e < deg[i + 1]; ++e) sumabs[i] += std::abs(entries[e] >> 16);
            F = std::max(F, sumabs[i] + std::abs((int)in.h[i]));
        }
        d.F = F;
        d.D = std::max(D, 1);
        d.fast = (in.M >= 8 && in.M % 8 == 0 && is_pow2(in.M / 8) && F <= 20) ? 1 : 0;
        // whole-replica tiles address a neighbour row as j*Mh taken straight from the
        // entry; when that exceeds 16 bits the entry holds j and only slice blocks run
        int lgMh = 0;
        while ((1 << lgMh) < d.Mh) ++lgMh;
        d.ent_sh = ((int64_t)(in.N - 1) * d.Mh <= 65535) ? lgMh : 0;
        d.tbl_words = table_words(F);
        d.rep_bytes = (int32_t)align_up((size_t)in.N * in.M, 16);
        d.rep_base = (int32_t)rep;
        d.pair_base = (int32_t)pair;
        d.adj_base = (int32_t)adjb;
        d.off_base = (int32_t)offb;
        d.site_base = (int32_t)siteb;
        d.ent_base = (int32_t)entb;
        d.cls_base = (int32_t)clsb;
        d.tbl_base = (int32_t)tblb;
        d.spin_base = spinb;
        if (bp) {
            d.bp_W = (in.R + 31) / 32;
            d.bp_row = 4 * d.G4;
            d.bp_wg_base = (int32_t)wgb;
        }
        // sites of each colour, colour by colour
        std::vector<int32_t> cls(in.n_colors + 1, 0);
        for (int i = 0; i < in.N; ++i) cls[in.color[i] + 1]++;
        for (int g = 0; g < in.n_colors; ++g) cls[g + 1] += cls[g];
        std::vector<int32_t> cfill(in.n_colors, 0);
        std::vector<uint16_t> sites(in.N);
        for (int i = 0; i < in.N; ++i) sites[cls[in.color[i]] + cfill[in.color[i]]++] = (uint16_t)i;
        // fast-path rows: D entries per site, (j << ent_sh) << 16 | w1 << 8 | w0 with w0 / w1 the
        // contribution |J| [J < 0] / |J| [J > 0] of a neighbour whose spin byte is 0 / 1;
        // padding entries point at the site itself with weight 0.  When every |J| = 1, every
        // site has degree D and a one-replica tile would take more than half a compute
        // unit's LDS, the entries shrink to 16 bits (kEntXad16: j * Mh fits 15 bits), so
        // that two such tiles fit one unit.
        d.ent_mode = kEntPerm;
        if (d.fast) {
            bool unit = true, regular = true;
            for (int e = 0; e < in.n_edges; ++e) unit = unit && std::abs((int)in.edge_J[e]) == 1;
            for (int i = 0; i < in.N; ++i) regular = regular && deg[i + 1] - deg[i] == d.D;
            int lg = 0;
            while ((1 << lg) < d.Mh) ++lg;
            if (unit && regular && in.n_edges > 0 && d.ent_sh == lg &&
                (int64_t)(in.N - 1) * d.Mh <= 32767 &&
                d.D >= 4 && d.G4 >= 2 &&
                !(flags & (PT_FLAG_SLICE_BLOCKS | PT_FLAG_FOUR_SLICE_LANES)) &&
                sweep_tile_lds_bytes(d, 2 * in.n_edges, 1) > kLdsPerWorkgroup / 2) {
                InstDesc d16 = d;
                d16.ent_mode = kEntXad16;
                if (sweep_tile_lds_bytes(d16, 2 * in.n_edges, 1) <= kLdsPerWorkgroup / 2)
                    d.ent_mode = kEntXad16;
            }
        }
        if (d.fast) {
            std::vector<uint32_t> row;
            for (int i = 0; i < in.N; ++i) {
                int e = deg[i];
                for (int k = 0; k < d.D; ++k, ++e) {
                    uint32_t word = ((uint32_t)i << d.ent_sh) << 16;
                    if (e < deg[i + 1]) {
                        const int j = entries[e] & 0xFFFF;
                        const int J = entries[e] >> 16;
                        const uint32_t w0 = (J < 0) ? (uint32_t)(-J) : 0u;
                        const uint32_t w1 = (J > 0) ? (uint32_t)J : 0u;
                        word = (d.ent_mode == kEntXad16)
                                   ? (((uint32_t)j << d.ent_sh) | (J < 0 ? 0x8000u : 0u))
                                   : ((((uint32_t)j << d.ent_sh) << 16) | (w1 << 8) | w0);
                    }
                    row.push_back(word);
                }
                const uint32_t b = (uint32_t)(in.h[i] - sumabs[i] + F) & 0xFFu;
                P.bias.push_back(b * 0x01010101u);
            }
            if (d.ent_mode == kEntXad16) {
                for (size_t k = 0; k < row.size(); k += 2)
                    P.ent.push_back(row[k] | (k + 1 < row.size() ? row[k + 1] << 16 : 0u));
            } else {
                P.ent.insert(P.ent.end(), row.begin(), row.end());
            }
        } else {
            for (int i = 0; i < in.N; ++i) P.bias.push_back(0);
        }
        // bit-packed encoding: the octet kernels take +-1 couplings, |h| <= 1 and one degree
        // D <= 8 on the fast shapes (M a power-of-two multiple of 8)
        d.oct = 0;
        if (bp && d.fast && in.n_edges > 0 && in.N <= 32767) {
            bool ok = D <= 8;
            for (int e = 0; ok && e < in.n_edges; ++e) ok = std::abs((int)in.edge_J[e]) == 1;
            for (int i = 0; ok && i < in.N; ++i)
                ok = std::abs((int)in.h[i]) <= 1 && deg[i + 1] - deg[i] == D;
            d.oct = ok ? 1 : 0;
        }
        if (d.oct) {
            // entries and field codes padded to 16 bytes per instance (the kernels copy them
            // in 16-byte pieces)
            d.oent_base = (int32_t)P.oent.size();
            for (int i = 0; i < in.N; ++i)
                for (int e = deg[i]; e < deg[i + 1]; ++e) {
                    const int j = entries[e] & 0xFFFF;
                    const int J = entries[e] >> 16;
                    P.oent.push_back((uint16_t)(j | (J < 0 ? 0x8000 : 0)));
                }
            P.oent.resize(align_up(P.oent.size(), 8), 0);
            d.opad = (int32_t)P.ohinfo.size();
            for (int i = 0; i < in.N; ++i)
                P.ohinfo.push_back((uint8_t)((in.h[i] < 0 ? 1 : 0) | (in.h[i] != 0 ? 2 : 0)));
            P.ohinfo.resize(align_up(P.ohinfo.size(), 16), 0);
            d.otbl_base = (int32_t)P.otbl.size();
            P.otbl.resize(P.otbl.size() + (size_t)in.R * kOctTableWords);
            for (int r = 0; r < in.R; ++r)
                build_oct_table(P.otbl.data() + d.otbl_base + (size_t)r * kOctTableWords, D,
                                in.rung_b[r], in.rung_K[r]);
        }
        P.desc.push_back(d);
        P.adj.insert(P.adj.end(), entries.begin(), entries.end());
        P.adj_off.insert(P.adj_off.end(), deg.begin(), deg.end());
        for (int i = 0; i < in.N; ++i) P.hfield.push_back(in.h[i]);
        P.csite.insert(P.csite.end(), sites.begin(), sites.end());
        P.cls_off.insert(P.cls_off.end(), cls.begin(), cls.end());
        const size_t t0 = P.tbl.size();
        P.tbl.resize(t0 + (size_t)in.R * d.tbl_words);
        for (int r = 0; r < in.R; ++r)
            build_table(P.tbl.data() + t0 + (size_t)r * d.tbl_words, F, in.M, in.rung_b[r],
                        in.rung_K[r]);
        for (int r = 0; r + 1 < in.R; ++r) {
            P.db.push_back(in.rung_b[r] - in.rung_b[r + 1]);
            P.dK.push_back(in.M >= 2 ? in.rung_K[r] - in.rung_K[r + 1] : 0.0);
        }
        for (int c = 0; c < in.R; ++c) P.rep_inst.push_back(n);
        P.n_adj.push_back(2 * in.n_edges);
        // byte-encoding tiles and slice-block records (the bit-packed kernels use neither)
        if (P.encoding == PT_INT8) P.max_tiles += (int64_t)in.R * std::max(1, d.G4);
        if (d.fast && P.encoding == PT_INT8) {
            // boundary records for slice blocks: three N-word rows per block, at most one
            // block per four-slice group, for every instance that may run as blocks
            const int lgMh_n = 31 - __builtin_clz((unsigned)d.Mh);
            const bool may_block = d.ent_sh != lgMh_n || (flags & PT_FLAG_SLICE_BLOCKS) ||
                                   sweep_tile_lds_bytes(d, 2 * in.n_edges, 1) > kLdsPerWorkgroup;
            if (may_block) P.halo_words += 3ll * in.N * in.R * std::max(1, d.G4);
        }
        P.flips_per_sweep += (uint64_t)in.R * in.N * in.M;
        rep += in.R;
        pair += in.R - 1;
        adjb += 2 * (int64_t)in.n_edges;
        offb += in.N + 1;
        siteb += in.N;
        entb += d.fast ? ent_words(in.N, d.D, d.ent_mode) : 0;
        clsb += in.n_colors + 1;
        tblb += (int64_t)in.R * d.tbl_words;
        spinb += bp ? (int64_t)d.bp_W * d.parities * in.N * d.bp_row * 4
                    : (int64_t)in.R * d.rep_bytes;
        wgb += d.bp_W;
        if (rep > (1 << 30) || tblb > (1ll << 31) || adjb > (1ll << 31) || entb > (1ll << 31))
            return fail(PT_EINVAL, "batch too large");
    }
    P.total_reps = rep;
    P.total_pairs = pair;
    P.spin_bytes = spinb;
    if (bp) {
        // sweep blocks: colour g of every instance that has it, 256 items per block
        int max_colors = 0;
        for (const auto &d : P.desc) max_colors = std::max(max_colors, d.n_colors);
        for (int g = 0; g < max_colors; ++g) {
            const int32_t first = (int32_t)(P.bp_sblk.size() / 2);
            for (int n = 0; n < n_inst; ++n) {
                const InstDesc &d = P.desc[n];
                if (g >= d.n_colors || d.oct) continue;
                const int64_t sg = P.cls_off[d.cls_base + g + 1] - P.cls_off[d.cls_base + g];
                const int64_t items = (int64_t)d.bp_W * sg * d.G4 * kBpSweepLanes;
                for (int64_t it = 0; it < items; it += kBpThreadsHost) {
                    P.bp_sblk.push_back(n);
                    P.bp_sblk.push_back((int32_t)it);
                }
                if (items > 0x7fffffff) return fail(PT_EINVAL, "batch too large");
            }
            P.bp_colour.emplace_back(first, (int32_t)(P.bp_sblk.size() / 2) - first);
        }
        // position blocks of every word group
        for (int n = 0; n < n_inst; ++n) {
            const InstDesc &d = P.desc[n];
            const int64_t Q = (int64_t)d.parities * d.N * d.G4;
            const int32_t chunks = (int32_t)std::min<int64_t>(kBpMaxChunks, std::max<int64_t>(1, (Q + 63) / 64));
            for (int w = 0; w < d.bp_W; ++w) {
                P.bp_wg.push_back((int32_t)(P.bp_eblk.size() / 4));
                P.bp_wg.push_back(chunks);
                for (int k = 0; k < chunks; ++k) {
                    P.bp_eblk.push_back(n);
                    P.bp_eblk.push_back(w);
                    P.bp_eblk.push_back(k);
                    P.bp_eblk.push_back(chunks);
                }
            }
        }
        P.bp_n_eblk = (int32_t)(P.bp_eblk.size() / 4);
        // octet work: whole octets where one takes at most half a compute unit's LDS
        // (largest first), else slice blocks of ng groups, ng about 512 colour-class items
        // per launch and class
        std::vector<std::array<int32_t, kOctRec>> tiles, blocks;
        for (int n = 0; n < n_inst; ++n) {
            const InstDesc &d = P.desc[n];
            if (!d.oct) {
                P.bp_generic = true;
                continue;
            }
            const bool whole = oct_lds_bytes(d, d.G4, kOctTile) <= kLdsPerWorkgroup / 2;
            int ng = d.G4;
            if (!whole) {
                ng = 1;
                while (2 * ng < d.G4 && (int64_t)2 * ng * d.N <= 512 * (int64_t)d.n_colors &&
                       oct_lds_bytes(d, 2 * ng, kOctResident) <= kLdsPerWorkgroup / 2)
                    ng *= 2;
                if (oct_lds_bytes(d, ng, kOctResident) > kLdsPerWorkgroup)
                    return fail(PT_EINVAL, "instance " + std::to_string(n) +
                                               ": an octet slice block does not fit in LDS");
            }
            for (int w = 0; w < d.bp_W; ++w)
                for (int o = 0; o < 4 && 32 * w + 8 * o < d.R; ++o) {
                    if (whole) {
                        tiles.push_back({n, w, o, 0, d.G4, 0, 0, 0});
                        P.otile_lds = std::max(P.otile_lds, oct_lds_bytes(d, d.G4, kOctTile) + kOctQueueLds);
                    } else {
                        // the octet's ring of blocks (at least two: ng < G4), consecutive in
                        // the list; neighbours and record offsets are filled in below
                        for (int g0 = 0; g0 < d.G4; g0 += ng) blocks.push_back({n, w, o, g0, ng, 0, 0, 0});
                        P.oblock_lds = std::max(P.oblock_lds, oct_lds_bytes(d, ng, kOctPhase));
                        P.oblock_res_lds = std::max(P.oblock_res_lds, oct_lds_bytes(d, ng, kOctResident));
                    }
                }
        }
        // Whole octets go out in one launch, largest first: the small ones, whose sweeps are
        // short chains of dependent colour classes, then run beside the large ones (launched
        // apart, a class of small octets took as long as one octet's chain).
        std::stable_sort(tiles.begin(), tiles.end(), [&](const std::array<int32_t, kOctRec> &a,
                                                         const std::array<int32_t, kOctRec> &b) {
            const InstDesc &da = P.desc[a[0]], &db = P.desc[b[0]];
            return (int64_t)da.N * da.M > (int64_t)db.N * db.M;
        });
        // The octets of one word group read the same 16-byte pieces of device memory and
        // write different bytes of them, so they should share an XCD's L2.  Workgroups go to
        // the XCDs round robin by index: the word groups (still largest first) are dealt to
        // per-XCD queues, each to the least loaded, and workgroup 8 s + x takes entry s of
        // queue x (the last rounds, where queue lengths differ, keep their order only).
        {
            constexpr int kXcds = 8;
            std::vector<std::vector<std::array<int32_t, kOctRec>>> q(kXcds);
            std::vector<int64_t> load(kXcds, 0);
            for (size_t k = 0; k < tiles.size();) {
                size_t e = k + 1;
                while (e < tiles.size() && tiles[e][0] == tiles[k][0] && tiles[e][1] == tiles[k][1]) ++e;
                const InstDesc &d = P.desc[tiles[k][0]];
                const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                for (size_t j = k; j < e; ++j) q[x].push_back(tiles[j]);
                load[x] += (int64_t)d.N * d.M * (int64_t)(e - k);
                k = e;
            }
            std::vector<std::array<int32_t, kOctRec>> dealt;
            dealt.reserve(tiles.size());
            std::vector<std::vector<int32_t>> pos(kXcds);
            for (size_t r = 0; dealt.size() < tiles.size(); ++r)
                for (int x = 0; x < kXcds; ++x)
                    if (r < q[x].size()) {
                        pos[x].push_back((int32_t)dealt.size());
                        dealt.push_back(q[x][r]);
                    }
            tiles.swap(dealt);
            // the same queues for the work-queue launch, whose workgroups take positions
            // from their own XCD's queue
            P.oqitems.assign(kXcds + 1, 0);
            for (int x = 0; x < kXcds; ++x) P.oqitems[x + 1] = P.oqitems[x] + (int32_t)pos[x].size();
            for (int x = 0; x < kXcds; ++x) P.oqitems.insert(P.oqitems.end(), pos[x].begin(), pos[x].end());
        }
        // Resident slice blocks pass boundary records to their ring neighbours twice per
        // sweep.  When every ring lies in one run of the resident launch's workgroup-to-block
        // map (so on one XCD), the records pass through that XCD's L2 instead of
        // device-scope operations.
        const int base = (int)tiles.size();  // blocks follow the tiles in the list
        std::vector<int32_t> prev(blocks.size()), next(blocks.size());
        for (size_t k = 0; k < blocks.size(); ++k) {
            const auto &t = blocks[k];
            const int ring = P.desc[t[0]].G4 / t[4];   // blocks of the octet
            const int first = (int)k - t[3] / t[4];    // its block at group 0
            prev[k] = first + (t[3] / t[4] + ring - 1) % ring;
            next[k] = first + (t[3] / t[4] + 1) % ring;
        }
        {
            std::vector<std::pair<int, int>> rings;  // [first, end) in blocks
            const int nb = (int)blocks.size();
            for (int k = 0; k < nb;) {
                int e = k + 1;
                while (e < nb && blocks[e][0] == blocks[k][0] && blocks[e][1] == blocks[k][1] &&
                       blocks[e][2] == blocks[k][2])
                    ++e;
                rings.emplace_back(k, e);
                k = e;
            }
            P.oblock_xcd = rings_in_runs(rings, nb);
        }
        for (size_t k = 0; k < blocks.size(); ++k) {
            auto &t = blocks[k];
            t[5] = (int32_t)P.orec_words;
            t[6] = base + prev[k];
            t[7] = base + next[k];
            P.orec_words += P.desc[t[0]].N;
        }
        for (const auto &t : tiles) P.otiles.insert(P.otiles.end(), t.begin(), t.end());
        for (const auto &t : blocks) P.otiles.insert(P.otiles.end(), t.begin(), t.end());
        P.n_otile = (int32_t)tiles.size();
        P.n_oblock = (int32_t)blocks.size();
        // slice blocks: one pass over a colour class of the largest block, with two lanes per
        // (site, group) when a class has at most 512 of them
        int most = 1;
        for (const auto &t : blocks) {
            const InstDesc &d = P.desc[t[0]];
            most = std::max<int>(most, (int)std::min<int64_t>(1024, ((int64_t)d.N * t[4] + d.n_colors - 1) / d.n_colors));
        }
        P.oblock_split = most <= 512;
        if (P.oblock_split) most *= 2;
        P.oblock_threads = 64;
        while (P.oblock_threads < most && P.oblock_threads < 1024) P.oblock_threads *= 2;
        if (P.bp_sblk.size() / 2 > 0x7fffffff || P.bp_eblk.size() / 4 > 0x7fffffff ||
            P.orec_words > 0x3fffffff)
            return fail(PT_EINVAL, "batch too large");
    }
    // layout
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + std::max<size_t>(bytes, 1), 256);
        return at;
    };
    P.o_inst = take(P.desc.size() * sizeof(InstDesc));
    P.o_adj = take(P.adj.size() * 4);
    P.o_off = take(P.adj_off.size() * 4);
    P.o_h = take(P.hfield.size() * 2);
    P.o_ent = take(P.ent.size() * 4);
    P.o_bias = take(P.bias.size() * 4);
    P.o_csite = take(P.csite.size() * 2);
    P.o_cls = take(P.cls_off.size() * 4);
    P.o_tbl = take(P.tbl.size() * 4);
    P.o_db = take(P.db.size() * 8);
    P.o_dK = take(P.dK.size() * 8);
    P.o_tiles = take((size_t)P.max_tiles * sizeof(Tile));
    P.o_repinst = take((size_t)rep * 4);
    P.o_halo = take((size_t)P.halo_words * 2 * 4);
    P.o_itiles = take((size_t)n_inst * 4);
    P.o_icount = take((size_t)n_inst * 4);  // zero in the uploaded image
    P.o_prog = take((size_t)P.max_tiles * 4);
    P.o_err = take(4);                       // zero in the uploaded image
    P.o_bp_sblk = take(P.bp_sblk.size() * 4);
    P.o_bp_eblk = take(P.bp_eblk.size() * 4);
    P.o_bp_wg = take(P.bp_wg.size() * 4);
    P.o_bp_part = take((size_t)P.bp_n_eblk * 32 * 2 * 8);
    P.o_oent = take(P.oent.size() * 2);
    P.o_ohinfo = take(P.ohinfo.size());
    P.o_otbl = take(P.otbl.size() * 4);
    P.o_otiles = take(P.otiles.size() * 4);
    P.o_orec = take((size_t)P.orec_words * 2 * 4);
    P.o_oprog = take((size_t)(P.n_otile + P.n_oblock) * 2 * 4);
    P.o_oqueue = take(9 * 4);  // zero in the uploaded image
    P.o_oqitems = take(P.oqitems.size() * 4);
    P.o_xseen = take(2 * 4);
    P.o_state = o;
    P.o_spins = take((size_t)spinb);
    P.o_E = take((size_t)rep * 8);
    P.o_C = take((size_t)rep * 8);
    P.o_rung = take((size_t)rep * 4);
    P.o_label = take((size_t)rep * 4);
    P.o_rt = take((size_t)rep * 8);
    P.o_repof = take((size_t)rep * 4);
    P.o_sumE = take((size_t)rep * 8);
    P.o_sumC = take((size_t)rep * 8);
    P.o_sumE2 = take((size_t)rep * 8);
    P.o_sumC2 = take((size_t)rep * 8);
    P.o_sumCt = take((size_t)rep * PT_TAU_LAGS * 8);
    P.o_nup = take((size_t)rep * 8);
    P.o_ndown = take((size_t)rep * 8);
    P.o_acc = take((size_t)pair * 8);
    P.o_att = take((size_t)pair * 8);
    P.o_ctr = take((size_t)n_inst * sizeof(Counters));
    P.state_bytes = o - P.o_state;
    P.total_bytes = o;
    return PT_OK;
}

struct CkptHeader {
    uint32_t magic, version;
    uint64_t state_bytes;
    uint64_t seed;
    int32_t n_inst, encoding;
    uint64_t flips_per_sweep;
};
static_assert(sizeof(CkptHeader) == 40, "checkpoint header layout is part of the ABI");

// A checkpoint for these instances and options: the header matches, and every value that
// the kernels use as an index is in range -- spin bytes in {0, 1} (they index threshold
// tables; any bit pattern is a valid bit-packed state), replica_of and rung_of inverse
// permutations of [0, R) per instance (they index energies and tables), labels in
// {NONE, UP, DOWN}.  Nothing is copied anywhere.
int check_checkpoint(const Plan &P, const pt_options &opt, int32_t n_inst, const void *buf,
                     size_t len)
{
    if (!buf) return fail(PT_EINVAL, "null checkpoint");
    if (len < sizeof(CkptHeader)) return fail(PT_ESTATE, "checkpoint too short");
    CkptHeader h;
    std::memcpy(&h, buf, sizeof h);
    if (h.magic != kMagic || h.version != kVersion) return fail(PT_ESTATE, "not a checkpoint");
    if (h.state_bytes != P.state_bytes || h.n_inst != n_inst || h.seed != opt.seed ||
        h.flips_per_sweep != P.flips_per_sweep || len != sizeof h + h.state_bytes)
        return fail(PT_ESTATE, "checkpoint belongs to different instances or options");
    if (h.encoding != opt.encoding)
        return fail(PT_ESTATE, "checkpoint was written under another spin encoding");
    const char *state = (const char *)buf + sizeof h;
    if (P.encoding == PT_INT8) {
        const uint8_t *sp = (const uint8_t *)(state + (P.o_spins - P.o_state));
        for (int64_t b = 0; b < P.spin_bytes; ++b)
            if (sp[b] > 1) return fail(PT_ESTATE, "checkpoint holds invalid spins");
    }
    auto i32_at = [&](size_t off, int64_t k) {
        int32_t v;
        std::memcpy(&v, state + (off - P.o_state) + 4 * k, 4);
        return v;
    };
    for (int32_t n = 0; n < n_inst; ++n) {
        const InstDesc &d = P.desc[n];
        for (int r = 0; r < d.R; ++r) {
            const int32_t c = i32_at(P.o_repof, d.rep_base + r);
            if (c < 0 || c >= d.R || i32_at(P.o_rung, d.rep_base + c) != r)
                return fail(PT_ESTATE, "checkpoint of instance " + std::to_string(n) +
                                           ": replica_of and rung_of are not inverse permutations");
        }
        for (int c = 0; c < d.R; ++c) {
            const int32_t lab = i32_at(P.o_label, d.rep_base + c);
            if (lab != PT_LABEL_NONE && lab != PT_LABEL_UP && lab != PT_LABEL_DOWN)
                return fail(PT_ESTATE, "checkpoint of instance " + std::to_string(n) +
                                           ": invalid round-trip label");
        }
    }
    return PT_OK;
}

}  // namespace

struct pt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *ws = nullptr;
    bool own_ws = false;
    Plan plan;
    DevState st{};
    pt_options opt{};
    uint32_t key_flip0 = 0, key_flip1 = 0, key_swap0 = 0, key_swap1 = 0;
    // launch shape
    std::vector<Tile> tiles;   // fast-kernel tiles, then generic ones, then slice blocks
    int n_fast_tiles = 0, n_generic_tiles = 0, n_block_tiles = 0;
    int lds_block = 0;
    // resident slice blocks: compute-unit occupancy for (block threads, block LDS)
    std::pair<int, int> resident_key{-1, -1};
    int resident_per_cu = 0;
    int block_persistent = 0;   // the last slice-block call ran as one resident launch
    int lane_words = 2;         // whole-replica tiles: four-slice words per lane
    bool block_xcd = false;     // resident slice blocks: every replica's ring on one XCD
    bool lat = false;           // whole-replica tiles: the latency path
    bool oct_resident = false;  // octet slice blocks: one resident launch per call
    // Recovery when a resident launch's wait gave up: a device copy of the state region at
    // the last clean synchronisation, the calls queued since (kind, count: 0 pt_sweep,
    // 1 pt_exchange, 2 pt_run), and whether resident launches are off since a recovery.
    char *shadow = nullptr;
    std::vector<std::pair<int, int>> journal;
    bool replaying = false, resident_off = false;
    int64_t recoveries = 0;
    uint32_t last_device_error = 0;  // the device error word of the last failed synchronisation
    // whole octets from the device work queue; the exchange fused into the octet that
    // completes an instance (every instance of the batch in whole octets)
    bool oct_queue = false, oct_fuse = false;
    int block_threads = 256;
    int tile_bytes = 0;        // target spin bytes per tile in use
    // self-tuning: candidate (tile bytes, threads) shapes timed on the first sweep launches
    bool tuning = false;
    std::vector<std::pair<int, int>> cand;
    std::vector<double> cand_ms;
    size_t cand_next = 0;
    hipEvent_t tune_ev[2] = {nullptr, nullptr};
    int lds_fast = 0, lds_generic = 0;
    int max_P = 1;
    int lds_limit = 65536;     // LDS one workgroup may use
    int cu_lds = 65536;        // LDS of one compute unit
    int cu_threads = 2048;     // resident threads of one compute unit
    int cus = 256;
    std::vector<int> tile_lds; // LDS bytes of every whole-replica tile (block tiles: 0)
    std::vector<int32_t> itiles;  // tiles per instance (host copy)
    int fallbacks = 0;
    bool inject_pending = false;
    // graph of whole cycles for pt_run
    hipGraphExec_t graph = nullptr;
    int graph_cycles = 0;
    // timing
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, int>> sweep_ev, exch_ev;  // indices into ev_pool
    std::vector<int> sweep_ev_calls;  // sweep calls each sweep_ev pair covers
    size_t ev_used = 0;
    double sweep_ms = 0, exch_ms = 0;
    int64_t sweep_n = 0, exch_n = 0;
    // multi-cycle launches: how many were issued and the cycles they ran (always counted),
    // and their event time under PT_FLAG_TIMING (kept apart from the sweep calls)
    std::vector<std::pair<int, int>> multi_ev;
    double multi_ms = 0;
    int64_t multi_launches = 0, multi_cycles = 0;
};

namespace {

int n_inst_of(const pt_ctx *c) { return (int)c->plan.desc.size(); }

// Choose tiles: P replicas of one instance per workgroup, P limited by LDS (and a power of
// two on the fast path), sized so the batch yields a few workgroups per CU when it can
// (the paper's chain packing, Section 5, stops packing once multiprocessors would go
// idle).
int build_tiles(pt_ctx *c, int force_P, int tile_bytes)
{
    const Plan &P = c->plan;
    // the tile list is uploaded from c->tiles: let any earlier upload finish first
    HIP_TRY(hipStreamSynchronize(c->stream));
    int64_t total_bytes = 0;
    for (const auto &d : P.desc) total_bytes += (int64_t)d.R * d.N * d.M;
    int64_t target_bytes = std::max<int64_t>(total_bytes / (2ll * c->cus), 4096);
    target_bytes = std::min<int64_t>(target_bytes, 64 * 1024);
    if (tile_bytes > 0) target_bytes = tile_bytes;
    c->tile_bytes = (int)target_bytes;
    const bool force_blocks = (c->opt.flags & PT_FLAG_SLICE_BLOCKS) != 0;
    std::vector<Tile> fast, generic, block;
    int lds_f = 0, lds_g = 0, lds_b = 0, maxP = 1;
    for (int n = 0; n < (int)P.desc.size(); ++n) {
        const InstDesc &d = P.desc[n];
        int pmax = 0;
        for (int p = d.R; p >= 1; --p)
            if (sweep_tile_lds_bytes(d, P.n_adj[n], p) <= c->lds_limit &&
                (!d.fast || is_pow2(p))) {
                pmax = p;
                break;
            }
        const int lgMh_n = d.fast ? 31 - __builtin_clz((unsigned)d.Mh) : 0;
        const bool blocked = d.fast && (pmax < 1 || d.ent_sh != lgMh_n || (force_blocks && d.G4 >= 2));
        if (blocked && d.ent_mode == kEntXad16)
            return fail(PT_EINVAL, "instance " + std::to_string(n) +
                                       ": 16-bit neighbour entries need whole-replica tiles, "
                                       "but the device's LDS is smaller than the library assumes");
        if (blocked) {
            // slice blocks: ng four-slice groups per parity, halving until a block fits
            int ng = force_blocks ? std::max(1, d.G4 / 4) : d.G4;
            while (ng > 1 && ((int64_t)2 * d.N * 4 * (ng + 1) > std::max<int64_t>(target_bytes, 8 * d.N) ||
                              block_tile_lds_bytes(d, 1, ng) > c->lds_limit))
                ng /= 2;
            if (block_tile_lds_bytes(d, 1, ng) > c->lds_limit)
                return fail(PT_EINVAL, "instance " + std::to_string(n) +
                                           ": even one slice group does not fit in LDS");
            for (int c0 = 0; c0 < d.R; ++c0) {
                const int first = (int)block.size(), nb = d.G4 / ng;
                for (int k = 0; k < nb; ++k) {
                    // prev/next are indices within the block list here, made global below
                    block.push_back(Tile{n, c0, 1, kTileBlock, k * ng, ng, 0,
                                         first + (k + nb - 1) % nb, first + (k + 1) % nb});
                }
            }
            lds_b = std::max(lds_b, block_tile_lds_bytes(d, 1, ng));
            continue;
        }
        if (pmax < 1)
            return fail(PT_EINVAL, "instance " + std::to_string(n) +
                                       ": one replica does not fit in LDS (N*M too large)");
        int p = (int)std::max<int64_t>(1, target_bytes / ((int64_t)d.N * d.M));
        if (force_P > 0) p = force_P;
        p = std::max(1, std::min(p, pmax));
        if (d.fast)
            while (!is_pow2(p)) --p;
        // at most half a compute unit's LDS per tile where fewer replicas allow it, so that
        // two workgroups share a unit and the batch's tiles form one occupancy class
        if (force_P <= 0)
            while (p > 1 && sweep_tile_lds_bytes(d, P.n_adj[n], p) > c->cu_lds / 2)
                p = d.fast ? p / 2 : p - 1;
        for (int c0 = 0; c0 < d.R;) {
            int q = std::min(p, d.R - c0);
            if (d.fast)
                while (!is_pow2(q)) --q;
            Tile t{n, c0, q, d.fast ? kTileFast : kTileGeneric, 0, d.G4};
            (d.fast ? fast : generic).push_back(t);
            const int b = sweep_tile_lds_bytes(d, P.n_adj[n], q);
            (d.fast ? lds_f : lds_g) = std::max(d.fast ? lds_f : lds_g, b);
            maxP = std::max(maxP, q);
            c0 += q;
        }
    }
    // Tiles in order of decreasing LDS need, ties by decreasing work.  Launches then split
    // the list into occupancy classes (see launch_groups) and each class starts with its
    // largest tiles: the device dispatches workgroups roughly in order, so the longest work
    // starts earliest (the paper's "hardest chains first" work pool, Section 4).
    auto lds_of = [&](const Tile &t) { return sweep_tile_lds_bytes(P.desc[t.inst], P.n_adj[t.inst], t.P); };
    auto bigger = [&](const Tile &a, const Tile &b) {
        const int la = lds_of(a), lb = lds_of(b);
        if (la != lb) return la > lb;
        const InstDesc &da = P.desc[a.inst], &db = P.desc[b.inst];
        return (int64_t)a.P * da.M * da.N > (int64_t)b.P * db.M * db.N;
    };
    std::stable_sort(fast.begin(), fast.end(), bigger);
    std::stable_sort(generic.begin(), generic.end(), bigger);
    if ((int64_t)(fast.size() + generic.size() + block.size()) > P.max_tiles)
        return fail(PT_ESTATE, "internal: more tiles than reserved tile slots");
    // slice blocks: global neighbour indices and boundary-record offsets
    const int block0 = (int)(fast.size() + generic.size());
    int64_t hb = 0;
    for (Tile &t : block) {
        t.prev += block0;
        t.next += block0;
        t.hb = (int32_t)hb;
        hb += 3ll * P.desc[t.inst].N;
    }
    if (hb > P.halo_words || hb > 0x7fffffff)
        return fail(PT_EINVAL, "slice blocks need more boundary records than were reserved "
                               "(the device's LDS is smaller than the library assumes)");
    // Resident slice blocks pass boundary records to the neighbouring blocks of their
    // replica every sweep: when every replica's ring of blocks lies in one run of the
    // launches' workgroup-to-tile map (so on one XCD), the records pass through that XCD's
    // L2 instead of device-scope operations.
    {
        std::vector<std::pair<int, int>> rings;
        const int nb = (int)block.size();
        for (int k = 0; k < nb;) {
            int e = k + 1;
            while (e < nb && block[e].inst == block[k].inst && block[e].c0 == block[k].c0) ++e;
            rings.emplace_back(k, e);
            k = e;
        }
        c->block_xcd = rings_in_runs(rings, nb);
    }
    c->tiles = fast;
    c->tiles.insert(c->tiles.end(), generic.begin(), generic.end());
    c->tiles.insert(c->tiles.end(), block.begin(), block.end());
    c->n_fast_tiles = (int)fast.size();
    c->n_generic_tiles = (int)generic.size();
    c->tile_lds.assign(c->tiles.size(), 0);
    for (size_t k = 0; k < fast.size() + generic.size(); ++k) c->tile_lds[k] = lds_of(c->tiles[k]);
    c->n_block_tiles = (int)block.size();
    c->lds_fast = lds_f;
    c->lds_generic = lds_g;
    c->lds_block = lds_b;
    c->max_P = maxP;
    HIP_TRY(hipMemcpyAsync(c->ws + P.o_tiles, c->tiles.data(), c->tiles.size() * sizeof(Tile),
                           hipMemcpyHostToDevice, c->stream));
    // tiles per instance: a PT cycle's exchange runs in the tile that completes the instance
    c->itiles.assign(P.desc.size(), 0);
    for (const Tile &t : c->tiles) c->itiles[t.inst] += 1;
    HIP_TRY(hipMemcpyAsync(c->ws + P.o_itiles, c->itiles.data(), c->itiles.size() * 4,
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(sweep_kernels_set_lds(c->lds_fast, c->lds_generic, c->lds_block));
    // Whole-replica tiles: two four-slice words per lane, unless the batch's lanes of one
    // colour class at that width would not give every SIMD of the device one wave; then
    // the sweep is a chain of short, barely parallel class steps, and one word per lane
    // (twice the lanes, half the dependent work each) shortens every step (measured on
    // config 2, 2304 lanes per class: 3.6e10 attempts/s against 3.0e10).  Instances with
    // 16-bit neighbour entries are swept by the two-word instantiations only, so any such
    // instance keeps the batch at two words.
    int64_t lanes = 0;
    bool ent16 = false;
    for (int k = 0; k < c->n_fast_tiles; ++k) {
        const Tile &t = c->tiles[k];
        const InstDesc &d = P.desc[t.inst];
        ent16 = ent16 || d.ent_mode == kEntXad16;
        int64_t most = 0;
        for (int g = 0; g < d.n_colors; ++g)
            most = std::max<int64_t>(most, P.cls_off[d.cls_base + g + 1] - P.cls_off[d.cls_base + g]);
        lanes += (int64_t)t.P * most * std::max(1, d.G4 / 2);
    }
    c->lane_words = (c->opt.flags & PT_FLAG_FOUR_SLICE_LANES) ? 1
                    : ((c->opt.flags & PT_FLAG_TWO_WORD_LANES) || ent16) ? 2
                    : lanes < (int64_t)c->cus * 256 ? 1
                                                    : 2;
    // At most one whole-replica tile per compute unit: no other workgroup's waves overlap a
    // tile's class steps, so the kernel forms each thread's next item while the current one
    // is in flight (the tiles whose classes fit one pass of the workgroup).
    c->lat = !(c->opt.flags & PT_FLAG_NO_LATENCY_PATH) && c->n_fast_tiles > 0 &&
             c->n_fast_tiles <= c->cus;
    return PT_OK;
}

void drop_graph(pt_ctx *c)
{
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
    c->graph_cycles = 0;
}

int event_pair(pt_ctx *c, int &a, int &b)
{
    while (c->ev_pool.size() < c->ev_used + 2) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        c->ev_pool.push_back(e);
    }
    a = (int)c->ev_used++;
    b = (int)c->ev_used++;
    return PT_OK;
}

// Accumulate the elapsed times of recorded event pairs (synchronises).
int harvest_events(pt_ctx *c)
{
    if (c->ev_used == 0) return PT_OK;
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (size_t k = 0; k < c->sweep_ev.size(); ++k) {
        const auto &p = c->sweep_ev[k];
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev_pool[p.first], c->ev_pool[p.second]));
        c->sweep_ms += ms;
        c->sweep_n += k < c->sweep_ev_calls.size() ? c->sweep_ev_calls[k] : 1;
    }
    for (auto &p : c->exch_ev) {
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev_pool[p.first], c->ev_pool[p.second]));
        c->exch_ms += ms;
        c->exch_n++;
    }
    for (auto &p : c->multi_ev) {
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev_pool[p.first], c->ev_pool[p.second]));
        c->multi_ms += ms;
    }
    c->sweep_ev.clear();
    c->sweep_ev_calls.clear();
    c->exch_ev.clear();
    c->multi_ev.clear();
    c->ev_used = 0;
    return PT_OK;
}

bool out_of_resources(hipError_t e)
{
    return e == hipErrorLaunchOutOfResources || e == hipErrorOutOfMemory ||
           e == hipErrorInvalidConfiguration;
}

// Launch n sweeps of every tile; on a resource failure halve the tile (and, at one
// replica per tile, the workgroup) and retry, as the paper's Figure 7 halves its chain
// packing when a launch runs out of registers.
// One launch of whole-replica tiles: a run of consecutive tiles of one kind that the
// compute units can hold `per_cu` at a time.
struct LaunchGroup {
    int kind, tile0, n_tiles, lds_bytes, per_cu;
};

// Workgroups of `lds` bytes a compute unit holds at once with the current block size.
int occupancy(const pt_ctx *c, int lds)
{
    const int by_threads = std::max(1, c->cu_threads / std::max(1, c->block_threads));
    const int by_lds = lds > 0 ? std::max(1, c->cu_lds / lds) : by_threads;
    return std::min(by_threads, by_lds);
}

// Split the (LDS-descending) tile lists into occupancy classes, one launch each, sized to
// the largest tile of the class.  A single launch would reserve the largest tile's LDS for
// every workgroup and hold small tiles to the occupancy of the largest.
std::vector<LaunchGroup> launch_groups(const pt_ctx *c)
{
    std::vector<LaunchGroup> out;
    auto add_range = [&](int kind, int begin, int end) {
        int t = begin;
        while (t < end) {
            const int k = occupancy(c, c->tile_lds[t]);
            int u = t + 1;
            while (u < end && occupancy(c, c->tile_lds[u]) == k) ++u;
            out.push_back(LaunchGroup{kind, t, u - t, c->tile_lds[t], k});
            t = u;
        }
    };
    add_range(kTileFast, 0, c->n_fast_tiles);
    add_range(kTileGeneric, c->n_fast_tiles, c->n_fast_tiles + c->n_generic_tiles);
    return out;
}

// Whether the resident slice-block kernel can hold every block tile at once with the
// current block size: the grid must fit the compute units' occupancy, or the blocks that
// wait for their neighbours could wait for blocks that never start.
hipError_t blocks_resident(pt_ctx *c, bool &resident)
{
    resident = false;
    if ((c->opt.flags & PT_FLAG_BLOCK_LAUNCH_PER_SWEEP) || c->resident_off) return hipSuccess;
    if (c->resident_key != std::make_pair(c->block_threads, c->lds_block)) {
        int32_t per_cu = 0;
        const hipError_t e = block_resident_per_cu(c->block_threads, c->lds_block, &per_cu);
        if (e != hipSuccess) return e;
        c->resident_key = std::make_pair(c->block_threads, c->lds_block);
        c->resident_per_cu = per_cu;
    }
    resident = (int64_t)c->n_block_tiles <= (int64_t)c->resident_per_cu * c->cus;
    return hipSuccess;
}

int recover(pt_ctx *c);

// The state region copied to the shadow copy, the journal cleared (stream-ordered: the
// copy reads the state as the calls queued so far leave it).
hipError_t take_snapshot(pt_ctx *c)
{
    c->journal.clear();
    if (!c->shadow) return hipSuccess;
    return hipMemcpyAsync(c->shadow, c->ws + c->plan.o_state, c->plan.state_bytes,
                          hipMemcpyDeviceToDevice, c->stream);
}

void journal_add(pt_ctx *c, int kind, int n)
{
    if (c->shadow && !c->replaying) c->journal.emplace_back(kind, n);
}

// Wait for the stream, then check the device error word (a resident slice-block launch
// that gave up a wait, an octet kernel that refused to run).  After a wait that gave up,
// the state is restored from the copy of the last clean synchronisation and the calls
// queued since are replayed with every slice block launched per sweep (or per parity),
// which gives the chain's state again; otherwise the call fails with PT_ESTATE (the word
// is cleared, and the chain state after such a launch is not the sampler's).  A clean
// synchronisation after new calls takes a new copy.
int sync_and_check(pt_ctx *c)
{
    HIP_TRY(hipStreamSynchronize(c->stream));
    uint32_t err = 0;
    HIP_TRY(hipMemcpy(&err, c->ws + c->plan.o_err, 4, hipMemcpyDeviceToHost));
    if (err != 0) {
        c->last_device_error = err;
        const uint32_t zero = 0;
        HIP_TRY(hipMemcpy(c->ws + c->plan.o_err, &zero, 4, hipMemcpyHostToDevice));
        if (err & kErrLdsBase)
            return fail(PT_ESTATE, "an octet kernel found its dynamic LDS away from address 0 "
                                   "and did not run; the state is inconsistent");
        if ((err & kErrPlace) && c->shadow && !c->replaying) return recover(c);
        if (err & kErrPlace)
            return fail(PT_ESTATE, "the workgroups of a resident slice-block launch did not keep "
                                   "to round-robin XCDs; the state is inconsistent");
        if (err & kErrQueue)
            return fail(PT_ESTATE, "a whole-octet workgroup found every work queue empty; the "
                                   "state is inconsistent");
        if (c->shadow && !c->replaying) return recover(c);
        return fail(PT_ESTATE, "a resident slice-block launch waited too long for its "
                               "neighbouring blocks; the state is inconsistent");
    }
    if (!c->journal.empty() && !c->replaying) HIP_TRY(take_snapshot(c));
    return PT_OK;
}

// E_cl and C of replicas [rep_first, rep_first + n) from the spins in device memory (the
// bit-packed encoding recomputes every replica).
hipError_t energies_from_spins(pt_ctx *c, int rep_first, int n)
{
    if (c->plan.encoding == PT_BITPACK32)
        return launch_bp_energy(c->st, c->plan.bp_n_eblk, (int32_t)c->plan.total_reps, c->stream);
    return launch_energy(c->st, rep_first, n, c->stream);
}

// Whole octets from the device work queue: as many workgroups as the compute units hold at
// once for the current block size (at most one per octet).
// Resident byte slice blocks pass their records through the L2 of the XCD that holds their
// replica's ring.
bool block_ring_xcd(const pt_ctx *c)
{
    return c->block_xcd && c->n_block_tiles > 0 && !c->resident_off &&
           !(c->opt.flags & (PT_FLAG_DEVICE_SCOPE_RECORDS | PT_FLAG_BLOCK_LAUNCH_PER_SWEEP));
}

// Resident octet slice blocks pass their records through the L2 of the XCD that holds
// their ring (the rings were placed one per XCD).
bool oct_ring_xcd(const pt_ctx *c)
{
    return c->oct_resident && c->plan.oblock_xcd &&
           !(c->opt.flags & PT_FLAG_DEVICE_SCOPE_RECORDS);
}

// Bit-packed encoding: n_sweeps sweeps as one launch per colour class (parity, colour) of
// every instance, then E_cl and C of every replica.
int enqueue_bp_sweep(pt_ctx *c, int n_sweeps, bool fuse_exchange)
{
    const Plan &P = c->plan;
    const bool timing = (c->opt.flags & PT_FLAG_TIMING) != 0;
    int ea = -1, eb = -1;
    if (timing) {
        int rc = event_pair(c, ea, eb);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(c->ev_pool[ea], c->stream));
    }
    // octets: whole octets in one launch for all sweeps of the call; slice blocks in one
    // resident launch, or else one launch per parity of every sweep, their E_cl and C
    // cleared first and summed by the resident launch or the last phase launch
    OctLaunch O{};
    O.st = c->st;
    O.key0 = c->key_flip0;
    O.key1 = c->key_flip1;
    O.n_sweeps = n_sweeps;
    if (P.n_otile > 0) {
        O.tile0 = 0;
        O.n_tiles = P.n_otile;
        O.threads = c->block_threads;
        O.lds_bytes = P.otile_lds;
        O.queue = c->oct_queue ? 1 : 0;
        if (fuse_exchange) {
            O.fuse = 1;
            O.swap_key0 = c->key_swap0;
            O.swap_key1 = c->key_swap1;
            O.t_add = (uint32_t)n_sweeps;
        }
        const hipError_t e = launch_oct_tiles(O, c->stream);
        if (e != hipSuccess) return hip_fail(e, "octet tile launch");
        O.queue = O.fuse = 0;
    }
    if (P.n_oblock > 0) {
        O.tile0 = P.n_otile;
        O.n_tiles = P.n_oblock;
        O.threads = P.oblock_threads;
        O.lds_bytes = P.oblock_lds;
        O.split = P.oblock_split ? 1 : 0;
        hipError_t e = launch_oct_clear(O, c->stream);
        if (e != hipSuccess) return hip_fail(e, "octet clear launch");
        if (c->oct_resident) {
            O.lds_bytes = P.oblock_res_lds;
            O.rec_words = (int32_t)P.orec_words;
            O.xcd_local = !oct_ring_xcd(c) ? 0 : (c->opt.flags & PT_FLAG_TEST_XCD_MISMATCH) ? 2 : 1;
            if (c->opt.flags & PT_FLAG_TEST_BLOCK_WAIT_TIMEOUT) {
                O.wait_polls = 16;
                O.wait_extra = 1 << 30;
            }
            e = launch_oct_resident(O, c->stream);
            if (e != hipSuccess) return hip_fail(e, "octet resident launch");
        }
        for (int sw = 0; sw < n_sweeps && !c->oct_resident; ++sw)
            for (int p = 0; p < 2; ++p) {
                O.sweep_off = sw;
                O.p = p;
                O.last = (sw == n_sweeps - 1 && p == 1) ? 1 : 0;
                e = launch_oct_phase(O, c->stream);
                if (e != hipSuccess) return hip_fail(e, "octet slice-block launch");
            }
    }
    if (P.bp_generic) {
        int parities = 1;
        for (const auto &d : P.desc) parities = std::max(parities, d.parities);
        BpLaunch L{};
        L.st = c->st;
        L.key0 = c->key_flip0;
        L.key1 = c->key_flip1;
        for (int sw = 0; sw < n_sweeps; ++sw)
            for (int p = 0; p < parities; ++p)
                for (int g = 0; g < (int)P.bp_colour.size(); ++g) {
                    L.sweep_off = sw;
                    L.p = p;
                    L.g = g;
                    L.blk0 = P.bp_colour[g].first;
                    L.n_blocks = P.bp_colour[g].second;  // instances with one parity skip p = 1
                    if (L.n_blocks == 0) continue;
                    const hipError_t e = launch_bp_sweep(L, c->stream);
                    if (e != hipSuccess) return hip_fail(e, "bit-packed sweep launch");
                }
        // E_cl and C of every replica (the octets' are recomputed to the same values)
        const hipError_t e = energies_from_spins(c, 0, (int)P.total_reps);
        if (e != hipSuccess) return hip_fail(e, "bit-packed energy launch");
    }
    if (timing) {
        HIP_TRY(hipEventRecord(c->ev_pool[eb], c->stream));
        c->sweep_ev.emplace_back(ea, eb);
        c->sweep_ev_calls.push_back(1);
    }
    return PT_OK;
}

// n_sweeps sweeps of every tile; with fuse_exchange the tile that completes an instance
// then runs the instance's exchange step (a PT cycle in one set of launches).
// Every tile a fast whole-replica tile holding a whole instance (the condition for a
// launch of several PT cycles).
bool whole_instance_tiles(const pt_ctx *c)
{
    if (c->n_generic_tiles != 0 || c->n_block_tiles != 0 || c->n_fast_tiles != n_inst_of(c))
        return false;
    for (int k = 0; k < c->n_fast_tiles; ++k) {
        const Tile &t = c->tiles[k];
        const InstDesc &d = c->plan.desc[t.inst];
        // the multi-cycle kernel does not carry 16-bit neighbour entries
        if (t.c0 != 0 || t.P != d.R || d.ent_mode == kEntXad16) return false;
    }
    return true;
}

// Whether the whole-replica tiles sweep on the latency path with workgroups of `threads`:
// at most one tile per compute unit (no other workgroup overlaps a tile's class steps),
// and in some tile every step of the pipelined order (class k of parity 0 with class k - 1
// of parity 1) fits one pass of the workgroup, at least two classes and a degree of at
// most eight.  The kernel checks the per-tile condition again and sweeps the other tiles
// as usual.
bool latency_path(const pt_ctx *c, int threads)
{
    if (!c->lat) return false;
    bool any = false;
    for (int k = 0; k < c->n_fast_tiles && !any; ++k) {
        const Tile &t = c->tiles[k];
        const InstDesc &d = c->plan.desc[t.inst];
        if (d.n_colors < 2 || d.D < 1 || d.D > 8) continue;
        const int nw = (c->lane_words == 2 && d.G4 >= 2) ? 2 : 1;
        const int64_t lanes = (int64_t)t.P * (d.G4 / nw);  // per site
        if (lanes > threads) continue;
        const int32_t *off = c->plan.cls_off.data() + d.cls_base;
        int most = 0;
        for (int g = 0; g < d.n_colors; ++g) {
            const int gb = (g == 0 ? d.n_colors : g) - 1;
            most = std::max(most, off[g + 1] - off[g] + off[gb + 1] - off[gb]);
        }
        any = (int64_t)most * lanes <= threads;
    }
    return any;
}

// enqueue_sweep_once with cycles > 1 found the tiles no longer whole instances (after a
// launch-failure fallback): nothing was queued, run the cycles one by one.
constexpr int kCycleByCycle = 1;

int enqueue_sweep_once(pt_ctx *c, int n_sweeps, bool fuse_exchange, int cycles = 1)
{
    if (n_sweeps <= 0) return PT_OK;
    const bool timing = (c->opt.flags & PT_FLAG_TIMING) != 0;
    for (;;) {
        if (cycles > 1 && !whole_instance_tiles(c)) return kCycleByCycle;
        SweepLaunch L{};
        L.st = c->st;
        L.key0 = c->key_flip0;
        L.key1 = c->key_flip1;
        L.n_sweeps = n_sweeps;
        L.block_threads = c->block_threads;
        L.lane_words = c->lane_words;
        L.lat = latency_path(c, c->block_threads) ? 1 : 0;
        L.fuse_exchange = fuse_exchange ? 1 : 0;
        L.swap_key0 = c->key_swap0;
        L.swap_key1 = c->key_swap1;
        L.t_add = (uint32_t)n_sweeps;
        L.cycles = cycles;
        int ea = -1, eb = -1;
        if (timing) {
            int rc = event_pair(c, ea, eb);
            if (rc) return rc;
            HIP_TRY(hipEventRecord(c->ev_pool[ea], c->stream));
        }
        hipError_t e = hipSuccess;
        int queued = 0;  // launches of this call already queued
        if (c->inject_pending) {
            c->inject_pending = false;
            e = hipErrorLaunchOutOfResources;
        } else {
            for (const LaunchGroup &g : launch_groups(c)) {
                L.tile0 = g.tile0;
                L.n_tiles = g.n_tiles;
                L.lds_bytes = g.lds_bytes;
                e = launch_sweep(L, g.kind, c->stream);
                if (e != hipSuccess) break;
                ++queued;
            }
            // slice blocks: boundary records of the current state (and E_cl, C cleared),
            // then all sweeps in one launch when every block can be resident at once,
            // else one launch per sweep
            L.tile0 = c->n_fast_tiles + c->n_generic_tiles;
            L.n_tiles = c->n_block_tiles;
            L.lds_bytes = c->lds_block;
            if (e == hipSuccess && L.n_tiles > 0) {
                e = launch_block_prepare(L, c->stream);
                if (e == hipSuccess) ++queued;
            }
            if (e == hipSuccess && L.n_tiles > 0) {
                bool resident = false;
                e = blocks_resident(c, resident);
                c->block_persistent = resident ? 1 : 0;
                if (e == hipSuccess && resident) {
                    L.persist = 1;
                    L.xcd_local = !block_ring_xcd(c) ? 0
                                  : (c->opt.flags & PT_FLAG_TEST_XCD_MISMATCH) ? 2 : 1;
                    if (c->opt.flags & PT_FLAG_TEST_BLOCK_WAIT_TIMEOUT) {
                        L.wait_polls = 16;
                        L.wait_extra = 1 << 30;
                    }
                    L.sweep_off = 0;
                    L.last = 1;
                    e = launch_sweep(L, kTileBlock, c->stream);
                    if (e == hipSuccess) ++queued;
                } else {
                    for (int sw = 0; sw < n_sweeps && e == hipSuccess; ++sw) {
                        L.sweep_off = sw;
                        L.last = (sw == n_sweeps - 1);
                        e = launch_sweep(L, kTileBlock, c->stream);
                        if (e == hipSuccess) ++queued;
                    }
                }
            }
        }
        if (e == hipSuccess) {
            if (timing) {
                HIP_TRY(hipEventRecord(c->ev_pool[eb], c->stream));
                if (cycles > 1) {
                    c->multi_ev.emplace_back(ea, eb);
                } else {
                    c->sweep_ev.emplace_back(ea, eb);
                    c->sweep_ev_calls.push_back(1);
                }
            }
            if (cycles > 1) {
                c->multi_launches += 1;
                c->multi_cycles += cycles;
            }
            return PT_OK;
        }
        if (timing) c->ev_used -= 2;
        if (!out_of_resources(e)) return hip_fail(e, "sweep launch");
        if (queued > 0)  // part of the call already runs: retrying would sweep it twice
            return fail(PT_ESTATE, std::string("a sweep launch failed after part of the call "
                                               "was queued; the state is inconsistent: ") +
                                       hipGetErrorString(e));
        (void)hipGetLastError();
        c->fallbacks++;
        drop_graph(c);
        if (c->max_P > 1) {
            int rc = build_tiles(c, std::max(1, c->max_P / 2), 0);
            if (rc) return rc;
        } else if (c->block_threads > 64) {
            c->block_threads /= 2;
        } else {
            return fail(PT_ELAUNCH, std::string("sweep kernel cannot be launched: ") +
                                        hipGetErrorString(e));
        }
    }
}

// Self-tuning: while candidates remain, each sweep launch uses the next candidate shape
// and is timed (synchronously) with its own events.  The candidates are run in
// kTuneRounds rounds, each keeping its best per-sweep time (one timing of a short call
// can be off by more than the gap between shapes), and the fastest shape is kept.
// Launch shape does not change the trajectory, so tuning costs only the slower
// candidates' extra time.
constexpr size_t kTuneRounds = 3;
int enqueue_sweep(pt_ctx *c, int n_sweeps, bool fuse_exchange)
{
    if (n_sweeps <= 0) return PT_OK;
    const bool bp = c->plan.encoding == PT_BITPACK32;
    if (!c->tuning)
        return bp ? enqueue_bp_sweep(c, n_sweeps, fuse_exchange)
                  : enqueue_sweep_once(c, n_sweeps, fuse_exchange);
    const size_t nc = c->cand.size();
    const size_t k = c->cand_next % nc;
    const auto shape = c->cand[k];
    int rc = PT_OK;
    if (!bp) {
        rc = build_tiles(c, 0, shape.first);
        if (rc) return rc;
    }
    c->block_threads = shape.second;
    HIP_TRY(hipEventRecord(c->tune_ev[0], c->stream));
    const int fb = c->fallbacks;
    rc = bp ? enqueue_bp_sweep(c, n_sweeps, fuse_exchange)
            : enqueue_sweep_once(c, n_sweeps, fuse_exchange);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(c->tune_ev[1], c->stream));
    HIP_TRY(hipEventSynchronize(c->tune_ev[1]));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, c->tune_ev[0], c->tune_ev[1]));
    const double t = (c->fallbacks == fb) ? (double)ms / n_sweeps : 1e30;
    c->cand_ms[k] = (c->cand_next < nc) ? t : std::min(c->cand_ms[k], t);
    if (++c->cand_next == kTuneRounds * nc) {
        size_t best = 0;
        for (size_t j = 1; j < nc; ++j)
            if (c->cand_ms[j] < c->cand_ms[best]) best = j;
        c->tuning = false;
        if (!bp) {
            rc = build_tiles(c, 0, c->cand[best].first);
            if (rc) return rc;
        }
        c->block_threads = c->cand[best].second;
    }
    return PT_OK;
}

int enqueue_exchange(pt_ctx *c, uint32_t t_add)
{
    const bool timing = (c->opt.flags & PT_FLAG_TIMING) != 0;
    int ea = -1, eb = -1;
    if (timing) {
        int rc = event_pair(c, ea, eb);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(c->ev_pool[ea], c->stream));
    }
    hipError_t e = launch_exchange(c->st, n_inst_of(c), c->key_swap0, c->key_swap1, t_add,
                                   c->stream);
    if (e != hipSuccess) return hip_fail(e, "exchange launch");
    if (timing) {
        HIP_TRY(hipEventRecord(c->ev_pool[eb], c->stream));
        c->exch_ev.emplace_back(ea, eb);
    }
    return PT_OK;
}

// Batches of at most this many tiles run a PT cycle as one set of launches, the exchange
// step in the tile that completes each instance.  Each tile then ends with an agent-scope
// release (its energies must reach the other XCDs' caches), which costs more than the
// separate exchange launch it saves once a call has thousands of tiles; small batches are
// launch-latency bound and gain (measured: 1 tile +22 %, 32 tiles +4 %, 256 tiles -4 %,
// 7797 tiles -9 %).
constexpr size_t kFuseMaxTiles = 64;

static_assert(kTauLags == PT_TAU_LAGS, "device and ABI correlation lags differ");

// With PT_FLAG_TAU_CORR: after an exchange step, the imaginary-time correlations of
// every replica at its new rung.
int enqueue_tau_corr(pt_ctx *c)
{
    if (!(c->opt.flags & PT_FLAG_TAU_CORR)) return PT_OK;
    // workgroups per replica: about 8192 (parity, site, four-slice group) positions each,
    // for the largest replica of the batch
    int64_t most = 1;
    for (const auto &d : c->plan.desc) most = std::max<int64_t>(most, (int64_t)d.parities * d.N * d.G4);
    const int32_t chunks = (int32_t)std::min<int64_t>(64, (most + 8191) / 8192);
    const hipError_t e = launch_tau_corr(c->st, (int32_t)c->plan.total_reps, chunks, c->stream);
    if (e != hipSuccess) return hip_fail(e, "correlation launch");
    return PT_OK;
}

int enqueue_cycle(pt_ctx *c)
{
    const int k = c->opt.sweeps_per_exchange;
    int rc;
    if ((c->plan.encoding == PT_INT8 && c->tiles.size() <= kFuseMaxTiles) || c->oct_fuse) {
        rc = enqueue_sweep(c, k, true);
    } else {
        rc = enqueue_sweep(c, k, false);
        if (rc == PT_OK) rc = enqueue_exchange(c, (uint32_t)k);
    }
    if (rc) return rc;
    return enqueue_tau_corr(c);
}

int check_inst(pt_ctx *c, int32_t inst)
{
    if (!c) return fail(PT_EINVAL, "null context");
    if (inst < 0 || inst >= n_inst_of(c)) return fail(PT_EINVAL, "instance index out of range");
    return PT_OK;
}

}  // namespace

int ptq::report_error(int code, const char *msg) { return fail(code, msg); }

extern "C" {

int pt_workspace_bytes(const pt_instance *inst, int32_t n_inst, const pt_options *opt,
                       size_t *bytes)
{
    if (!bytes || !opt) return fail(PT_EINVAL, "null argument");
    Plan P;
    int rc = make_plan(inst, n_inst, opt->flags, opt->encoding, P);
    if (rc) return rc;
    *bytes = P.total_bytes;
    return PT_OK;
}

int pt_init(pt_ctx **out, const pt_instance *inst, int32_t n_inst, const pt_options *opt,
            void *stream, void *workspace, size_t workspace_bytes)
{
    if (!out || !opt) return fail(PT_EINVAL, "null argument");
    *out = nullptr;
    if (opt->sweeps_per_exchange < 1) return fail(PT_EINVAL, "sweeps_per_exchange must be >= 1");
    if (opt->encoding != PT_INT8 && opt->encoding != PT_BITPACK32)
        return fail(PT_EINVAL, "unknown encoding");
    if (opt->encoding == PT_BITPACK32 && (opt->flags & PT_FLAG_TAU_CORR))
        return fail(PT_EINVAL, "PT_FLAG_TAU_CORR needs PT_INT8 spins");
    if (opt->block_threads < 0 || opt->block_threads > 1024 || (opt->block_threads % 64))
        return fail(PT_EINVAL, "block_threads must be a multiple of 64 in [64, 1024] or 0");
    if (opt->tile_replicas < 0 || opt->tile_bytes < 0)
        return fail(PT_EINVAL, "tile_replicas and tile_bytes must be >= 0");
    pt_ctx *c = new (std::nothrow) pt_ctx();
    if (!c) return fail(PT_ENOMEM, "host allocation failed");
    int rc = make_plan(inst, n_inst, opt->flags, opt->encoding, c->plan);
    if (rc) {
        delete c;
        return rc;
    }
    const Plan &P = c->plan;
    c->opt = *opt;
    c->inject_pending = (opt->flags & PT_FLAG_INJECT_LAUNCH_OOR_ONCE) != 0;
    c->key_flip0 = (uint32_t)opt->seed;
    c->key_flip1 = (uint32_t)(opt->seed >> 32);
    c->key_swap0 = c->key_flip0;
    c->key_swap1 = c->key_flip1 ^ kDomainSwap;
    auto cleanup = [&](int code) {
        pt_free(c);
        return code;
    };
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hipGetDevice"));
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) ==
            hipSuccess && v > 0)
        c->lds_limit = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, c->device) ==
            hipSuccess && v > 0)
        c->cus = v;
    c->cu_lds = c->lds_limit;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, c->device) ==
            hipSuccess && v > 0)
        c->cu_lds = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxThreadsPerMultiProcessor, c->device) ==
            hipSuccess && v > 0)
        c->cu_threads = v;
    if (workspace) {
        if (workspace_bytes < P.total_bytes)
            return cleanup(fail(PT_ENOMEM, "workspace smaller than pt_workspace_bytes()"));
        if (((uintptr_t)workspace) % 256)
            return cleanup(fail(PT_EINVAL, "workspace must be 256-byte aligned"));
        c->ws = (char *)workspace;
    } else {
        e = hipMalloc((void **)&c->ws, P.total_bytes);
        if (e != hipSuccess) return cleanup(fail(PT_ENOMEM, "hipMalloc of the workspace failed"));
        c->own_ws = true;
    }
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        e = hipStreamCreate(&c->stream);
        if (e != hipSuccess) return cleanup(hip_fail(e, "hipStreamCreate"));
        c->own_stream = true;
    }
    char *w = c->ws;
    DevState &st = c->st;
    st.inst = (const InstDesc *)(w + P.o_inst);
    st.adj = (const int32_t *)(w + P.o_adj);
    st.adj_off = (const int32_t *)(w + P.o_off);
    st.hfield = (const int16_t *)(w + P.o_h);
    st.ent = (const uint32_t *)(w + P.o_ent);
    st.bias = (const uint32_t *)(w + P.o_bias);
    st.csite = (const uint16_t *)(w + P.o_csite);
    st.cls_off = (const int32_t *)(w + P.o_cls);
    st.tbl = (const uint32_t *)(w + P.o_tbl);
    st.db = (const double *)(w + P.o_db);
    st.dK = (const double *)(w + P.o_dK);
    st.tiles = (const Tile *)(w + P.o_tiles);
    st.spins = (uint8_t *)(w + P.o_spins);
    st.E = (int64_t *)(w + P.o_E);
    st.C = (int64_t *)(w + P.o_C);
    st.rung_of = (int32_t *)(w + P.o_rung);
    st.label = (int32_t *)(w + P.o_label);
    st.rt = (uint64_t *)(w + P.o_rt);
    st.replica_of = (int32_t *)(w + P.o_repof);
    st.sumE = (int64_t *)(w + P.o_sumE);
    st.sumC = (int64_t *)(w + P.o_sumC);
    st.sumE2 = (int64_t *)(w + P.o_sumE2);
    st.sumC2 = (int64_t *)(w + P.o_sumC2);
    st.sumCt = (int64_t *)(w + P.o_sumCt);
    st.nup = (uint64_t *)(w + P.o_nup);
    st.ndown = (uint64_t *)(w + P.o_ndown);
    st.acc = (uint64_t *)(w + P.o_acc);
    st.att = (uint64_t *)(w + P.o_att);
    st.ctr = (Counters *)(w + P.o_ctr);
    st.rep_inst = (const int32_t *)(w + P.o_repinst);
    st.halo = (uint32_t *)(w + P.o_halo);
    st.halo_words = P.halo_words;
    st.itiles = (const int32_t *)(w + P.o_itiles);
    st.icount = (uint32_t *)(w + P.o_icount);
    st.prog = (int32_t *)(w + P.o_prog);
    st.err = (uint32_t *)(w + P.o_err);
    st.bp_sblk = (const int32_t *)(w + P.o_bp_sblk);
    st.bp_eblk = (const int32_t *)(w + P.o_bp_eblk);
    st.bp_wg = (const int32_t *)(w + P.o_bp_wg);
    st.bp_part = (int64_t *)(w + P.o_bp_part);
    st.oent = (const uint16_t *)(w + P.o_oent);
    st.ohinfo = (const uint8_t *)(w + P.o_ohinfo);
    st.otbl = (const uint32_t *)(w + P.o_otbl);
    st.otiles = (const int32_t *)(w + P.o_otiles);
    st.orec = (uint32_t *)(w + P.o_orec);
    st.oprog = (int32_t *)(w + P.o_oprog);
    st.oqueue = (int32_t *)(w + P.o_oqueue);
    st.oqitems = (const int32_t *)(w + P.o_oqitems);
    st.xseen = (uint32_t *)(w + P.o_xseen);

    // one host image of the whole workspace, uploaded in a single copy
    std::vector<char> img;
    try {
        img.assign(P.total_bytes, 0);
    } catch (...) {
        return cleanup(fail(PT_ENOMEM, "host staging allocation failed"));
    }
    auto put = [&](size_t off, const void *src, size_t bytes) {
        if (bytes) std::memcpy(img.data() + off, src, bytes);
    };
    put(P.o_inst, P.desc.data(), P.desc.size() * sizeof(InstDesc));
    put(P.o_adj, P.adj.data(), P.adj.size() * 4);
    put(P.o_off, P.adj_off.data(), P.adj_off.size() * 4);
    put(P.o_h, P.hfield.data(), P.hfield.size() * 2);
    put(P.o_ent, P.ent.data(), P.ent.size() * 4);
    put(P.o_bias, P.bias.data(), P.bias.size() * 4);
    put(P.o_csite, P.csite.data(), P.csite.size() * 2);
    put(P.o_cls, P.cls_off.data(), P.cls_off.size() * 4);
    put(P.o_tbl, P.tbl.data(), P.tbl.size() * 4);
    put(P.o_db, P.db.data(), P.db.size() * 8);
    put(P.o_dK, P.dK.data(), P.dK.size() * 8);
    put(P.o_repinst, P.rep_inst.data(), P.rep_inst.size() * 4);
    put(P.o_bp_sblk, P.bp_sblk.data(), P.bp_sblk.size() * 4);
    put(P.o_bp_eblk, P.bp_eblk.data(), P.bp_eblk.size() * 4);
    put(P.o_bp_wg, P.bp_wg.data(), P.bp_wg.size() * 4);
    put(P.o_oent, P.oent.data(), P.oent.size() * 2);
    put(P.o_ohinfo, P.ohinfo.data(), P.ohinfo.size());
    put(P.o_otbl, P.otbl.data(), P.otbl.size() * 4);
    put(P.o_otiles, P.otiles.data(), P.otiles.size() * 4);
    put(P.o_oqitems, P.oqitems.data(), P.oqitems.size() * 4);
    for (int n = 0; n < n_inst; ++n) {
        const InstDesc &d = P.desc[n];
        for (int r = 0; r < d.R; ++r) {
            ((int32_t *)(img.data() + P.o_rung))[d.rep_base + r] = r;
            ((int32_t *)(img.data() + P.o_repof))[d.rep_base + r] = r;
            ((int32_t *)(img.data() + P.o_label))[d.rep_base + r] = (r == 0) ? PT_LABEL_UP : PT_LABEL_NONE;
        }
    }
    e = hipMemcpyAsync(c->ws, img.data(), P.total_bytes, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return cleanup(hip_fail(e, "upload"));
    if (P.encoding == PT_BITPACK32) {
        e = launch_bp_init(st, P.bp_n_eblk, c->key_flip0, c->key_flip1 ^ kDomainInit, c->stream);
        if (e != hipSuccess) return cleanup(hip_fail(e, "init launch"));
    } else {
        e = launch_init_spins(st, (int)P.total_reps, c->key_flip0,
                              c->key_flip1 ^ kDomainInit, c->stream);
        if (e != hipSuccess) return cleanup(hip_fail(e, "init launch"));
    }
    e = energies_from_spins(c, 0, (int)P.total_reps);
    if (e != hipSuccess) return cleanup(hip_fail(e, "energy launch"));
    c->block_threads = opt->block_threads > 0 ? opt->block_threads : 1024;
    if (P.encoding == PT_INT8) {
        rc = build_tiles(c, opt->tile_replicas, opt->tile_bytes);
        if (rc) return cleanup(rc);
    } else {
        if (P.otile_lds > c->lds_limit || P.oblock_lds > c->lds_limit ||
            P.oblock_res_lds > c->lds_limit)
            return cleanup(fail(PT_EINVAL, "octet work needs more LDS than the device has"));
        e = oct_kernels_set_lds(P.otile_lds, P.oblock_lds, P.oblock_res_lds);
        if (e != hipSuccess) return cleanup(hip_fail(e, "octet kernel LDS attribute"));
        // whole octets in list order (or from the device work queues), and the exchange step
        // in the octet that completes an instance when every instance is in whole octets
        c->oct_queue = P.n_otile > 0 && (opt->flags & PT_FLAG_WORK_QUEUE);
        c->oct_fuse = P.n_otile > 0 && P.n_oblock == 0 && !P.bp_generic;
        if (c->oct_fuse) {
            c->itiles.assign(P.desc.size(), 0);
            for (int32_t k = 0; k < P.n_otile; ++k) c->itiles[P.otiles[(size_t)k * kOctRec]] += 1;
            e = hipMemcpyAsync(c->ws + P.o_itiles, c->itiles.data(), c->itiles.size() * 4,
                               hipMemcpyHostToDevice, c->stream);
            if (e != hipSuccess) return cleanup(hip_fail(e, "octet counts upload"));
        }
        // octet slice blocks run resident (one launch per call) when every block fits the
        // compute units at once: blocks wait for their neighbours, which must all have started
        if (P.n_oblock > 0 && !(opt->flags & PT_FLAG_BLOCK_LAUNCH_PER_SWEEP)) {
            int32_t per_cu = 0;
            e = oct_resident_per_cu(P.oblock_threads, P.oblock_res_lds, &per_cu);
            if (e != hipSuccess) return cleanup(hip_fail(e, "octet occupancy query"));
            c->oct_resident = (int64_t)P.n_oblock <= (int64_t)per_cu * c->cus;
        }
    }
    if (P.encoding == PT_BITPACK32) {
        c->block_threads = opt->block_threads > 0 ? opt->block_threads : 256;
    }
    const bool tune_int8 = P.encoding == PT_INT8 && opt->tile_replicas == 0 &&
                           opt->tile_bytes == 0 && opt->block_threads == 0;
    // packed: the workgroup size of the whole-octet launch
    const bool tune_bp = P.encoding == PT_BITPACK32 && P.n_otile > 0 && opt->block_threads == 0;
    if (tune_int8 || tune_bp) {
        if (tune_int8) {
            for (int tb : {8 * 1024, 16 * 1024, 32 * 1024, 64 * 1024, 128 * 1024})
                for (int th : {256, 512, 1024}) c->cand.emplace_back(tb, th);
        } else {
            for (int th : {256, 512, 1024}) c->cand.emplace_back(0, th);
        }
        c->cand_ms.assign(c->cand.size(), 0.0);
        c->tuning = true;
        for (auto &ev : c->tune_ev) {
            e = hipEventCreate(&ev);
            if (e != hipSuccess) return cleanup(hip_fail(e, "hipEventCreate"));
        }
    }
    // a resident slice-block launch may give up a wait: keep a copy of the state to restore
    if (P.halo_words > 0 || P.n_oblock > 0) {
        e = hipMalloc((void **)&c->shadow, std::max<size_t>(P.state_bytes, 1));
        if (e != hipSuccess) {
            c->shadow = nullptr;
            return cleanup(hip_fail(e, "hipMalloc (state copy)"));
        }
        e = take_snapshot(c);
        if (e != hipSuccess) return cleanup(hip_fail(e, "state copy"));
    }
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return cleanup(hip_fail(e, "init synchronise"));
    *out = c;
    return PT_OK;
}

int pt_sweep(pt_ctx *c, int32_t n_sweeps)
{
    if (!c) return fail(PT_EINVAL, "null context");
    if (n_sweeps < 0) return fail(PT_EINVAL, "n_sweeps < 0");
    if (n_sweeps == 0) return PT_OK;
    journal_add(c, 0, n_sweeps);
    int rc = enqueue_sweep(c, n_sweeps, false);
    if (rc) return rc;
    hipError_t e = launch_advance(c->st, n_inst_of(c), (uint32_t)n_sweeps, c->stream);
    if (e != hipSuccess) return hip_fail(e, "advance launch");
    return PT_OK;
}

int pt_exchange(pt_ctx *c)
{
    if (!c) return fail(PT_EINVAL, "null context");
    journal_add(c, 1, 0);
    int rc = enqueue_exchange(c, 0);
    if (rc) return rc;
    return enqueue_tau_corr(c);
}

int pt_run(pt_ctx *c, int32_t n_cycles)
{
    if (!c) return fail(PT_EINVAL, "null context");
    if (n_cycles < 0) return fail(PT_EINVAL, "n_cycles < 0");
    if (n_cycles > 0) journal_add(c, 2, n_cycles);
    // Batches whose instances each fit one whole-replica tile run up to kLaunchCycles
    // cycles per launch, each workgroup doing its instance's exchange steps itself (no
    // launch per cycle, no graph).  Not with the correlations (a launch of their own per
    // exchange), while tuning, with a launch failure to inject, or under PT_FLAG_NO_GRAPH
    // (which asks for one set of launches per cycle).
    constexpr int kLaunchCycles = 1024;
    if (n_cycles > 1 && c->plan.encoding == PT_INT8 &&
        !(c->opt.flags & (PT_FLAG_TAU_CORR | PT_FLAG_NO_GRAPH)) && !c->tuning &&
        !c->inject_pending && whole_instance_tiles(c)) {
        const int k = c->opt.sweeps_per_exchange;
        while (n_cycles > 0) {
            const int m = std::min(n_cycles, kLaunchCycles);
            const int rc = enqueue_sweep_once(c, k, true, m);
            if (rc == kCycleByCycle) break;
            if (rc) return rc;
            n_cycles -= m;
        }
        if (n_cycles == 0) return PT_OK;
    }
    const bool eager = (c->opt.flags & (PT_FLAG_NO_GRAPH | PT_FLAG_TIMING)) != 0 ||
                       c->inject_pending || c->tuning;
    if (eager) {
        for (int i = 0; i < n_cycles; ++i) {
            int rc = enqueue_cycle(c);
            if (rc) return rc;
        }
        return PT_OK;
    }
    // replay a captured graph of G cycles; the remainder runs eagerly
    const int G = 16;
    int done = 0;
    if (n_cycles >= G) {
        if (!c->graph) {
            hipGraph_t g = nullptr;
            HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            int rc = PT_OK;
            for (int i = 0; i < G && rc == PT_OK; ++i) rc = enqueue_cycle(c);
            hipError_t e = hipStreamEndCapture(c->stream, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                c->graph = nullptr;
                return hip_fail(e, "hipGraphInstantiate");
            }
            c->graph_cycles = G;
        }
        for (; done + G <= n_cycles; done += G) HIP_TRY(hipGraphLaunch(c->graph, c->stream));
    }
    for (; done < n_cycles; ++done) {
        int rc = enqueue_cycle(c);
        if (rc) return rc;
    }
    return PT_OK;
}

}  // extern "C"

namespace {

// After a resident launch gave up a wait: restore the state of the last clean
// synchronisation, turn resident launches off (and drop the captured graph, which holds
// them), and replay the calls queued since; the result is the chain's state.
int recover(pt_ctx *c)
{
    HIP_TRY(hipMemcpyAsync(c->ws + c->plan.o_state, c->shadow, c->plan.state_bytes,
                           hipMemcpyDeviceToDevice, c->stream));
    c->resident_off = true;
    c->oct_resident = false;
    drop_graph(c);
    const auto calls = c->journal;
    c->replaying = true;
    int rc = PT_OK;
    for (const auto &op : calls) {
        rc = op.first == 0 ? pt_sweep(c, op.second) : op.first == 1 ? pt_exchange(c) : pt_run(c, op.second);
        if (rc) break;
    }
    if (rc == PT_OK) rc = sync_and_check(c);
    c->replaying = false;
    if (rc) return rc;
    c->recoveries += 1;
    HIP_TRY(take_snapshot(c));
    return PT_OK;
}

}  // namespace

extern "C" {

int pt_sync(pt_ctx *c)
{
    if (!c) return fail(PT_EINVAL, "null context");
    return sync_and_check(c);
}

int pt_observables(pt_ctx *c, int32_t inst, pt_obs *o)
{
    int rc = check_inst(c, inst);
    if (rc) return rc;
    if (!o) return fail(PT_EINVAL, "null output");
    const InstDesc &d = c->plan.desc[inst];
    const int R = d.R, b = d.rep_base, pb = d.pair_base;
    char *w = c->ws;
    const Plan &P = c->plan;
    auto get = [&](void *dst, size_t off, size_t bytes) -> int {
        if (!dst || !bytes) return PT_OK;
        HIP_TRY(hipMemcpyAsync(dst, w + off, bytes, hipMemcpyDeviceToHost, c->stream));
        return PT_OK;
    };
    std::vector<int32_t> label(R);
    Counters ctr{};
    if ((rc = get(o->E_cl, P.o_E + (size_t)b * 8, (size_t)R * 8))) return rc;
    if ((rc = get(o->C, P.o_C + (size_t)b * 8, (size_t)R * 8))) return rc;
    if ((rc = get(o->rung_of, P.o_rung + (size_t)b * 4, (size_t)R * 4))) return rc;
    if ((rc = get(o->replica_of, P.o_repof + (size_t)b * 4, (size_t)R * 4))) return rc;
    if ((rc = get(o->acc, P.o_acc + (size_t)pb * 8, (size_t)(R - 1) * 8))) return rc;
    if ((rc = get(o->att, P.o_att + (size_t)pb * 8, (size_t)(R - 1) * 8))) return rc;
    if ((rc = get(o->roundtrips, P.o_rt + (size_t)b * 8, (size_t)R * 8))) return rc;
    if ((rc = get(label.data(), P.o_label + (size_t)b * 4, (size_t)R * 4))) return rc;
    if ((rc = get(o->sumE, P.o_sumE + (size_t)b * 8, (size_t)R * 8))) return rc;
    if ((rc = get(o->sumC, P.o_sumC + (size_t)b * 8, (size_t)R * 8))) return rc;
    if ((rc = get(o->sumE2, P.o_sumE2 + (size_t)b * 8, (size_t)R * 8))) return rc;
    if ((rc = get(o->sumC2, P.o_sumC2 + (size_t)b * 8, (size_t)R * 8))) return rc;
    if ((rc = get(o->nup, P.o_nup + (size_t)b * 8, (size_t)R * 8))) return rc;
    if ((rc = get(o->ndown, P.o_ndown + (size_t)b * 8, (size_t)R * 8))) return rc;
    if ((rc = get(o->sumCt, P.o_sumCt + (size_t)b * PT_TAU_LAGS * 8, (size_t)R * PT_TAU_LAGS * 8)))
        return rc;
    if ((rc = get(&ctr, P.o_ctr + (size_t)inst * sizeof(Counters), sizeof(Counters)))) return rc;
    if ((rc = sync_and_check(c))) return rc;
    if (o->label)
        for (int r = 0; r < R; ++r) o->label[r] = (int8_t)label[r];
    o->t = ctr.t;
    o->e = ctr.e;
    o->n_acc = ctr.n_acc;
    return PT_OK;
}

// Device layout of one replica: bytes x = (s + 1)/2 ordered [p][i][m], slice k = 2m + p.
// Bit-packed encoding: words of an instance, and the word that holds slot r at (k, i).
static inline int64_t bp_words(const InstDesc &d)
{
    return (int64_t)d.bp_W * d.parities * d.N * d.bp_row;
}
static inline size_t bp_pos(const InstDesc &d, int r, int k, int i)
{
    const int p = (d.M >= 2) ? (k & 1) : 0;
    const int m = (d.M >= 2) ? (k >> 1) : 0;
    return (((size_t)(r / 32) * d.parities + p) * d.N + i) * d.bp_row + m;
}

static inline size_t spin_pos(const InstDesc &d, int k, int i)
{
    const int p = (d.M >= 2) ? (k & 1) : 0;
    const int m = (d.M >= 2) ? (k >> 1) : 0;
    return (size_t)p * d.N * d.Mh + (size_t)i * d.Mh + m;
}

int pt_get_spins(pt_ctx *c, int32_t inst, int8_t *out)
{
    int rc = check_inst(c, inst);
    if (rc) return rc;
    if (!out) return fail(PT_EINVAL, "null output");
    const InstDesc &d = c->plan.desc[inst];
    if (c->plan.encoding == PT_BITPACK32) {
        std::vector<uint32_t> wb((size_t)bp_words(d));
        HIP_TRY(hipMemcpyAsync(wb.data(), c->ws + c->plan.o_spins + d.spin_base, wb.size() * 4,
                               hipMemcpyDeviceToHost, c->stream));
        if ((rc = sync_and_check(c))) return rc;
        for (int r = 0; r < d.R; ++r)
            for (int k = 0; k < d.M; ++k)
                for (int i = 0; i < d.N; ++i)
                    out[((size_t)r * d.M + k) * d.N + i] =
                        (int8_t)(2 * (int)((wb[bp_pos(d, r, k, i)] >> (r & 31)) & 1u) - 1);
        return PT_OK;
    }
    std::vector<uint8_t> buf((size_t)d.R * d.rep_bytes);
    HIP_TRY(hipMemcpyAsync(buf.data(), c->ws + c->plan.o_spins + d.spin_base, buf.size(),
                           hipMemcpyDeviceToHost, c->stream));
    if ((rc = sync_and_check(c))) return rc;
    for (int r = 0; r < d.R; ++r)
        for (int k = 0; k < d.M; ++k)
            for (int i = 0; i < d.N; ++i)
                out[((size_t)r * d.M + k) * d.N + i] =
                    (int8_t)(2 * buf[(size_t)r * d.rep_bytes + spin_pos(d, k, i)] - 1);
    return PT_OK;
}

int pt_set_spins(pt_ctx *c, int32_t inst, const int8_t *in)
{
    int rc = check_inst(c, inst);
    if (rc) return rc;
    if (!in) return fail(PT_EINVAL, "null input");
    const InstDesc &d = c->plan.desc[inst];
    for (size_t x = 0; x < (size_t)d.R * d.M * d.N; ++x)
        if (in[x] != 1 && in[x] != -1) return fail(PT_EINVAL, "spins must be +1 or -1");
    if (c->plan.encoding == PT_BITPACK32) {
        std::vector<uint32_t> wb((size_t)bp_words(d), 0u);
        for (int r = 0; r < d.R; ++r)
            for (int k = 0; k < d.M; ++k)
                for (int i = 0; i < d.N; ++i)
                    if (in[((size_t)r * d.M + k) * d.N + i] == 1) wb[bp_pos(d, r, k, i)] |= 1u << (r & 31);
        HIP_TRY(hipMemcpyAsync(c->ws + c->plan.o_spins + d.spin_base, wb.data(), wb.size() * 4,
                               hipMemcpyHostToDevice, c->stream));
        // pageable source: the copy has been staged once the stream reaches this point
        HIP_TRY(hipStreamSynchronize(c->stream));
    } else {
        std::vector<uint8_t> buf((size_t)d.R * d.rep_bytes, 0);
        for (int r = 0; r < d.R; ++r)
            for (int k = 0; k < d.M; ++k)
                for (int i = 0; i < d.N; ++i)
                    buf[(size_t)r * d.rep_bytes + spin_pos(d, k, i)] =
                        (uint8_t)((in[((size_t)r * d.M + k) * d.N + i] + 1) / 2);
        HIP_TRY(hipMemcpyAsync(c->ws + c->plan.o_spins + d.spin_base, buf.data(), buf.size(),
                               hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    hipError_t e = energies_from_spins(c, d.rep_base, d.R);
    if (e != hipSuccess) return hip_fail(e, "energy launch");
    HIP_TRY(take_snapshot(c));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return PT_OK;
}

int pt_save(pt_ctx *c, void *buf, size_t *len)
{
    if (!c || !len) return fail(PT_EINVAL, "null argument");
    const size_t need = sizeof(CkptHeader) + c->plan.state_bytes;
    if (!buf) {
        *len = need;
        return PT_OK;
    }
    if (*len < need) return fail(PT_EINVAL, "checkpoint buffer too small");
    CkptHeader h{kMagic, kVersion, c->plan.state_bytes, c->opt.seed, n_inst_of(c),
                 c->opt.encoding, c->plan.flips_per_sweep};
    std::memcpy(buf, &h, sizeof h);
    HIP_TRY(hipMemcpyAsync((char *)buf + sizeof h, c->ws + c->plan.o_state, c->plan.state_bytes,
                           hipMemcpyDeviceToHost, c->stream));
    const int rc = sync_and_check(c);
    if (rc) return rc;
    *len = need;
    return PT_OK;
}

int pt_load(pt_ctx *c, const void *buf, size_t len)
{
    if (!c || !buf) return fail(PT_EINVAL, "null argument");
    const int rc = check_checkpoint(c->plan, c->opt, n_inst_of(c), buf, len);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(c->ws + c->plan.o_state, (const char *)buf + sizeof(CkptHeader),
                           c->plan.state_bytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(take_snapshot(c));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return PT_OK;
}

int pt_checkpoint_validate(const pt_instance *inst, int32_t n_inst, const pt_options *opt,
                           const void *buf, size_t len, size_t *need)
{
    if (!opt) return fail(PT_EINVAL, "null options");
    Plan P;
    int rc = make_plan(inst, n_inst, opt->flags, opt->encoding, P);
    if (rc) return rc;
    if (need) *need = sizeof(CkptHeader) + P.state_bytes;
    if (!buf) return PT_OK;
    return check_checkpoint(P, *opt, n_inst, buf, len);
}

int pt_get_info(pt_ctx *c, pt_info *o)
{
    if (!c || !o) return fail(PT_EINVAL, "null argument");
    int rc = harvest_events(c);
    if (rc) return rc;
    o->n_instances = n_inst_of(c);
    o->n_tiles = (int)c->tiles.size();
    o->block_threads = c->block_threads;
    o->lds_bytes = std::max(c->lds_fast, std::max(c->lds_generic, c->lds_block));
    o->max_tile_replicas = c->max_P;
    o->fallbacks = c->fallbacks;
    o->encoding = c->opt.encoding;
    o->device_cus = c->cus;
    o->tile_bytes = c->tile_bytes;
    o->tuned = c->tuning ? 0 : 1;
    o->flips_per_sweep = c->plan.flips_per_sweep;
    o->sweep_ms = c->sweep_ms;
    o->sweep_launches = c->sweep_n;
    o->exchange_ms = c->exch_ms;
    o->exchange_launches = c->exch_n;
    o->sweep_groups = (int32_t)launch_groups(c).size();
    o->block_tiles = c->n_block_tiles;
    o->block_resident = c->block_persistent;
    o->class_launches = 0;
    o->oct_tiles = c->plan.n_otile;
    o->oct_blocks = c->plan.n_oblock;
    o->oct_tile_launches = c->plan.n_otile > 0 ? 1 : 0;
    o->oct_resident = c->oct_resident ? 1 : 0;
    o->oct_queue = c->oct_queue ? 1 : 0;
    o->oct_fused = c->oct_fuse ? 1 : 0;
    o->oct_ring_xcd = oct_ring_xcd(c) ? 1 : 0;
    o->block_ring_xcd = block_ring_xcd(c) ? 1 : 0;
    o->recoveries = c->recoveries;
    o->last_device_error = c->last_device_error;
    o->lane_words = c->lane_words;
    o->latency_path = latency_path(c, c->block_threads) ? 1 : 0;
    o->ent16_instances = 0;
    for (const auto &d : c->plan.desc) o->ent16_instances += (d.fast && d.ent_mode == kEntXad16) ? 1 : 0;
    if (c->plan.encoding == PT_BITPACK32 && c->plan.bp_generic) {
        int parities = 1;
        for (const auto &d : c->plan.desc) parities = std::max(parities, d.parities);
        o->class_launches = parities * (int32_t)c->plan.bp_colour.size();
    }
    o->multi_launches = c->multi_launches;
    o->multi_cycles = c->multi_cycles;
    o->multi_ms = c->multi_ms;
    return PT_OK;
}

int pt_timing_enable(pt_ctx *c, int32_t on)
{
    if (!c) return fail(PT_EINVAL, "null context");
    int rc = harvest_events(c);
    if (rc) return rc;
    if (on)
        c->opt.flags |= PT_FLAG_TIMING;
    else
        c->opt.flags &= ~PT_FLAG_TIMING;
    return PT_OK;
}

int pt_timing_reset(pt_ctx *c)
{
    if (!c) return fail(PT_EINVAL, "null context");
    int rc = harvest_events(c);
    if (rc) return rc;
    c->sweep_ms = c->exch_ms = c->multi_ms = 0;
    c->sweep_n = c->exch_n = 0;
    return PT_OK;
}

void pt_free(pt_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_graph(c);
    if (c->shadow) (void)hipFree(c->shadow);
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    for (auto e : c->tune_ev)
        if (e) (void)hipEventDestroy(e);
    if (c->own_ws && c->ws) (void)hipFree(c->ws);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char *pt_strerror(int code)
{
    switch (code) {
    case PT_OK: return "ok";
    case PT_EINVAL: return "invalid argument";
    case PT_ENOMEM: return "out of memory";
    case PT_EHIP: return "HIP runtime error";
    case PT_ELAUNCH: return "kernel launch failed in every configuration";
    case PT_ESTATE: return "invalid state";
    default: return "unknown error";
    }
}

const char *pt_last_error(void) { return g_last_error.c_str(); }

uint32_t pt_threshold(double dS) { return threshold(dS); }

int pt_threshold_device(const double *dS, uint32_t *out, int32_t n, void *stream)
{
    if (n < 0 || (n > 0 && (!dS || !out))) return fail(PT_EINVAL, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_threshold_eval(dS, out, n, s);
    if (e != hipSuccess) return hip_fail(e, "threshold launch");
    HIP_TRY(hipStreamSynchronize(s));
    return PT_OK;
}

}  // extern "C"
