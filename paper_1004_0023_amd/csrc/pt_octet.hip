// pt_octet.hip -- octet kernels of the bit-packed spin encoding (PT_BITPACK32).
//
// In device memory a 32-bit word holds one spin of 32 replica slots (bit c mod 32 of word
// group c / 32).  These kernels work on octets: byte o of every word of word group w, the
// eight slots 32 w + 8 o .. 32 w + 8 o + 7.  A workgroup stages its octet's bytes into LDS
// (one LDS word = the eight slots at four same-parity slices of one site) and writes only
// those bytes back, so the workgroups of the four octets of a word never write the same
// byte.  The chain is the one every encoding runs: the same colour classes, Philox words
// and thresholds.
//
// The local field is bit-sliced.  For instances whose couplings are all +-1 and fields
// in {-1, 0, 1}, with every site of one degree D <= 8, a site's Metropolis move depends on
// n, the number of its inputs (D couplings and, when h != 0, the field) that agree with its
// spin (a = s f = 2 n - D - [h != 0]), and on sigma, the number of agreeing time
// neighbours.  For one LDS word each input gives a word of agreement bits (one three-input
// operation), a carry-save adder tree turns D + 1 of them into the four bit planes of n
// for all 32 (slot, slice) pairs at once, and two operations give sigma's planes.  Per slot
// the planes' bits are gathered into a word of four table byte offsets, one per slice;
// each attempt then takes its threshold with one v_perm (the byte joined to its table's
// base) and one LDS read, as in the byte encoding.
//
//   oct_tile   whole octets resident in LDS for all sweeps of a call (octets of at most
//              half a compute unit's LDS), then their E_cl and C
//   oct_phase  octet slice blocks: one launch per parity of every sweep, staging ng
//              four-slice groups of the parity swept and ng + 1 of the other; the last
//              launch of a call adds each block's part of E_cl and C
//   oct_clear  E_cl and C of the slice-block octets set to zero before a call
#include "pt_exchange.h"
#include "pt_xcd.h"
#include "pt_internal.h"

#pragma clang fp contract(off)

namespace ptq {
namespace {

constexpr int kWave = 64;

template <int V>
struct IC {
    static constexpr int value = V;
};

// LDS words and halfwords by byte address.  These kernels use dynamic LDS only, which
// starts at address 0 (each kernel checks this on entry), so a layout offset is an LDS
// address and a computed address needs no base added (a table address comes straight out
// of one v_perm).
typedef __attribute__((address_space(3))) uint32_t LdsU32;
typedef __attribute__((address_space(3))) uint16_t LdsU16;
typedef __attribute__((address_space(3))) uint8_t LdsU8;
__device__ __forceinline__ uint32_t ld32(uint32_t a) { return *(const LdsU32 *)(uintptr_t)a; }
__device__ __forceinline__ void st32(uint32_t a, uint32_t v) { *(LdsU32 *)(uintptr_t)a = v; }
__device__ __forceinline__ uint32_t ld16(uint32_t a) { return *(const LdsU16 *)(uintptr_t)a; }
__device__ __forceinline__ uint32_t ld8(uint32_t a) { return *(const LdsU8 *)(uintptr_t)a; }

// s_waitcnt immediate with the vector-memory count 0 and the export and LDS counts at
// their maxima (no wait on them): vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8.
constexpr int kOctWaitVmcnt0 = 0x0F70;

// Philox4x32-10 (the sampler's generator) with each round key formed in its round: left to
// itself the compiler keeps all twenty live in scalar registers across the sweep loops.
__device__ __forceinline__ Words4 philox10_rk(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        __asm__ volatile("" : "+s"(k0), "+s"(k1));
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

// Byte o of each of the four words of v as one word (byte b from word b); sel = (4 + o) << 8
// | o with zero upper bytes.
__device__ __forceinline__ uint32_t octet_of(const uint4 &v, uint32_t sel)
{
    const uint32_t lo = __builtin_amdgcn_perm(v.y, v.x, sel);
    const uint32_t hi = __builtin_amdgcn_perm(v.w, v.z, sel);
    return __builtin_amdgcn_perm(hi, lo, 0x05040100u);
}

__device__ __forceinline__ uint32_t xor3w(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t maj3w(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
}
// ~(a ^ b ^ c): with c = 0 for J > 0 and ~0 for J < 0 the bits where J s_i s_j > 0
__device__ __forceinline__ uint32_t xnor3w(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x69);
}

// Bit planes of the number of set bits among v[0..8] at every bit position: a carry-save
// adder tree (five full adders, two half adders); absent inputs are zero and fold away.
__device__ __forceinline__ void count9(const uint32_t (&v)[9], uint32_t &n0, uint32_t &n1,
                                       uint32_t &n2, uint32_t &n3)
{
    const uint32_t h1 = maj3w(v[0], v[1], v[2]);
    const uint32_t o1 = xor3w(v[0], v[1], v[2]);
    const uint32_t h2 = maj3w(o1, v[3], v[4]);
    const uint32_t o2 = xor3w(o1, v[3], v[4]);
    const uint32_t t = h1 ^ h2, fa = h1 & h2;
    const uint32_t h3 = maj3w(o2, v[5], v[6]);
    const uint32_t o3 = xor3w(o2, v[5], v[6]);
    const uint32_t h4 = maj3w(o3, v[7], v[8]);
    n0 = xor3w(o3, v[7], v[8]);
    n1 = xor3w(t, h3, h4);
    const uint32_t fb = maj3w(t, h3, h4);
    n2 = fa ^ fb;
    n3 = fa & fb;
}

// Rows a and b of a bit matrix exchange the bits where (a >> sh) and b differ under mask m
// (one step of a bit-matrix transpose).
__device__ __forceinline__ void delta_swap(uint32_t &a, uint32_t &b, int sh, uint32_t m)
{
    const uint32_t t = ((a >> sh) ^ b) & m;
    b ^= t;
    a ^= t << sh;
}

// Table byte offsets 4 (n + 16 sigma) of the four slices of each of the lane's SPL slots:
// byte b of w[r] takes bit 8 b + r of n0 .. n3, s0, s1 at bits 2 .. 7.  In every byte lane
// this is the transpose of the 8 x 8 bit matrix with rows (0, 0, n0, n1, n2, n3, s0, s1);
// with four slots per lane only the first four rows of the result are formed.
template <int SPL>
__device__ __forceinline__ void slot_offsets(uint32_t n0, uint32_t n1, uint32_t n2, uint32_t n3,
                                             uint32_t s0, uint32_t s1, uint32_t (&w)[SPL])
{
    uint32_t a[8] = {0u, 0u, n0, n1, n2, n3, s0, s1};
    if constexpr (SPL == 8) {
#pragma unroll
        for (int i = 0; i < 4; ++i) delta_swap(a[i], a[i + 4], 4, 0x0F0F0F0Fu);
#pragma unroll
        for (int i : {0, 1, 4, 5}) delta_swap(a[i], a[i + 2], 2, 0x33333333u);
#pragma unroll
        for (int i : {0, 2, 4, 6}) delta_swap(a[i], a[i + 1], 1, 0x55555555u);
    } else {
        // rows 0 .. 3 after the first step: their low nibbles, and the low nibbles of rows
        // 4 .. 7 as high nibbles
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = (a[i] & 0x0F0F0F0Fu) | ((a[i + 4] << 4) & 0xF0F0F0F0u);
        delta_swap(a[0], a[2], 2, 0x33333333u);
        delta_swap(a[1], a[3], 2, 0x33333333u);
        delta_swap(a[0], a[1], 1, 0x55555555u);
        delta_swap(a[2], a[3], 1, 0x55555555u);
    }
#pragma unroll
    for (int r = 0; r < SPL; ++r) w[r] = a[r];
}

// The per-item constants of a site.
struct OctSite {
    uint32_t hneg;   // ~0 when h < 0
    uint32_t hzm;    // ~0 when h != 0
    uint32_t hzbase; // LDS byte address of the slot-0 table half for [h != 0] (low byte 0)
};

// New octet word of one site at four same-parity slices: X its word, Tlo / Thi the words of
// its time neighbours below and above (byte b = slice 4 g + b), Y / nm the words and sign
// masks of its D neighbours.  ctr0: Philox counter word 0 of (site, parity, global group);
// slot 8 o + r of word group w is replica cbase + r.  A lane takes SPL of the eight slots,
// those from SPL * half on; with SPL = 4 the two lanes of an item are neighbours and join
// their flips with one lane exchange (both must call).  MASK = false: slots is the number of
// the lane's slots in use, nslots - SPL * half (at most SPL counts), and each slot is
// tested against it.  MASK = true: every slot is drawn and
// looked up (the tables of all eight slots lie in LDS) and slots is the lane's flip mask
// (oct_slot_mask), which clears the flips of slots beyond the count: no per-slot test, more
// registers live.
template <int DT, int SPL, bool MASK>
__device__ __forceinline__ uint32_t oct_update(uint32_t X, uint32_t Tlo,
                                               uint32_t Thi, const uint32_t (&Y)[DT],
                                               const uint32_t (&nm)[DT], const OctSite &site,
                                               uint32_t ctr0, uint32_t tt, uint32_t cbase,
                                               uint32_t n, uint32_t key0, uint32_t key1,
                                               uint32_t slots, int half)
{
    uint32_t v[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) v[e] = 0u;
#pragma unroll
    for (int e = 0; e < DT; ++e) v[e] = xnor3w(X, Y[e], nm[e]);
    v[DT] = (X ^ site.hneg) & site.hzm;  // the field: agrees when h s > 0
    uint32_t n0, n1, n2, n3;
    count9(v, n0, n1, n2, n3);
    uint32_t s0 = Tlo ^ Thi;                                   // sigma bit 0
    uint32_t s1 = __builtin_amdgcn_bitop3_b32(X, Tlo, Thi, 0x81);  // sigma bit 1
    // this lane's slots to bit positions 0 .. SPL - 1 of every byte
    const int sh = SPL * half;
    n0 >>= sh;
    n1 >>= sh;
    n2 >>= sh;
    n3 >>= sh;
    s0 >>= sh;
    s1 >>= sh;
    const uint32_t tbase = site.hzbase + 512u * (uint32_t)sh;
    uint32_t offs[SPL];
    slot_offsets<SPL>(n0, n1, n2, n3, s0, s1, offs);
    uint32_t flip = 0u;
#pragma unroll
    for (int r = 0; r < SPL; ++r) {
        if (MASK || r < (int)slots) {
            const uint32_t idx = offs[r];  // table byte offsets of slot sh + r's four slices
            const Words4 u = philox10_rk(ctr0, tt, cbase + (uint32_t)(sh + r), n, key0, key1);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const uint32_t addr = __builtin_amdgcn_perm(tbase, idx, 0x0C060500u | (uint32_t)b);
                const uint32_t thr = ld32(addr + 512u * (uint32_t)r);
                flip |= (u.w[b] <= thr ? 1u : 0u) << (8 * b + r);
            }
        }
    }
    if constexpr (MASK) flip &= slots;
    flip <<= sh;
    if constexpr (SPL < 8) flip |= (uint32_t)__shfl_xor((int)flip, 1, kWave);
    return X ^ flip;
}

// The flip mask of oct_update for a lane of the given half: in every byte, the bits of the
// lane's SPL slots that are among the octet's nslots in use.
template <int SPL>
__device__ __forceinline__ uint32_t oct_slot_mask(int nslots, int half)
{
    const int nv = min(max(nslots - SPL * half, 0), SPL);
    return 0x01010101u * ((1u << nv) - 1u);
}

// count elements through load(k) -> store(k, value) with up to four loads in flight per
// thread: indices past the end are clamped so that every load is unconditional (a load
// under a branch would be waited for where the branch ends).  count >= 1.
template <int K = 4, class Load, class Store>
__device__ __forceinline__ void batched(int count, Load &&load, Store &&store)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int base = tid; base < count; base += K * nt) {
        decltype(load(0)) v[K];
#pragma unroll
        for (int u = 0; u < K; ++u) v[u] = load(min(base + u * nt, count - 1));
#pragma unroll
        for (int u = 0; u < K; ++u)
            if (base + u * nt < count) store(base + u * nt, v[u]);
    }
}

// LDS layout of an octet work item.  Whole octets: sp holds [p][i][g] words (two parities,
// G4 groups, N * M bytes).  Phase slice blocks: sp holds [i][gl] words of the parity swept
// (ng groups), oth [i][x] words of the other parity (ng + 1 groups).  Resident slice
// blocks: sp and oth hold [i][x] words of parities 0 and 1 (ng + 1 groups each).  Then the eight slots'
// tables (256-byte aligned, 512 bytes each), the 16-bit neighbour entries, field codes,
// colour lists and a reduction area of 16 int64.
struct OctLds {
    uint32_t sp, oth, tbl, ent, hinfo, csite, coff, red, end;
};

__host__ __device__ __forceinline__ uint32_t a16u(uint32_t x) { return (x + 15u) & ~15u; }
__host__ __device__ __forceinline__ uint32_t a256u(uint32_t x) { return (x + 255u) & ~255u; }

__host__ __device__ __forceinline__ OctLds oct_layout(const InstDesc &d, int ng, int mode)
{
    OctLds o;
    const uint32_t N = (uint32_t)d.N;
    o.sp = 0;
    if (mode == kOctTile) {
        o.oth = 0;
        o.tbl = a256u(2u * N * (uint32_t)d.G4 * 4u);
    } else {
        // phase: own rows of ng words; resident: P0 rows of ng + 1 words
        o.oth = a16u(N * (uint32_t)(mode == kOctPhase ? ng : ng + 1) * 4u);
        o.tbl = a256u(o.oth + N * (uint32_t)(ng + 1) * 4u);
    }
    o.ent = o.tbl + 8u * 512u;
    o.hinfo = a16u(o.ent + N * (uint32_t)d.D * 2u);
    o.csite = a16u(o.hinfo + N);
    o.coff = a16u(o.csite + N * 2u);
    o.red = a16u(o.coff + (uint32_t)(d.n_colors + 1) * 4u);
    o.end = a16u(o.red + 16u * 8u);
    return o;
}

// Stage the tables of the eight slots (by their current rungs), the neighbour entries,
// field codes and colour lists.  Entries and field codes are padded to 16 bytes per
// instance in device memory, so they move as 16-byte pieces.
__device__ __forceinline__ void oct_stage_common(const DevState &st, const InstDesc &d, char *lds,
                                                 const OctLds &o, int c0, int nslots)
{
    const int tid = threadIdx.x;
    uint4 *tb = reinterpret_cast<uint4 *>(lds + o.tbl);
    constexpr int kQ = kOctTableWords / 4;  // 16-byte pieces per table
    batched<2>(nslots * kQ,
            [&](int k) {
                const int r = k / kQ, e = k - r * kQ;
                const int rg = st.rung_of[d.rep_base + c0 + r];
                return reinterpret_cast<const uint4 *>(st.otbl + d.otbl_base + (int64_t)rg * kOctTableWords)[e];
            },
            [&](int k, uint4 v) { tb[k] = v; });
    const uint4 *es = reinterpret_cast<const uint4 *>(st.oent + d.oent_base);
    uint4 *ed = reinterpret_cast<uint4 *>(lds + o.ent);
    batched<2>((d.N * d.D + 7) / 8, [&](int k) { return es[k]; }, [&](int k, uint4 v) { ed[k] = v; });
    const uint4 *hs = reinterpret_cast<const uint4 *>(st.ohinfo + d.opad);
    uint4 *hd = reinterpret_cast<uint4 *>(lds + o.hinfo);
    batched<2>((d.N + 15) / 16, [&](int k) { return hs[k]; }, [&](int k, uint4 v) { hd[k] = v; });
    uint16_t *cs = reinterpret_cast<uint16_t *>(lds + o.csite);
    const uint16_t *css = st.csite + d.site_base;
    batched(d.N, [&](int k) { return css[k]; }, [&](int k, uint16_t v) { cs[k] = v; });
    int32_t *co = reinterpret_cast<int32_t *>(lds + o.coff);
    for (int g = tid; g <= d.n_colors; g += blockDim.x) co[g] = st.cls_off[d.cls_base + g];
    int64_t *red = reinterpret_cast<int64_t *>(lds + o.red);
    if (tid < 16) red[tid] = 0;
}

__device__ __forceinline__ OctSite oct_site(const OctLds &o, int i)
{
    const uint32_t hb = ld8(o.hinfo + (uint32_t)i);
    OctSite s;
    s.hneg = (hb & 1u) ? 0xFFFFFFFFu : 0u;
    s.hzm = (hb & 2u) ? 0xFFFFFFFFu : 0u;
    s.hzbase = o.tbl + ((hb & 2u) ? 256u : 0u);
    return s;
}

// Neighbour e of site i: its site index and sign mask (~0 when J < 0).
__device__ __forceinline__ void oct_entry(const OctLds &o, int idx, uint32_t &j,
                                          uint32_t &nm)
{
    const uint32_t v = ld16(o.ent + 2u * (uint32_t)idx);
    j = v & 0x7FFFu;
    nm = (uint32_t)((int32_t)(v << 16) >> 31);
}

// Per-slot sums of 2 E_cl and C over one (site, four-slice group) position: X0, X1 the
// site's words of parities 0 and 1, X0n its parity-0 word of the next group, Y0 / Y1 its
// neighbours' words, h its field.
template <int DT>
__device__ __forceinline__ void oct_energy_item(uint32_t X0, uint32_t X1, uint32_t X0n,
                                                const uint32_t (&Y0)[DT], const uint32_t (&Y1)[DT],
                                                const uint32_t (&nm)[DT], int h, int (&e2)[8],
                                                int (&cc)[8])
{
    uint32_t A0[DT], A1[DT];
#pragma unroll
    for (int e = 0; e < DT; ++e) {
        A0[e] = xnor3w(X0, Y0[e], nm[e]);
        A1[e] = xnor3w(X1, Y1[e], nm[e]);
    }
    const uint32_t d1 = X0 ^ X1;                                        // bonds (2m, 2m+1)
    const uint32_t d2 = X1 ^ __builtin_amdgcn_alignbyte(X0n, X0, 1);    // bonds (2m+1, 2m+2)
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const uint32_t m = 0x01010101u << r;
        int agree = 0;
#pragma unroll
        for (int e = 0; e < DT; ++e) agree += __popc(A0[e] & m) + __popc(A1[e] & m);
        const int up = __popc(X0 & m) + __popc(X1 & m);
        e2[r] += 2 * agree - 8 * DT + 2 * h * (2 * up - 8);
        cc[r] += 8 - 2 * (__popc(d1 & m) + __popc(d2 & m));
    }
}

// Wave sums of the per-slot partials added into the block's LDS reduction area.
__device__ __forceinline__ void oct_reduce(char *lds, const OctLds &o, const int (&e2)[8],
                                           const int (&cc)[8])
{
    int64_t *red = reinterpret_cast<int64_t *>(lds + o.red);
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        int a = e2[r], b = cc[r];
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
            a += __shfl_xor(a, off, kWave);
            b += __shfl_xor(b, off, kWave);
        }
        if (lane == 0) {
            atomicAdd(reinterpret_cast<unsigned long long *>(&red[r]), (unsigned long long)(int64_t)a);
            atomicAdd(reinterpret_cast<unsigned long long *>(&red[8 + r]), (unsigned long long)(int64_t)b);
        }
    }
}

// Spin words of the instance's word group w, parity p, site i (4 G4 words per row).
__device__ __forceinline__ uint32_t *oct_row(const DevState &st, const InstDesc &d, int w, int p, int i)
{
    return reinterpret_cast<uint32_t *>(st.spins + d.spin_base) +
           ((int64_t)(w * d.parities + p) * d.N + i) * d.bp_row;
}

// The octet's byte of the four words of group g in a row.
__device__ __forceinline__ uint32_t oct_load(const uint32_t *row, int g, uint32_t sel)
{
    return octet_of(*reinterpret_cast<const uint4 *>(row + 4 * g), sel);
}
__device__ __forceinline__ void oct_store(uint32_t *row, int g, int o, uint32_t v)
{
    uint8_t *p = reinterpret_cast<uint8_t *>(row + 4 * g) + o;
    p[0] = (uint8_t)v;
    p[4] = (uint8_t)(v >> 8);
    p[8] = (uint8_t)(v >> 16);
    p[12] = (uint8_t)(v >> 24);
}

// The degree switch and the slots-per-lane choice around a work item's body.
template <class Body>
__device__ __forceinline__ void oct_dispatch(int D, bool split, Body &&body)
{
    auto go = [&](auto spl) {
        switch (D) {
        case 1: body(IC<1>{}, spl); break;
        case 2: body(IC<2>{}, spl); break;
        case 3: body(IC<3>{}, spl); break;
        case 4: body(IC<4>{}, spl); break;
        case 5: body(IC<5>{}, spl); break;
        case 6: body(IC<6>{}, spl); break;
        case 7: body(IC<7>{}, spl); break;
        default: body(IC<8>{}, spl); break;
        }
    };
    if (split)
        go(IC<4>{});
    else
        go(IC<8>{});
}

// ------------------------------------------------------------------ whole octets

// All sweeps of a call over a whole octet.  SPL: slots per lane (8, or 4 with two lanes per
// item when the largest colour class has at most half a workgroup of items).
template <int DT, int SPL>
__device__ __forceinline__ void oct_tile_sweeps(const OctLaunch &L, const InstDesc &d, const OctLds &o,
                                                int n, int c0, int nslots, uint64_t t0)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int N = d.N, G4 = d.G4, lgG4 = 31 - __clz(G4);
    constexpr int lgL = SPL == 8 ? 0 : 1;  // lanes per item
    // items come in lane pairs and the block size is even, so a thread keeps its half
    const int half = tid & ((1 << lgL) - 1);
    const uint32_t nv = (uint32_t)(nslots - SPL * half);  // this lane's slots in use (signed)
    const uint32_t plane = (uint32_t)N * (uint32_t)G4 * 4u;
    const int nc = d.n_colors;
    if (nc >= 2) {
        // Class k of parity 0 and class k - 1 of parity 1 (mod nc; of the previous sweep
        // when k = 0) touch disjoint words: each writes its own sites' words of its parity
        // and reads the other parity only at those sites.  So they run as one step, every
        // update reading what it reads in the plain order, and a sweep is nc steps.
        int sw = 0, k = 0;
        for (int step = 0; step <= nc * L.n_sweeps; ++step) {
            const int kB = (k == 0 ? nc : k) - 1, swB = sw - (k == 0 ? 1 : 0);
            const int a0 = (int)ld32(o.coff + 4u * (uint32_t)k);
            const int b0 = (int)ld32(o.coff + 4u * (uint32_t)kB);
            const int itemsA = sw < L.n_sweeps
                                   ? ((int)ld32(o.coff + 4u * (uint32_t)(k + 1)) - a0) << (lgG4 + lgL)
                                   : 0;
            const int itemsB = swB >= 0 && swB < L.n_sweeps
                                   ? ((int)ld32(o.coff + 4u * (uint32_t)(kB + 1)) - b0) << (lgG4 + lgL)
                                   : 0;
            for (int it = tid; it < itemsA + itemsB; it += nt) {
                const bool inA = it < itemsA;
                const int p = inA ? 0 : 1;
                const int jt = inA ? it : it - itemsA;
                const uint32_t tt = (uint32_t)(t0 + (uint64_t)(inA ? sw : swB));
                const uint32_t pb = inA ? 0u : plane, ob = inA ? plane : 0u;
                const int gg = (jt >> lgL) & (G4 - 1);
                const int i = (int)ld16(o.csite + 2u * (uint32_t)((inA ? a0 : b0) + (jt >> (lgG4 + lgL))));
                const uint32_t rowi = (uint32_t)(i << lgG4) * 4u;
                const uint32_t X = ld32(pb + rowi + 4u * (uint32_t)gg);
                const uint32_t Wc = ld32(ob + rowi + 4u * (uint32_t)gg);
                // the other parity's word before the item's (parity 0) or after it (parity 1)
                const uint32_t Wx = ld32(ob + rowi + 4u * (uint32_t)((gg + (inA ? -1 : 1)) & (G4 - 1)));
                const uint32_t Tlo = inA ? __builtin_amdgcn_alignbyte(Wc, Wx, 3) : Wc;
                const uint32_t Thi = inA ? Wc : __builtin_amdgcn_alignbyte(Wx, Wc, 1);
                uint32_t Y[DT], nm[DT];
#pragma unroll
                for (int e = 0; e < DT; ++e) {
                    uint32_t j;
                    oct_entry(o, i * DT + e, j, nm[e]);
                    Y[e] = ld32(pb + ((j << lgG4) + (uint32_t)gg) * 4u);
                }
                const OctSite site = oct_site(o, i);
                const uint32_t ctr0 = (uint32_t)(2 * i + p) * (uint32_t)G4 + (uint32_t)gg;
                const uint32_t nx = oct_update<DT, SPL, false>(X, Tlo, Thi, Y, nm, site, ctr0, tt,
                                                               (uint32_t)c0, (uint32_t)n, L.key0,
                                                               L.key1, nv, half);
                if (half == 0) st32(pb + rowi + 4u * (uint32_t)gg, nx);
            }
            __syncthreads();
            if (++k == nc) {
                k = 0;
                ++sw;
            }
        }
        return;
    }
    for (int sw = 0; sw < L.n_sweeps; ++sw) {
        const uint32_t tt = (uint32_t)(t0 + (uint64_t)sw);
        for (int p = 0; p < 2; ++p) {
            const uint32_t pb = (uint32_t)p * plane, ob = (uint32_t)(p ^ 1) * plane;
            for (int g = 0; g < d.n_colors; ++g) {
                const int s0 = (int)ld32(o.coff + 4u * (uint32_t)g);
                const int items = ((int)ld32(o.coff + 4u * (uint32_t)(g + 1)) - s0) << (lgG4 + lgL);
                for (int it = tid; it < items; it += nt) {
                    const int gg = (it >> lgL) & (G4 - 1);
                    const int i = (int)ld16(o.csite + 2u * (uint32_t)(s0 + (it >> (lgG4 + lgL))));
                    const uint32_t rowi = (uint32_t)(i << lgG4) * 4u;
                    const uint32_t X = ld32(pb + rowi + 4u * (uint32_t)gg);
                    const uint32_t Wc = ld32(ob + rowi + 4u * (uint32_t)gg);
                    uint32_t Tlo, Thi;
                    if (p == 0) {
                        Tlo = __builtin_amdgcn_alignbyte(Wc, ld32(ob + rowi + 4u * (uint32_t)((gg - 1) & (G4 - 1))), 3);
                        Thi = Wc;
                    } else {
                        Tlo = Wc;
                        Thi = __builtin_amdgcn_alignbyte(ld32(ob + rowi + 4u * (uint32_t)((gg + 1) & (G4 - 1))), Wc, 1);
                    }
                    uint32_t Y[DT], nm[DT];
#pragma unroll
                    for (int e = 0; e < DT; ++e) {
                        uint32_t j;
                        oct_entry(o, i * DT + e, j, nm[e]);
                        Y[e] = ld32(pb + ((j << lgG4) + (uint32_t)gg) * 4u);
                    }
                    const OctSite site = oct_site(o, i);
                    const uint32_t ctr0 = (uint32_t)(2 * i + p) * (uint32_t)G4 + (uint32_t)gg;
                    const uint32_t nx = oct_update<DT, SPL, false>(X, Tlo, Thi, Y, nm, site, ctr0, tt,
                                                                   (uint32_t)c0, (uint32_t)n, L.key0,
                                                                   L.key1, nv, half);
                    if (half == 0) st32(pb + rowi + 4u * (uint32_t)gg, nx);
                }
                __syncthreads();
            }
        }
    }
}

// E_cl and C of the octet's slots from its final spins, into the LDS reduction area.
template <int DT>
__device__ __forceinline__ void oct_tile_energy(const OctLaunch &L, const InstDesc &d, char *lds,
                                                const OctLds &o)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int N = d.N, G4 = d.G4, lgG4 = 31 - __clz(G4);
    const uint32_t plane = (uint32_t)N * (uint32_t)G4 * 4u;
    int e2[8], cc[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) e2[r] = cc[r] = 0;
    for (int it = tid; it < (N << lgG4); it += nt) {
        const int gg = it & (G4 - 1), i = it >> lgG4;
        const uint32_t rowi = (uint32_t)(i << lgG4) * 4u;
        const uint32_t X0 = ld32(rowi + 4u * (uint32_t)gg);
        const uint32_t X1 = ld32(plane + rowi + 4u * (uint32_t)gg);
        const uint32_t X0n = ld32(rowi + 4u * (uint32_t)((gg + 1) & (G4 - 1)));
        uint32_t Y0[DT], Y1[DT], nm[DT];
#pragma unroll
        for (int e = 0; e < DT; ++e) {
            uint32_t j;
            oct_entry(o, i * DT + e, j, nm[e]);
            const uint32_t a = ((j << lgG4) + (uint32_t)gg) * 4u;
            Y0[e] = ld32(a);
            Y1[e] = ld32(plane + a);
        }
        const int h = L.st.hfield[d.site_base + i];
        oct_energy_item<DT>(X0, X1, X0n, Y0, Y1, nm, h, e2, cc);
    }
    oct_reduce(lds, o, e2, cc);
}

// One whole octet (work item `item`): stage, all sweeps of the call, E_cl and C, write-back;
// with L.fuse, count the octet for its instance and run the instance's exchange step in
// the workgroup that completes it.  flag: an LDS word past the octet's layout.
__device__ __forceinline__ void oct_tile_item(const OctLaunch &L, char *lds, int item, uint32_t flag)
{
    const DevState &st = L.st;
    const int32_t *rec = st.otiles + (int64_t)item * kOctRec;
    const int n = rec[0], w = rec[1], oct = rec[2];
    const InstDesc d = st.inst[n];
    const OctLds o = oct_layout(d, d.G4, kOctTile);
    const int tid = threadIdx.x, nt = blockDim.x;
    const int N = d.N, G4 = d.G4, lgG4 = 31 - __clz(G4);
    const int c0 = 32 * w + 8 * oct;
    const int nslots = min(8, d.R - c0);
    const uint32_t sel = ((uint32_t)(4 + oct) << 8) | (uint32_t)oct | 0x0C0C0000u;
    // the octet's bytes of both parities: LDS word [p][i][g]
    const int words = 2 * (N << lgG4);
    batched(words,
            [&](int k) {
                const int g = k & (G4 - 1), pi = k >> lgG4;
                const int p = pi >= N ? 1 : 0, i = pi - p * N;
                return oct_load(oct_row(st, d, w, p, i), g, sel);
            },
            [&](int k, uint32_t v) { st32(4u * (uint32_t)k, v); });
    oct_stage_common(st, d, lds, o, c0, nslots);
    const uint64_t t0 = st.ctr[n].t;
    __syncthreads();
    // two lanes per item when every step's items fit half the workgroup (a step sweeps two
    // classes when there are two or more)
    int most = 0;
    for (int g = 0; g < d.n_colors; ++g)
        most = max(most, (int)(ld32(o.coff + 4u * (uint32_t)(g + 1)) - ld32(o.coff + 4u * (uint32_t)g)));
    const bool split = ((d.n_colors >= 2 ? 4 : 2) * most) << lgG4 <= nt;
    oct_dispatch(d.D, split, [&](auto dt, auto spl) {
        constexpr int DT = decltype(dt)::value, SPL = decltype(spl)::value;
        oct_tile_sweeps<DT, SPL>(L, d, o, n, c0, nslots, t0);
    });
    switch (d.D) {
    case 1: oct_tile_energy<1>(L, d, lds, o); break;
    case 2: oct_tile_energy<2>(L, d, lds, o); break;
    case 3: oct_tile_energy<3>(L, d, lds, o); break;
    case 4: oct_tile_energy<4>(L, d, lds, o); break;
    case 5: oct_tile_energy<5>(L, d, lds, o); break;
    case 6: oct_tile_energy<6>(L, d, lds, o); break;
    case 7: oct_tile_energy<7>(L, d, lds, o); break;
    default: oct_tile_energy<8>(L, d, lds, o); break;
    }
    __syncthreads();
    const int64_t *red = reinterpret_cast<const int64_t *>(lds + o.red);
    if (tid < nslots) {
        if (L.fuse) {
            // read by the exchange step in this launch, possibly on another XCD
            __hip_atomic_store(&st.E[d.rep_base + c0 + tid], red[tid] / 2, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&st.C[d.rep_base + c0 + tid], red[8 + tid], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else {
            st.E[d.rep_base + c0 + tid] = red[tid] / 2;
            st.C[d.rep_base + c0 + tid] = red[8 + tid];
        }
    }
    // write the octet's bytes back
    for (int k = tid; k < words; k += nt) {
        const int g = k & (G4 - 1), pi = k >> lgG4;
        const int p = pi >= N ? 1 : 0, i = pi - p * N;
        oct_store(oct_row(st, d, w, p, i), g, oct, ld32(4u * (uint32_t)k));
    }
    if (!L.fuse) return;
    // every wave's E_cl, C stores complete before the count (a barrier does not wait for
    // them); the completing workgroup reads them with agent-scope atomic loads
    __builtin_amdgcn_s_waitcnt(kOctWaitVmcnt0);
    __syncthreads();
    if (tid == 0) {
        const uint32_t before =
            __hip_atomic_fetch_add(&st.icount[n], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t done = before + 1u == (uint32_t)st.itiles[n] ? 1u : 0u;
        if (done) __hip_atomic_store(&st.icount[n], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        st32(flag, done);
    }
    __syncthreads();
    if (ld32(flag)) exchange_instance<true>(st, n, L.swap_key0, L.swap_key1, L.t_add);
}

// Whole octets, one workgroup each.  Workgroup b sweeps list position tile0 + b: the
// hardware hands workgroups to each XCD in index order as its units free up, and the list
// is dealt to the XCDs largest first, so that order already runs the largest octets first.
// With L.queue the workgroup instead takes its position from the work queues as it starts
// (each start then waits for device-scope atomics).
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) oct_tile_kernel(OctLaunch L)
{
    extern __shared__ __align__(16) char lds[];
    const DevState &st = L.st;
    if ((uint32_t)(uintptr_t)lds != 0u) {  // the addressing below assumes LDS address 0
        if (threadIdx.x == 0) atomicOr(st.err, kErrLdsBase);
        return;
    }
    // two LDS words past every octet's layout: the taken position and the exchange flag
    const uint32_t slot = (uint32_t)L.lds_bytes - (uint32_t)kOctQueueLds;
    int k = (int)blockIdx.x;
    if (L.queue) {
        if (threadIdx.x == 0) st32(slot, (uint32_t)xcd_take(st.oqitems, st.oqueue, (int)gridDim.x));
        __syncthreads();
        // the same in every lane: scalar, so that everything derived from the octet's
        // record (its instance descriptor above all) stays in scalar registers
        k = __builtin_amdgcn_readfirstlane((int)ld32(slot));
        if (k < 0) {
            if (threadIdx.x == 0) atomicOr(st.err, kErrQueue);
            return;
        }
    }
    oct_tile_item(L, lds, L.tile0 + k, slot + 4u);
}

// ------------------------------------------------------------------ slice blocks

// A slice block's words of the parity swept ("own") and of the other parity ("oth") in LDS:
// word (site i, local group x) at base + i * stride + 4 x.  own's x = 0 is the block's first
// group g0; oth's x = 0 is group g0 - 1 when parity 0 is swept and g0 when parity 1 is.
struct OctPlanes {
    uint32_t own, own_stride, oth, oth_stride;
};

// Every colour class of parity p over the block's ng groups.  SPL: slots per lane (8, or 4
// with two lanes per item, for blocks with few items per colour class).
template <int DT, int SPL>
__device__ __forceinline__ void oct_block_sweep(const OctLaunch &L, const InstDesc &d, const OctLds &o,
                                                const OctPlanes &pl, int p, int n, int c0,
                                                int nslots, int g0, int ng, uint32_t tt)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int G4 = d.G4, lgng = 31 - __clz(ng);
    constexpr int lgL = SPL == 8 ? 0 : 1;  // lanes per item
    // items come in lane pairs and the block size is even, so a thread keeps its half
    const int half = tid & ((1 << lgL) - 1);
    const uint32_t vmask = oct_slot_mask<SPL>(nslots, half);
    for (int g = 0; g < d.n_colors; ++g) {
        const int s0 = (int)ld32(o.coff + 4u * (uint32_t)g);
        const int items = ((int)ld32(o.coff + 4u * (uint32_t)(g + 1)) - s0) << (lgng + lgL);
        for (int it = tid; it < items; it += nt) {
            const uint32_t gl4 = 4u * (uint32_t)((it >> lgL) & (ng - 1));
            const int i = (int)ld16(o.csite + 2u * (uint32_t)(s0 + (it >> (lgng + lgL))));
            const uint32_t own = pl.own + (uint32_t)i * pl.own_stride + gl4;
            const uint32_t oth = pl.oth + (uint32_t)i * pl.oth_stride + gl4;
            const uint32_t X = ld32(own);
            const uint32_t W0 = ld32(oth), W1 = ld32(oth + 4u);
            uint32_t Tlo, Thi;
            if (p == 0) {
                Tlo = __builtin_amdgcn_alignbyte(W1, W0, 3);
                Thi = W1;
            } else {
                Tlo = W0;
                Thi = __builtin_amdgcn_alignbyte(W1, W0, 1);
            }
            uint32_t Y[DT], nm[DT];
#pragma unroll
            for (int e = 0; e < DT; ++e) {
                uint32_t j;
                oct_entry(o, i * DT + e, j, nm[e]);
                Y[e] = ld32(pl.own + j * pl.own_stride + gl4);
            }
            const OctSite site = oct_site(o, i);
            const uint32_t ctr0 = (uint32_t)(2 * i + p) * (uint32_t)G4 + (uint32_t)g0 + (gl4 >> 2);
            const uint32_t nx = oct_update<DT, SPL, true>(X, Tlo, Thi, Y, nm, site, ctr0, tt,
                                                          (uint32_t)c0, (uint32_t)n, L.key0, L.key1,
                                                          vmask, half);
            if (half == 0) st32(own, nx);
        }
        __syncthreads();
    }
}

// The block's part of E_cl and C into its LDS reduction area, from the final spins: p1
// holds parity 1 of the block's groups (as own), p0 parity 0 of groups g0 .. g0 + ng (as
// oth of a parity-1 sweep).
template <int DT>
__device__ __forceinline__ void oct_block_energy(const OctLaunch &L, const InstDesc &d, char *lds,
                                                 const OctLds &o, const OctPlanes &p1, int ng)
{
    const int tid = threadIdx.x, nt = blockDim.x, lgng = 31 - __clz(ng);
    int e2[8], cc[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) e2[r] = cc[r] = 0;
    for (int it = tid; it < (d.N << lgng); it += nt) {
        const uint32_t gl4 = 4u * (uint32_t)(it & (ng - 1));
        const int i = it >> lgng;
        const uint32_t X1 = ld32(p1.own + (uint32_t)i * p1.own_stride + gl4);
        const uint32_t oth = p1.oth + (uint32_t)i * p1.oth_stride + gl4;
        const uint32_t X0 = ld32(oth), X0n = ld32(oth + 4u);
        uint32_t Y0[DT], Y1[DT], nm[DT];
#pragma unroll
        for (int e = 0; e < DT; ++e) {
            uint32_t j;
            oct_entry(o, i * DT + e, j, nm[e]);
            Y0[e] = ld32(p1.oth + j * p1.oth_stride + gl4);
            Y1[e] = ld32(p1.own + j * p1.own_stride + gl4);
        }
        const int h = L.st.hfield[d.site_base + i];
        oct_energy_item<DT>(X0, X1, X0n, Y0, Y1, nm, h, e2, cc);
    }
    oct_reduce(lds, o, e2, cc);
}

// The block's reduced part of 2 E_cl and C added to the replicas' E_cl and C (cleared before
// the call).  Every block's part of 2 E_cl is even (its bonds come in pairs i-j, j-i and the
// field term is 2 h s), so the halves add up exactly.
__device__ __forceinline__ void oct_block_energy_out(const DevState &st, const InstDesc &d,
                                                     const char *lds, const OctLds &o, int c0,
                                                     int nslots)
{
    const int tid = threadIdx.x;
    if (tid < nslots) {
        const int64_t *red = reinterpret_cast<const int64_t *>(lds + o.red);
        atomicAdd(reinterpret_cast<unsigned long long *>(&st.E[d.rep_base + c0 + tid]),
                  (unsigned long long)(red[tid] / 2));
        atomicAdd(reinterpret_cast<unsigned long long *>(&st.C[d.rep_base + c0 + tid]),
                  (unsigned long long)red[8 + tid]);
    }
}

// ng1 consecutive groups of parity p from group gb on (cyclically) into LDS rows of ng1
// words at base, x-major so that neighbouring threads read neighbouring rows.
__device__ __forceinline__ void oct_stage_rows(const DevState &st, const InstDesc &d, int w, int p,
                                               int gb, int ng1, uint32_t base, uint32_t sel)
{
    const int N = d.N, G4 = d.G4;
    batched(N * ng1,
            [&](int k) {
                const int x = k / N, i = k - x * N;
                return oct_load(oct_row(st, d, w, p, i), (gb + x + G4) & (G4 - 1), sel);
            },
            [&](int k, uint32_t v) {
                const int x = k / N, i = k - x * N;
                st32(base + 4u * (uint32_t)(i * ng1 + x), v);
            });
}

__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) oct_phase_kernel(OctLaunch L)
{
    extern __shared__ __align__(16) char lds[];
    const DevState &st = L.st;
    if ((uint32_t)(uintptr_t)lds != 0u) {  // the addressing below assumes LDS address 0
        if (threadIdx.x == 0) atomicOr(st.err, kErrLdsBase);
        return;
    }
    const int32_t *rec = st.otiles + (int64_t)(L.tile0 + blockIdx.x) * kOctRec;
    const int n = rec[0], w = rec[1], oct = rec[2], g0 = rec[3], ng = rec[4];
    const InstDesc d = st.inst[n];
    const OctLds o = oct_layout(d, ng, kOctPhase);
    const int tid = threadIdx.x, nt = blockDim.x;
    const int N = d.N, p = L.p, lgng = 31 - __clz(ng);
    const int c0 = 32 * w + 8 * oct;
    const int nslots = min(8, d.R - c0);
    const uint32_t sel = ((uint32_t)(4 + oct) << 8) | (uint32_t)oct | 0x0C0C0000u;
    // own: parity p, groups g0 .. g0 + ng - 1; oth: parity 1 - p, ng + 1 groups from g0 - 1
    // (p = 0) or g0 (p = 1)
    batched(N << lgng,
            [&](int k) {
                const int gl = k & (ng - 1), i = k >> lgng;
                return oct_load(oct_row(st, d, w, p, i), g0 + gl, sel);
            },
            [&](int k, uint32_t v) { st32(o.sp + 4u * (uint32_t)k, v); });
    oct_stage_rows(st, d, w, p ^ 1, p == 0 ? g0 - 1 : g0, ng + 1, o.oth, sel);
    oct_stage_common(st, d, lds, o, c0, nslots);
    const uint32_t tt = (uint32_t)(st.ctr[n].t + (uint64_t)L.sweep_off);
    __syncthreads();
    const OctPlanes pl = {o.sp, 4u * (uint32_t)ng, o.oth, 4u * (uint32_t)(ng + 1)};
    const bool energy = L.last && p == 1;
    oct_dispatch(d.D, L.split != 0, [&](auto dt, auto spl) {
        constexpr int DT = decltype(dt)::value, SPL = decltype(spl)::value;
        oct_block_sweep<DT, SPL>(L, d, o, pl, p, n, c0, nslots, g0, ng, tt);
        if (energy) oct_block_energy<DT>(L, d, lds, o, pl, ng);
    });
    __syncthreads();
    if (energy) oct_block_energy_out(st, d, lds, o, c0, nslots);
    for (int k = tid; k < (N << lgng); k += nt) {
        const int gl = k & (ng - 1), i = k >> lgng;
        oct_store(oct_row(st, d, w, p, i), g0 + gl, oct, ld32(o.sp + 4u * (uint32_t)k));
    }
}

// ------------------------------------------------------------------ resident slice blocks

// Boundary records and progress counts pass between workgroups on different XCDs, whose
// L2 caches are not coherent with one another.  They are read and written only with
// agent-scope atomic operations, which the hardware performs coherently for the whole
// device, so no L2 write-back or invalidation is needed: a block's waves each wait for
// their record stores to complete before the barrier that precedes the count's store, and
// a reader issues its record loads only after it has seen the count.  (Publishing through
// an agent-scope release and acquire instead, which write the whole XCD's L2 back and
// invalidate it, made config 4's sweeps 1.4x slower.)
//
// When every ring of blocks sits on one XCD (LOCAL), a block's reader and writer share that
// XCD's L2, and the stores need not go through to the coherence point: records and counts
// are written with plain stores, which land in the L2, and read with the same
// device-scope loads, which bypass the L1 and find the L2's line (measured between two
// workgroups of one XCD: a round trip of 0.76 us against 2.8 us with device-scope stores).
constexpr int kOctWaitPolls = 1 << 18;
__device__ __forceinline__ uint32_t rec_ld(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool LOCAL>
__device__ __forceinline__ void rec_st(uint32_t *p, uint32_t v)
{
    if constexpr (LOCAL)
        *p = v;
    else
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 polls *flag until it reaches need while the workgroup waits at a barrier.  The
// wait is bounded: a block that gives up sets the error word and carries on, so every wave
// always exits (the host then reports the call as failed); once any block has given up,
// the others stop waiting too.
__device__ __forceinline__ void oct_wait(const DevState &st, const int32_t *flag, int need,
                                         int max_polls)
{
    if (threadIdx.x == 0) {
        int polls = 0;
        while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
            if (++polls > max_polls ||
                __hip_atomic_load(st.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                atomicOr(st.err, kErrWait);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
}

// After the workgroup's record stores: every wave waits for its own stores to complete
// (a workgroup barrier does not wait for them), then thread 0 stores v.
template <bool LOCAL>
__device__ __forceinline__ void oct_publish(int32_t *flag, int v)
{
    __builtin_amdgcn_s_waitcnt(kOctWaitVmcnt0);
    __syncthreads();
    if (threadIdx.x == 0) rec_st<LOCAL>(reinterpret_cast<uint32_t *>(flag), (uint32_t)v);
}

// All sweeps of a call over one octet slice block, with every block of the launch resident.
// LDS keeps P0 = parity 0 of groups g0 .. g0 + ng and P1 = parity 1 of groups g0 - 1 ..
// g0 + ng - 1 (rows of ng + 1 words); the first group of P0 and of P1 are halos owned by
// the neighbouring blocks of the octet's ring of blocks (prev ends at g0 - 1, next starts at
// g0 + ng).  Per sweep:
//   1. (after the first sweep) wait for prev's parity-1 progress of the previous sweep and
//      take its last parity-1 group as P1's halo;
//   2. parity 0 over the own groups;
//   3. publish the first own parity-0 group (record R0) and the parity-0 progress;
//   4. wait for next's parity-0 progress of this sweep and take its first parity-0 group
//      as P0's halo;
//   5. parity 1 over the own groups;
//   6. (before another sweep) publish the last own parity-1 group (record R1) and the
//      parity-1 progress.
// One record buffer of each kind suffices: a block rewrites R0 in step 3 of sweep s + 1
// only after step 1 has seen prev finish sweep s (whose step 4 read R0), and R1 in step 6 of
// sweep s + 1 only after step 4 has seen next reach step 3 of sweep s + 1 (after its step 1
// read R1).  Progress counts are per call (zeroed by oct_clear).  After the last sweep the
// block adds its part of E_cl and C and writes its own groups back.
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4))) oct_resident_kernel(OctLaunch L)
{
    extern __shared__ __align__(16) char lds[];
    const DevState &st = L.st;
    if ((uint32_t)(uintptr_t)lds != 0u) {  // the addressing below assumes LDS address 0
        if (threadIdx.x == 0) atomicOr(st.err, kErrLdsBase);
        return;
    }
    // runs of consecutive blocks share an XCD (xcd_tile); with L.xcd_local every ring of
    // blocks lies in one run, and a launch whose workgroups did not keep to that fails the
    // call (checked at the end; the host recovers), each block running to its end, its
    // waits bounded
    const int b = L.tile0 + xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int32_t *rec = st.otiles + (int64_t)b * kOctRec;
    const int n = rec[0], w = rec[1], oct = rec[2], g0 = rec[3], ng = rec[4];
    const int roff = rec[5], prev = rec[6], next = rec[7];
    const int roff_prev = st.otiles[(int64_t)prev * kOctRec + 5];
    const int roff_next = st.otiles[(int64_t)next * kOctRec + 5];
    const InstDesc d = st.inst[n];
    const OctLds o = oct_layout(d, ng, kOctResident);
    const int tid = threadIdx.x, nt = blockDim.x;
    const int N = d.N, lgng = 31 - __clz(ng);
    const int c0 = 32 * w + 8 * oct;
    const int nslots = min(8, d.R - c0);
    const uint32_t sel = ((uint32_t)(4 + oct) << 8) | (uint32_t)oct | 0x0C0C0000u;
    const uint32_t RS = 4u * (uint32_t)(ng + 1), P0 = o.sp, P1 = o.oth;
    oct_stage_rows(st, d, w, 0, g0, ng + 1, P0, sel);
    oct_stage_rows(st, d, w, 1, g0 - 1, ng + 1, P1, sel);
    oct_stage_common(st, d, lds, o, c0, nslots);
    const uint64_t t0 = st.ctr[n].t;
    __syncthreads();
    uint32_t *R0 = st.orec + roff;                   // records: R0 region, then R1 region
    uint32_t *R1 = st.orec + L.rec_words + roff;
    const uint32_t *R1prev = st.orec + L.rec_words + roff_prev;
    const uint32_t *R0next = st.orec + roff_next;
    int32_t *prog = st.oprog;                        // [2 * work item + parity]
    const int polls = L.wait_polls > 0 ? L.wait_polls : kOctWaitPolls;
    const OctPlanes pl0 = {P0, RS, P1, RS}, pl1 = {P1 + 4u, RS, P0, RS};
    const uint32_t halo1 = P1, halo0 = P0 + 4u * (uint32_t)ng;  // x = 0 of P1, x = ng of P0
    auto sweeps = [&](auto local) __attribute__((always_inline)) {
        constexpr bool LOCAL = decltype(local)::value != 0;
        oct_dispatch(d.D, L.split != 0, [&](auto dt, auto spl) {
            constexpr int DT = decltype(dt)::value, SPL = decltype(spl)::value;
            for (int sw = 0; sw < L.n_sweeps; ++sw) {
                const uint32_t tt = (uint32_t)(t0 + (uint64_t)sw);
                if (sw > 0) {
                    oct_wait(st, prog + 2 * prev + 1, sw + L.wait_extra, polls);
                    for (int i = tid; i < N; i += nt)
                        st32(halo1 + (uint32_t)i * RS, rec_ld(R1prev + i));
                    __syncthreads();
                }
                oct_block_sweep<DT, SPL>(L, d, o, pl0, 0, n, c0, nslots, g0, ng, tt);
                for (int i = tid; i < N; i += nt) rec_st<LOCAL>(R0 + i, ld32(P0 + (uint32_t)i * RS));
                oct_publish<LOCAL>(prog + 2 * b, sw + 1);
                oct_wait(st, prog + 2 * next, sw + 1 + L.wait_extra, polls);
                for (int i = tid; i < N; i += nt)
                    st32(halo0 + (uint32_t)i * RS, rec_ld(R0next + i));
                __syncthreads();
                oct_block_sweep<DT, SPL>(L, d, o, pl1, 1, n, c0, nslots, g0, ng, tt);
                if (sw + 1 < L.n_sweeps) {
                    for (int i = tid; i < N; i += nt)
                        rec_st<LOCAL>(R1 + i, ld32(P1 + (uint32_t)i * RS + 4u * (uint32_t)ng));
                    oct_publish<LOCAL>(prog + 2 * b + 1, sw + 1);
                }
            }
            oct_block_energy<DT>(L, d, lds, o, pl1, ng);
        });
    };
    if (L.xcd_local)
        sweeps(IC<1>{});
    else
        sweeps(IC<0>{});
    __syncthreads();
    oct_block_energy_out(st, d, lds, o, c0, nslots);
    for (int k = tid; k < (N << lgng); k += nt) {
        const int x = k & (ng - 1), i = k >> lgng;
        oct_store(oct_row(st, d, w, 0, i), g0 + x, oct, ld32(P0 + (uint32_t)i * RS + 4u * (uint32_t)x));
        oct_store(oct_row(st, d, w, 1, i), g0 + x, oct, ld32(P1 + (uint32_t)i * RS + 4u * (uint32_t)(x + 1)));
    }
    if (L.xcd_local) xcd_check(st, st.xseen, (int)blockIdx.x, kErrPlace, L.xcd_local == 2);
}

// E_cl and C of the slice-block octets set to zero (the block at group 0 clears its
// octet's), and every block's progress counts.
__global__ void oct_clear_kernel(OctLaunch L)
{
    const int b = L.tile0 + (int)blockIdx.x;
    const int32_t *rec = L.st.otiles + (int64_t)b * kOctRec;
    const int r = threadIdx.x;
    if (r < 2) L.st.oprog[2 * b + r] = 0;
    if (blockIdx.x == 0 && r == 0) L.st.xseen[0] = 0u;
    if (rec[3] != 0) return;
    const InstDesc d = L.st.inst[rec[0]];
    const int c0 = 32 * rec[1] + 8 * rec[2];
    if (r < 8 && c0 + r < d.R) {
        L.st.E[d.rep_base + c0 + r] = 0;
        L.st.C[d.rep_base + c0 + r] = 0;
    }
}

}  // namespace

int32_t oct_lds_bytes(const InstDesc &d, int32_t ng, int mode)
{
    return (int32_t)oct_layout(d, ng, mode).end;
}

hipError_t oct_kernels_set_lds(int32_t tile_bytes, int32_t phase_bytes, int32_t resident_bytes)
{
    hipError_t e = hipSuccess;
    if (tile_bytes > 0)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&oct_tile_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, tile_bytes);
    if (e == hipSuccess && phase_bytes > 0)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&oct_phase_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, phase_bytes);
    if (e == hipSuccess && resident_bytes > 0)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&oct_resident_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, resident_bytes);
    return e;
}

hipError_t oct_resident_per_cu(int32_t threads, int32_t lds_bytes, int32_t *per_cu)
{
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &n, reinterpret_cast<const void *>(&oct_resident_kernel), threads, (size_t)lds_bytes);
    *per_cu = n;
    return e;
}

hipError_t launch_oct_resident(const OctLaunch &L, hipStream_t s)
{
    if (L.n_tiles <= 0 || L.n_sweeps <= 0) return hipSuccess;
    hipLaunchKernelGGL(oct_resident_kernel, dim3(L.n_tiles), dim3(L.threads), L.lds_bytes, s, L);
    return hipGetLastError();
}

hipError_t launch_oct_tiles(const OctLaunch &L, hipStream_t s)
{
    if (L.n_tiles <= 0 || L.n_sweeps <= 0) return hipSuccess;
    hipLaunchKernelGGL(oct_tile_kernel, dim3(L.n_tiles), dim3(L.threads), L.lds_bytes, s, L);
    return hipGetLastError();
}

hipError_t launch_oct_phase(const OctLaunch &L, hipStream_t s)
{
    if (L.n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(oct_phase_kernel, dim3(L.n_tiles), dim3(L.threads), L.lds_bytes, s, L);
    return hipGetLastError();
}

hipError_t launch_oct_clear(const OctLaunch &L, hipStream_t s)
{
    if (L.n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(oct_clear_kernel, dim3(L.n_tiles), dim3(64), 0, s, L);
    return hipGetLastError();
}

}  // namespace ptq
