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
#include "pt_internal.h"

#pragma clang fp contract(off)

namespace ptq {
namespace {

constexpr int kWave = 64;

template <int V>
struct IC {
    static constexpr int value = V;
};

__device__ __forceinline__ uint32_t ld32(const char *base, uint32_t off)
{
    return *reinterpret_cast<const uint32_t *>(base + off);
}
__device__ __forceinline__ void st32(char *base, uint32_t off, uint32_t v)
{
    *reinterpret_cast<uint32_t *>(base + off) = v;
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

// Bit r of every byte of plane p moved to bit q + 2 of that byte (q + 2 - r is a constant
// after unrolling).
template <int Q>
__device__ __forceinline__ uint32_t place(uint32_t p, int r)
{
    const int sh = Q + 2 - r;
    const uint32_t v = sh >= 0 ? (p << sh) : (p >> (-sh));
    return v & (0x01010101u << (Q + 2));
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
// their flips with one lane exchange (both must call).
template <int DT, int SPL>
__device__ __forceinline__ uint32_t oct_update(const char *lds, uint32_t X, uint32_t Tlo,
                                               uint32_t Thi, const uint32_t (&Y)[DT],
                                               const uint32_t (&nm)[DT], const OctSite &site,
                                               uint32_t ctr0, uint32_t tt, uint32_t cbase,
                                               uint32_t n, uint32_t key0, uint32_t key1,
                                               int nslots, int half)
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
    uint32_t flip = 0u;
#pragma unroll
    for (int r = 0; r < SPL; ++r) {
        if (sh + r < nslots) {
            // table byte offsets 4 (n + 16 sigma) of the four slices of slot sh + r
            const uint32_t idx = place<0>(n0, r) | place<1>(n1, r) | place<2>(n2, r) |
                                 place<3>(n3, r) | place<4>(s0, r) | place<5>(s1, r);
            const Words4 u = philox10(ctr0, tt, cbase + (uint32_t)(sh + r), n, key0, key1);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const uint32_t addr = __builtin_amdgcn_perm(tbase, idx, 0x0C060500u | (uint32_t)b);
                const uint32_t thr = ld32(lds, addr + 512u * (uint32_t)r);
                flip |= (u.w[b] <= thr ? 1u : 0u) << (8 * b + r);
            }
        }
    }
    flip <<= sh;
    if constexpr (SPL < 8) flip |= (uint32_t)__shfl_xor((int)flip, 1, kWave);
    return X ^ flip;
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
// G4 groups, N * M bytes).  Slice blocks: own holds [i][gl] words of the parity swept (ng
// groups), oth [i][x] words of the other parity (ng + 1 groups).  Then the eight slots'
// tables (256-byte aligned, 512 bytes each), the 16-bit neighbour entries, field codes,
// colour lists and a reduction area of 16 int64.
struct OctLds {
    uint32_t sp, oth, tbl, ent, hinfo, csite, coff, red, end;
};

__host__ __device__ __forceinline__ uint32_t a16u(uint32_t x) { return (x + 15u) & ~15u; }
__host__ __device__ __forceinline__ uint32_t a256u(uint32_t x) { return (x + 255u) & ~255u; }

__host__ __device__ __forceinline__ OctLds oct_layout(const InstDesc &d, int ng, bool phase)
{
    OctLds o;
    const uint32_t N = (uint32_t)d.N;
    o.sp = 0;
    if (phase) {
        o.oth = a16u(N * (uint32_t)ng * 4u);
        o.tbl = a256u(o.oth + N * (uint32_t)(ng + 1) * 4u);
    } else {
        o.oth = 0;
        o.tbl = a256u(2u * N * (uint32_t)d.G4 * 4u);
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

__device__ __forceinline__ OctSite oct_site(const char *lds, const OctLds &o, int i)
{
    const uint32_t hb = reinterpret_cast<const uint8_t *>(lds + o.hinfo)[i];
    OctSite s;
    s.hneg = (hb & 1u) ? 0xFFFFFFFFu : 0u;
    s.hzm = (hb & 2u) ? 0xFFFFFFFFu : 0u;
    s.hzbase = o.tbl + ((hb & 2u) ? 256u : 0u);
    return s;
}

// Neighbour e of site i: its site index and sign mask (~0 when J < 0).
__device__ __forceinline__ void oct_entry(const char *lds, const OctLds &o, int idx, uint32_t &j,
                                          uint32_t &nm)
{
    const uint32_t v = reinterpret_cast<const uint16_t *>(lds + o.ent)[idx];
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

// ------------------------------------------------------------------ whole octets

template <int DT>
__device__ __forceinline__ void oct_tile_sweeps(const OctLaunch &L, const InstDesc &d, char *lds,
                                                const OctLds &o, int n, int c0, int nslots,
                                                uint64_t t0)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int N = d.N, G4 = d.G4, lgG4 = 31 - __clz(G4);
    const uint32_t plane = (uint32_t)N * (uint32_t)G4 * 4u;
    const uint16_t *cs = reinterpret_cast<const uint16_t *>(lds + o.csite);
    const int32_t *co = reinterpret_cast<const int32_t *>(lds + o.coff);
    for (int sw = 0; sw < L.n_sweeps; ++sw) {
        const uint32_t tt = (uint32_t)(t0 + (uint64_t)sw);
        for (int p = 0; p < 2; ++p) {
            const uint32_t pb = (uint32_t)p * plane, ob = (uint32_t)(p ^ 1) * plane;
            for (int g = 0; g < d.n_colors; ++g) {
                const int s0 = co[g];
                const int items = (co[g + 1] - s0) << lgG4;
                for (int it = tid; it < items; it += nt) {
                    const int gg = it & (G4 - 1);
                    const int i = cs[s0 + (it >> lgG4)];
                    const uint32_t rowi = (uint32_t)(i << lgG4) * 4u;
                    const uint32_t X = ld32(lds, pb + rowi + 4u * (uint32_t)gg);
                    const uint32_t Wc = ld32(lds, ob + rowi + 4u * (uint32_t)gg);
                    uint32_t Tlo, Thi;
                    if (p == 0) {
                        Tlo = __builtin_amdgcn_alignbyte(Wc, ld32(lds, ob + rowi + 4u * (uint32_t)((gg - 1) & (G4 - 1))), 3);
                        Thi = Wc;
                    } else {
                        Tlo = Wc;
                        Thi = __builtin_amdgcn_alignbyte(ld32(lds, ob + rowi + 4u * (uint32_t)((gg + 1) & (G4 - 1))), Wc, 1);
                    }
                    uint32_t Y[DT], nm[DT];
#pragma unroll
                    for (int e = 0; e < DT; ++e) {
                        uint32_t j;
                        oct_entry(lds, o, i * DT + e, j, nm[e]);
                        Y[e] = ld32(lds, pb + ((j << lgG4) + (uint32_t)gg) * 4u);
                    }
                    const OctSite site = oct_site(lds, o, i);
                    const uint32_t ctr0 = (uint32_t)(2 * i + p) * (uint32_t)G4 + (uint32_t)gg;
                    st32(lds, pb + rowi + 4u * (uint32_t)gg,
                         oct_update<DT, 8>(lds, X, Tlo, Thi, Y, nm, site, ctr0, tt, (uint32_t)c0,
                                           (uint32_t)n, L.key0, L.key1, nslots, 0));
                }
                __syncthreads();
            }
        }
    }
    // E_cl and C of the eight slots
    int e2[8], cc[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) e2[r] = cc[r] = 0;
    for (int it = tid; it < (N << lgG4); it += nt) {
        const int gg = it & (G4 - 1), i = it >> lgG4;
        const uint32_t rowi = (uint32_t)(i << lgG4) * 4u;
        const uint32_t X0 = ld32(lds, rowi + 4u * (uint32_t)gg);
        const uint32_t X1 = ld32(lds, plane + rowi + 4u * (uint32_t)gg);
        const uint32_t X0n = ld32(lds, rowi + 4u * (uint32_t)((gg + 1) & (G4 - 1)));
        uint32_t Y0[DT], Y1[DT], nm[DT];
#pragma unroll
        for (int e = 0; e < DT; ++e) {
            uint32_t j;
            oct_entry(lds, o, i * DT + e, j, nm[e]);
            const uint32_t a = ((j << lgG4) + (uint32_t)gg) * 4u;
            Y0[e] = ld32(lds, a);
            Y1[e] = ld32(lds, plane + a);
        }
        const int h = L.st.hfield[d.site_base + i];
        oct_energy_item<DT>(X0, X1, X0n, Y0, Y1, nm, h, e2, cc);
    }
    oct_reduce(lds, o, e2, cc);
}

__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) oct_tile_kernel(OctLaunch L)
{
    extern __shared__ __align__(16) char lds[];
    const DevState &st = L.st;
    const int32_t *rec = st.otiles + (int64_t)(L.tile0 + blockIdx.x) * kOctRec;
    const int n = rec[0], w = rec[1], oct = rec[2];
    const InstDesc d = st.inst[n];
    const OctLds o = oct_layout(d, d.G4, false);
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
            [&](int k, uint32_t v) { st32(lds, 4u * (uint32_t)k, v); });
    oct_stage_common(st, d, lds, o, c0, nslots);
    const uint64_t t0 = st.ctr[n].t;
    __syncthreads();
    switch (d.D) {
    case 1: oct_tile_sweeps<1>(L, d, lds, o, n, c0, nslots, t0); break;
    case 2: oct_tile_sweeps<2>(L, d, lds, o, n, c0, nslots, t0); break;
    case 3: oct_tile_sweeps<3>(L, d, lds, o, n, c0, nslots, t0); break;
    case 4: oct_tile_sweeps<4>(L, d, lds, o, n, c0, nslots, t0); break;
    case 5: oct_tile_sweeps<5>(L, d, lds, o, n, c0, nslots, t0); break;
    case 6: oct_tile_sweeps<6>(L, d, lds, o, n, c0, nslots, t0); break;
    case 7: oct_tile_sweeps<7>(L, d, lds, o, n, c0, nslots, t0); break;
    default: oct_tile_sweeps<8>(L, d, lds, o, n, c0, nslots, t0); break;
    }
    __syncthreads();
    const int64_t *red = reinterpret_cast<const int64_t *>(lds + o.red);
    if (tid < nslots) {
        st.E[d.rep_base + c0 + tid] = red[tid] / 2;
        st.C[d.rep_base + c0 + tid] = red[8 + tid];
    }
    // write the octet's bytes back
    for (int k = tid; k < words; k += nt) {
        const int g = k & (G4 - 1), pi = k >> lgG4;
        const int p = pi >= N ? 1 : 0, i = pi - p * N;
        oct_store(oct_row(st, d, w, p, i), g, oct, ld32(lds, 4u * (uint32_t)k));
    }
}

// ------------------------------------------------------------------ slice blocks

// SPL: slots per lane (8, or 4 with two lanes per item, for blocks with few items per
// colour class)
template <int DT, int SPL>
__device__ __forceinline__ void oct_phase_body(const OctLaunch &L, const InstDesc &d, char *lds,
                                               const OctLds &o, int n, int c0, int nslots, int g0,
                                               int ng, uint32_t tt)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int p = L.p, G4 = d.G4, lgng = 31 - __clz(ng);
    constexpr int lgL = SPL == 8 ? 0 : 1;  // lanes per item
    const uint32_t orow = (uint32_t)(ng + 1) * 4u, rowb = (uint32_t)ng * 4u;
    const uint16_t *cs = reinterpret_cast<const uint16_t *>(lds + o.csite);
    const int32_t *co = reinterpret_cast<const int32_t *>(lds + o.coff);
    for (int g = 0; g < d.n_colors; ++g) {
        const int s0 = co[g];
        const int items = (co[g + 1] - s0) << (lgng + lgL);
        for (int it = tid; it < items; it += nt) {
            const int half = it & ((1 << lgL) - 1);
            const int gl = (it >> lgL) & (ng - 1);
            const int i = cs[s0 + (it >> (lgng + lgL))];
            const uint32_t own = (uint32_t)i * rowb + 4u * (uint32_t)gl;
            const uint32_t oth = o.oth + (uint32_t)i * orow + 4u * (uint32_t)gl;
            const uint32_t X = ld32(lds, own);
            const uint32_t W0 = ld32(lds, oth), W1 = ld32(lds, oth + 4u);
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
                oct_entry(lds, o, i * DT + e, j, nm[e]);
                Y[e] = ld32(lds, j * rowb + 4u * (uint32_t)gl);
            }
            const OctSite site = oct_site(lds, o, i);
            const uint32_t ctr0 = (uint32_t)(2 * i + p) * (uint32_t)G4 + (uint32_t)(g0 + gl);
            const uint32_t nx = oct_update<DT, SPL>(lds, X, Tlo, Thi, Y, nm, site, ctr0, tt,
                                                    (uint32_t)c0, (uint32_t)n, L.key0, L.key1,
                                                    nslots, half);
            if (half == 0) st32(lds, own, nx);
        }
        __syncthreads();
    }
    if (!(L.last && p == 1)) return;
    // the block's part of E_cl and C: own holds parity 1 (final), oth parity 0 of groups
    // g0 .. g0 + ng (final)
    int e2[8], cc[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) e2[r] = cc[r] = 0;
    for (int it = tid; it < (d.N << lgng); it += nt) {
        const int gl = it & (ng - 1), i = it >> lgng;
        const uint32_t X1 = ld32(lds, (uint32_t)i * rowb + 4u * (uint32_t)gl);
        const uint32_t oth = o.oth + (uint32_t)i * orow + 4u * (uint32_t)gl;
        const uint32_t X0 = ld32(lds, oth), X0n = ld32(lds, oth + 4u);
        uint32_t Y0[DT], Y1[DT], nm[DT];
#pragma unroll
        for (int e = 0; e < DT; ++e) {
            uint32_t j;
            oct_entry(lds, o, i * DT + e, j, nm[e]);
            Y0[e] = ld32(lds, o.oth + j * orow + 4u * (uint32_t)gl);
            Y1[e] = ld32(lds, j * rowb + 4u * (uint32_t)gl);
        }
        const int h = L.st.hfield[d.site_base + i];
        oct_energy_item<DT>(X0, X1, X0n, Y0, Y1, nm, h, e2, cc);
    }
    oct_reduce(lds, o, e2, cc);
}

__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) oct_phase_kernel(OctLaunch L)
{
    extern __shared__ __align__(16) char lds[];
    const DevState &st = L.st;
    const int32_t *rec = st.otiles + (int64_t)(L.tile0 + blockIdx.x) * kOctRec;
    const int n = rec[0], w = rec[1], oct = rec[2], g0 = rec[3], ng = rec[4];
    const InstDesc d = st.inst[n];
    const OctLds o = oct_layout(d, ng, true);
    const int tid = threadIdx.x, nt = blockDim.x;
    const int N = d.N, G4 = d.G4, p = L.p, lgng = 31 - __clz(ng);
    const int c0 = 32 * w + 8 * oct;
    const int nslots = min(8, d.R - c0);
    const uint32_t sel = ((uint32_t)(4 + oct) << 8) | (uint32_t)oct | 0x0C0C0000u;
    // own: parity p, groups g0 .. g0 + ng - 1; oth: parity 1 - p, groups from g0 - 1 (p = 0)
    // or g0 (p = 1), ng + 1 of them, cyclically
    batched(N << lgng,
            [&](int k) {
                const int gl = k & (ng - 1), i = k >> lgng;
                return oct_load(oct_row(st, d, w, p, i), g0 + gl, sel);
            },
            [&](int k, uint32_t v) { st32(lds, 4u * (uint32_t)k, v); });
    const int gb = p == 0 ? g0 - 1 : g0;
    // the other parity's ng + 1 groups, x-major so that neighbouring threads read
    // neighbouring rows: LDS word i (ng + 1) + x
    batched(N * (ng + 1),
            [&](int k) {
                const int x = k / N, i = k - x * N;
                return oct_load(oct_row(st, d, w, p ^ 1, i), (gb + x + G4) & (G4 - 1), sel);
            },
            [&](int k, uint32_t v) {
                const int x = k / N, i = k - x * N;
                st32(lds, o.oth + 4u * (uint32_t)(i * (ng + 1) + x), v);
            });
    oct_stage_common(st, d, lds, o, c0, nslots);
    const uint32_t tt = (uint32_t)(st.ctr[n].t + (uint64_t)L.sweep_off);
    __syncthreads();
    auto body = [&](auto spl) {
        constexpr int SPL = decltype(spl)::value;
        switch (d.D) {
        case 1: oct_phase_body<1, SPL>(L, d, lds, o, n, c0, nslots, g0, ng, tt); break;
        case 2: oct_phase_body<2, SPL>(L, d, lds, o, n, c0, nslots, g0, ng, tt); break;
        case 3: oct_phase_body<3, SPL>(L, d, lds, o, n, c0, nslots, g0, ng, tt); break;
        case 4: oct_phase_body<4, SPL>(L, d, lds, o, n, c0, nslots, g0, ng, tt); break;
        case 5: oct_phase_body<5, SPL>(L, d, lds, o, n, c0, nslots, g0, ng, tt); break;
        case 6: oct_phase_body<6, SPL>(L, d, lds, o, n, c0, nslots, g0, ng, tt); break;
        case 7: oct_phase_body<7, SPL>(L, d, lds, o, n, c0, nslots, g0, ng, tt); break;
        default: oct_phase_body<8, SPL>(L, d, lds, o, n, c0, nslots, g0, ng, tt); break;
        }
    };
    if (L.split)
        body(IC<4>{});
    else
        body(IC<8>{});
    __syncthreads();
    if (L.last && p == 1 && tid < nslots) {
        const int64_t *red = reinterpret_cast<const int64_t *>(lds + o.red);
        // halves of 2 E_cl: every block's sum is even (its bonds come in pairs i-j, j-i
        // and the field term is 2 h s), so the halves add up exactly
        atomicAdd(reinterpret_cast<unsigned long long *>(&st.E[d.rep_base + c0 + tid]),
                  (unsigned long long)(red[tid] / 2));
        atomicAdd(reinterpret_cast<unsigned long long *>(&st.C[d.rep_base + c0 + tid]),
                  (unsigned long long)red[8 + tid]);
    }
    for (int k = tid; k < (N << lgng); k += nt) {
        const int gl = k & (ng - 1), i = k >> lgng;
        oct_store(oct_row(st, d, w, p, i), g0 + gl, oct, ld32(lds, 4u * (uint32_t)k));
    }
}

__global__ void oct_clear_kernel(OctLaunch L)
{
    const int32_t *rec = L.st.otiles + (int64_t)(L.tile0 + blockIdx.x) * kOctRec;
    if (rec[3] != 0) return;  // the block at group 0 clears its octet
    const InstDesc d = L.st.inst[rec[0]];
    const int c0 = 32 * rec[1] + 8 * rec[2];
    const int r = threadIdx.x;
    if (r < 8 && c0 + r < d.R) {
        L.st.E[d.rep_base + c0 + r] = 0;
        L.st.C[d.rep_base + c0 + r] = 0;
    }
}

}  // namespace

int32_t oct_lds_bytes(const InstDesc &d, int32_t ng, bool phase)
{
    return (int32_t)oct_layout(d, ng, phase).end;
}

hipError_t oct_kernels_set_lds(int32_t tile_bytes, int32_t phase_bytes)
{
    hipError_t e = hipSuccess;
    if (tile_bytes > 0)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&oct_tile_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, tile_bytes);
    if (e == hipSuccess && phase_bytes > 0)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&oct_phase_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, phase_bytes);
    return e;
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
