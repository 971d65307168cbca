// pt_kernels.hip -- gfx950 kernels of the parallel-tempering sampler.
//
//   init_spins     initial spins from INIT-domain Philox words
//   energy         E_cl and C of replicas from their spins in device memory
//   sweep_fast     n Metropolis sweeps of a tile of whole replicas held in LDS: one lane
//                  per (site, two words of four same-parity slices), byte-SWAR local
//                  fields (v_perm per neighbour), one Philox call per word and class;
//                  then E_cl and C from the byte field with v_dot4
//   sweep_block    sweeps of slice blocks of replicas too large for one workgroup's LDS
//                  (or whose rows need offsets beyond 16 bits): all sweeps of a call in
//                  one launch with every block resident, or one launch per sweep
//   sweep_generic  the same chain for any other shape (slice groups that are not a power
//                  of two, M = 1, large fields), one byte at a time
//   exchange       one even/odd replica-exchange step per instance (one workgroup each)
//   tau_corr       imaginary-time spin correlations of every replica, added per rung
//   advance        t += n
//
// The sweep kernels visit colour classes (slice parity p, spatial colour g) in order; a
// class is an independent set, so its sites are updated in parallel and the result is
// independent of the launch shape.
#include "pt_exchange.h"
#include "pt_xcd.h"
#include "pt_internal.h"

#pragma clang fp contract(off)

namespace ptq {

namespace {

constexpr int kWave = 64;

// A compile-time int as a value (to instantiate a generic lambda per degree or mode).
template <int V>
struct IntC {
    static constexpr int value = V;
};

__device__ __forceinline__ long long wave_sum(long long v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Sum over the workgroup; every thread gets the total.  scratch: >= blockDim/64 slots.
__device__ __forceinline__ long long block_sum(long long v, long long *scratch)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    long long tot = 0;
    for (int w = 0; w < nw; ++w) tot += scratch[w];
    __syncthreads();
    return tot;
}

__host__ __device__ __forceinline__ int64_t a16(int64_t x) { return (x + 15) & ~(int64_t)15; }

// Philox counter word 0 of the draws of (site i, parity p, slice group g4).
__device__ __forceinline__ uint32_t spin_ctr0(int i, int p, int G4, int g4)
{
    return (uint32_t)(2 * i + p) * (uint32_t)G4 + (uint32_t)g4;
}

__device__ __forceinline__ int ilog2(int v) { return 31 - __clz(v); }

// ------------------------------------------------------------------ init

__global__ void init_spins_kernel(DevState st, uint32_t key0, uint32_t key1)
{
    const int g = blockIdx.x;  // global replica
    const int n = st.rep_inst[g];
    const InstDesc d = st.inst[n];
    const int c = g - d.rep_base;
    uint8_t *base = st.spins + d.spin_base + (int64_t)c * d.rep_bytes;
    const int items = d.N * d.parities * d.G4;
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
        const int g4 = it % d.G4;
        const int ip = it / d.G4;
        const int p = ip % d.parities;
        const int i = ip / d.parities;
        const Words4 u = philox10(spin_ctr0(i, p, d.G4, g4), 0u, (uint32_t)c, (uint32_t)n, key0, key1);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int m = 4 * g4 + b;
            if (m < d.Mh) base[(int64_t)p * d.N * d.Mh + (int64_t)i * d.Mh + m] = (uint8_t)(u.w[b] >> 31);
        }
    }
}

// ------------------------------------------------------------------ energy from device memory

__device__ __forceinline__ int spin_of(const uint8_t *rep, const InstDesc &d, int k, int i)
{
    const int p = (d.M >= 2) ? (k & 1) : 0;
    const int m = (d.M >= 2) ? (k >> 1) : 0;
    return 2 * (int)rep[(int64_t)p * d.N * d.Mh + (int64_t)i * d.Mh + m] - 1;
}

__global__ void energy_kernel(DevState st, int32_t rep_first)
{
    __shared__ long long scratch[16];
    const int g = rep_first + blockIdx.x;
    const int n = st.rep_inst[g];
    const InstDesc d = st.inst[n];
    const int c = g - d.rep_base;
    const uint8_t *rep = st.spins + d.spin_base + (int64_t)c * d.rep_bytes;
    const int32_t *off = st.adj_off + d.off_base;
    const int32_t *adj = st.adj + d.adj_base;
    const int16_t *hf = st.hfield + d.site_base;
    long long e2 = 0, cc = 0;
    for (int it = threadIdx.x; it < d.M * d.N; it += blockDim.x) {
        const int k = it / d.N;
        const int i = it - k * d.N;
        const int s = spin_of(rep, d, k, i);
        int f = 2 * hf[i];
        for (int e = off[i]; e < off[i + 1]; ++e) {
            const int a = adj[e];
            f += (a >> 16) * spin_of(rep, d, k, a & 0xFFFF);
        }
        e2 += (long long)s * f;
        if (d.M >= 2) cc += (long long)s * spin_of(rep, d, (k + 1 == d.M) ? 0 : k + 1, i);
    }
    e2 = block_sum(e2, scratch);
    cc = block_sum(cc, scratch);
    if (threadIdx.x == 0) {
        st.E[g] = e2 / 2;
        st.C[g] = cc;
    }
}

// ------------------------------------------------------------------ tile staging

struct TileLds {
    uint8_t *sp;       // P replicas, rep_lds bytes each
    uint32_t *ent;     // fast: N * D entries
    uint32_t *bias;    // fast: N
    int32_t *adj;      // generic: neighbour entries
    int32_t *off;      // generic: N + 1
    int16_t *h;        // generic: N
    uint16_t *csite;   // N
    int32_t *coff;     // n_colors + 1
    uint32_t *tbl;     // P tables
    long long *red;    // reduction scratch
};

// Bytes between the replicas of a tile in LDS: N*M rounded up to whole words, then padded
// so that the word stride is congruent to the slice-group count G4 modulo 64.  The lanes
// of a wave run over (replica, slice group) with groups fastest, so replica q's words then
// start at bank q*G4 and a wave's row reads spread over all banks instead of piling the
// replicas onto the same ones (which an unpadded stride N*M/4 = 2*N*G4 words does).
__host__ __device__ __forceinline__ int64_t rep_lds_bytes(const InstDesc &d)
{
    int64_t w = ((int64_t)d.N * d.M + 3) >> 2;
    if (d.G4 >= 1 && d.G4 < 64) w += (((int64_t)d.G4 - w) % 64 + 64) % 64;
    return 4 * w;
}

// Shared by the host (to size the launch) and the kernels (to carve LDS).
__host__ __device__ __forceinline__ int64_t carve_offsets(const InstDesc &d, int n_adj, int P,
                                                          int64_t o[10])
{
    int64_t x = 0;
    o[0] = x; x = a16(x + (int64_t)P * rep_lds_bytes(d));
    o[1] = x; x = a16(x + (d.fast ? ent_words(d.N, d.D, d.ent_mode) * 4 : 0));
    o[2] = x; x = a16(x + (d.fast ? (int64_t)d.N * 4 : 0));
    o[3] = x; x = a16(x + (d.fast ? 0 : (int64_t)n_adj * 4));
    o[4] = x; x = a16(x + (d.fast ? 0 : (int64_t)(d.N + 1) * 4));
    o[5] = x; x = a16(x + (d.fast ? 0 : (int64_t)d.N * 2));
    o[6] = x; x = a16(x + (int64_t)d.N * 2);
    o[7] = x; x = a16(x + (int64_t)(d.n_colors + 1) * 4);
    o[8] = x; x = a16(x + (int64_t)P * d.tbl_words * 4);
    o[9] = x; x = a16(x + 2 * 16 * 8);
    return x;
}

__device__ __forceinline__ TileLds carve(char *lds, const InstDesc &d, int n_adj, int P)
{
    int64_t o[10];
    carve_offsets(d, n_adj, P, o);
    TileLds t;
    t.sp = reinterpret_cast<uint8_t *>(lds + o[0]);
    t.ent = reinterpret_cast<uint32_t *>(lds + o[1]);
    t.bias = reinterpret_cast<uint32_t *>(lds + o[2]);
    t.adj = reinterpret_cast<int32_t *>(lds + o[3]);
    t.off = reinterpret_cast<int32_t *>(lds + o[4]);
    t.h = reinterpret_cast<int16_t *>(lds + o[5]);
    t.csite = reinterpret_cast<uint16_t *>(lds + o[6]);
    t.coff = reinterpret_cast<int32_t *>(lds + o[7]);
    t.tbl = reinterpret_cast<uint32_t *>(lds + o[8]);
    t.red = reinterpret_cast<long long *>(lds + o[9]);
    return t;
}

// Copy the `words` words of each of P replicas between device memory (replicas
// rep_words_dev apart) and LDS (replicas rep_words_lds apart, the padded stride); both
// strides are at least `words`, so the LDS padding never reaches device memory.  The
// (replica, word) position of a thread advances by blockDim.x each step without a
// division; when the word count and both strides are multiples of 4 the copy moves 16
// bytes per access.
template <bool IN>
__device__ __forceinline__ void copy_spins(uint32_t *lds_sp, uint32_t *dev, int P,
                                           int rep_words_dev, int rep_words_lds, int words)
{
    const int nt = blockDim.x;
    if (((words | rep_words_dev | rep_words_lds) & 3) == 0) {
        const int wv = words >> 2, dv = rep_words_dev >> 2, lv = rep_words_lds >> 2;
        uint4 *L4 = reinterpret_cast<uint4 *>(lds_sp);
        uint4 *D4 = reinterpret_cast<uint4 *>(dev);
        const int qs = nt / wv, rs = nt - qs * wv;
        int q = threadIdx.x / wv, r = threadIdx.x - q * wv;
        for (; q < P;) {
            if (IN)
                L4[q * lv + r] = D4[(int64_t)q * dv + r];
            else
                D4[(int64_t)q * dv + r] = L4[q * lv + r];
            q += qs;
            r += rs;
            if (r >= wv) {
                r -= wv;
                ++q;
            }
        }
    } else {
        const int qs = nt / words, rs = nt - qs * words;
        int q = threadIdx.x / words, r = threadIdx.x - q * words;
        for (; q < P;) {
            if (IN)
                lds_sp[q * rep_words_lds + r] = dev[(int64_t)q * rep_words_dev + r];
            else
                dev[(int64_t)q * rep_words_dev + r] = lds_sp[q * rep_words_lds + r];
            q += qs;
            r += rs;
            if (r >= words) {
                r -= words;
                ++q;
            }
        }
    }
}

// The threshold tables of the rungs that P consecutive replicas sit on, in one flat loop
// so that the rung lookups of all replicas are in flight together.
__device__ __forceinline__ void stage_tables(const DevState &st, const InstDesc &d, int c0, int P,
                                             uint32_t *dst)
{
    const int tw = d.tbl_words, nt = blockDim.x;
    const int qs = nt / tw, ks = nt - qs * tw;
    int q = threadIdx.x / tw, k = threadIdx.x - q * tw;
    for (; q < P;) {
        const int rung = st.rung_of[d.rep_base + c0 + q];
        dst[q * tw + k] = st.tbl[d.tbl_base + (int64_t)rung * tw + k];
        q += qs;
        k += ks;
        if (k >= tw) {
            k -= tw;
            ++q;
        }
    }
}

__device__ __forceinline__ void stage_common(const DevState &st, const InstDesc &d, int n,
                                             const Tile &tile, const TileLds &t, int n_adj)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(
        st.spins + d.spin_base + (int64_t)tile.c0 * d.rep_bytes);
    copy_spins<true>(reinterpret_cast<uint32_t *>(t.sp), const_cast<uint32_t *>(src), tile.P,
                     d.rep_bytes / 4, (int)(rep_lds_bytes(d) / 4), (d.N * d.M + 3) / 4);
    for (int i = tid; i < d.N; i += nt) t.csite[i] = st.csite[d.site_base + i];
    for (int g = tid; g <= d.n_colors; g += nt) t.coff[g] = st.cls_off[d.cls_base + g];
    stage_tables(st, d, tile.c0, tile.P, t.tbl);
    if (d.fast) {
        const int ew = (int)ent_words(d.N, d.D, d.ent_mode);
        for (int e = tid; e < ew; e += nt) t.ent[e] = st.ent[d.ent_base + e];
        for (int i = tid; i < d.N; i += nt) t.bias[i] = st.bias[d.site_base + i];
    } else {
        for (int e = tid; e < n_adj; e += nt) t.adj[e] = st.adj[d.adj_base + e];
        for (int i = tid; i <= d.N; i += nt) t.off[i] = st.adj_off[d.off_base + i];
        for (int i = tid; i < d.N; i += nt) t.h[i] = st.hfield[d.site_base + i];
    }
    (void)n;
}

__device__ __forceinline__ void write_back(const DevState &st, const InstDesc &d,
                                           const Tile &tile, const TileLds &t)
{
    uint32_t *dst = reinterpret_cast<uint32_t *>(st.spins + d.spin_base +
                                                 (int64_t)tile.c0 * d.rep_bytes);
    copy_spins<false>(reinterpret_cast<uint32_t *>(t.sp), dst, tile.P, d.rep_bytes / 4,
                      (int)(rep_lds_bytes(d) / 4), (d.N * d.M + 3) / 4);
}

// s_waitcnt immediate with the vector-memory count 0 and the export and LDS counts at
// their maxima (no wait on them): vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8.
constexpr int kWaitVmcnt0 = 0x0F70;

// End of a tile in a PT cycle: count the tile for its instance and, in the workgroup that
// completes the instance, run the instance's exchange step.  Every tile's spins and
// energies are written before its count (agent-scope release), and the completing
// workgroup acquires them before it reads the energies; nothing ever waits on another
// workgroup.  The completing workgroup also clears the count for the next call.  flag: one
// word of the tile's LDS scratch (no static LDS, which would add to every tile's footprint).
__device__ __forceinline__ void finish_tile(const SweepLaunch &L, const DevState &st, int n,
                                            long long *flag)
{
    // every wave's stores complete (a workgroup barrier does not wait for them), then thread
    // 0 writes the XCD's L2 back and waits for that write-back before it counts the tile
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        __builtin_amdgcn_s_waitcnt(0);
        const uint32_t before = atomicAdd(&st.icount[n], 1u);
        const int done = (before + 1u == (uint32_t)st.itiles[n]) ? 1 : 0;
        if (done) st.icount[n] = 0;
        *flag = done;
    }
    __syncthreads();
    if (*flag) {
        __threadfence();
        exchange_instance(st, n, L.swap_key0, L.swap_key1, L.t_add);
    }
}

// ------------------------------------------------------------------ fast sweep

__device__ __forceinline__ uint32_t lds32(const uint8_t *base, uint32_t byte_off)
{
    return *reinterpret_cast<const uint32_t *>(base + byte_off);
}

// NW consecutive words at an offset that is a multiple of 4 * NW (one ds_read_b64 for two)
template <int NW>
__device__ __forceinline__ void ldsw(const uint8_t *base, uint32_t byte_off, uint32_t (&w)[NW])
{
    if constexpr (NW == 2) {
        const uint2 v = *reinterpret_cast<const uint2 *>(base + byte_off);
        w[0] = v.x;
        w[1] = v.y;
    } else {
        w[0] = lds32(base, byte_off);
    }
}

template <int NW>
__device__ __forceinline__ void stsw(uint8_t *base, uint32_t byte_off, const uint32_t (&w)[NW])
{
    if constexpr (NW == 2)
        *reinterpret_cast<uint2 *>(base + byte_off) = make_uint2(w[0], w[1]);
    else
        *reinterpret_cast<uint32_t *>(base + byte_off) = w[0];
}

__device__ __forceinline__ uint32_t popc(uint32_t x) { return (uint32_t)__popc(x); }

// Per-launch constants of a fast tile.
struct FastArgs {
    uint32_t key0, key1, tt, n, c0;
    uint32_t NMh;       // bytes of one parity plane of a replica
    uint32_t rs;        // bytes between replicas in LDS
    uint32_t sel_x;     // v_perm selector: x -> x * (2F + 1)
    int G4, lgG4, lgMh, tbl_words;
};

// Neighbour entry e of site i's row in LDS as (byte offset of the neighbour's row within a
// parity plane, weight word): the weight word is the entry itself under kEntPerm (its low
// bytes are the v_perm table w0, w1), and the mask m = 0x01010101 [J < 0] under kEntXad16.
template <int EM>
__device__ __forceinline__ void fast_entry(const uint32_t *ent, int idx, uint32_t &off, uint32_t &w)
{
    if constexpr (EM == kEntXad16) {
        const uint32_t v = reinterpret_cast<const uint16_t *>(ent)[idx];
        off = v & 0x7FFFu;
        w = __builtin_amdgcn_perm(0u, v >> 15, 0u);
    } else {
        const uint32_t v = ent[idx];
        off = v >> 16;
        w = v;
    }
}

// acc + the weighted neighbour bytes of word y (w from fast_entry).
template <int EM>
__device__ __forceinline__ uint32_t fast_add(uint32_t acc, uint32_t w, uint32_t y)
{
    if constexpr (EM == kEntPerm)
        return acc + __builtin_amdgcn_perm(0u, w, y);
    else
        return (y ^ w) + acc;  // v_xad_u32
}

// A lane's own words X (slice groups g4 .. g4 + NW - 1 of parity PAR at byte offset own)
// and their time fields: byte b of T[k] is x(2m+PAR-1) + x(2m+PAR+1), read from the other
// parity's row at oth_row.
template <int NW, int PAR>
__device__ __forceinline__ void fast_own_time(const FastArgs &a, const TileLds &t, uint32_t own,
                                              uint32_t oth_row, int g4, uint32_t (&X)[NW],
                                              uint32_t (&T)[NW])
{
    const int G4 = a.G4;
    uint32_t Wc[NW];
    ldsw<NW>(t.sp, own, X);
    ldsw<NW>(t.sp, oth_row + 4u * (uint32_t)g4, Wc);
    if constexpr (PAR == 0) {
        const uint32_t Wp = lds32(t.sp, oth_row + 4u * (uint32_t)((g4 - 1) & (G4 - 1)));
        T[0] = __builtin_amdgcn_alignbyte(Wc[0], Wp, 3) + Wc[0];
        if constexpr (NW == 2) T[1] = __builtin_amdgcn_alignbyte(Wc[1], Wc[0], 3) + Wc[1];
    } else {
        const uint32_t Wn = lds32(t.sp, oth_row + 4u * (uint32_t)((g4 + NW) & (G4 - 1)));
        if constexpr (NW == 2) {
            T[0] = __builtin_amdgcn_alignbyte(Wc[1], Wc[0], 1) + Wc[0];
            T[1] = __builtin_amdgcn_alignbyte(Wn, Wc[1], 1) + Wc[1];
        } else {
            T[0] = __builtin_amdgcn_alignbyte(Wn, Wc[0], 1) + Wc[0];
        }
    }
}

// The updated words of a lane: per slice byte, the table index 3V + tau with
// V = x(2F+1) + f + F (f from the weighted neighbour count acc and the bias) selects the
// replica's threshold in tb, and the byte flips when the draw is at most that threshold.
// draw(k) gives the Philox words of word k.
template <int NW, typename Draw>
__device__ __forceinline__ void fast_flip(const FastArgs &a, const uint32_t *tb, const uint32_t (&X)[NW],
                                          const uint32_t (&acc)[NW], const uint32_t (&T)[NW],
                                          uint32_t bias, Draw draw, uint32_t (&out)[NW])
{
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const Words4 u = draw(k);
        const uint32_t V = __builtin_amdgcn_perm(0u, a.sel_x, X[k]) + (acc[k] << 1) + bias;
        const uint32_t IDX = V + (V << 1) + T[k];  // 3V + tau in every byte
        uint32_t flip = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t thr = tb[(IDX >> (8 * b)) & 0xFFu];
            flip |= (u.w[b] <= thr ? 1u : 0u) << (8 * b);
        }
        out[k] = X[k] ^ flip;
    }
}

// One lane's update of site i, replica q, slice groups g4 .. g4 + NW - 1 of parity PAR:
// 4 * NW Metropolis attempts served by NW Philox calls.  DT > 0 fixes the (padded) degree
// at compile time so the neighbour loads are issued together; EM is the instance's
// EntMode.
template <int DT, int NW, int PAR, int EM>
__device__ __forceinline__ void fast_item(const FastArgs &a, const TileLds &t, int D, int i,
                                          int q, int g4)
{
    const uint32_t qbase = (uint32_t)q * a.rs;
    const uint32_t irow = (uint32_t)i << a.lgMh;
    const uint32_t nb_base = qbase + (uint32_t)PAR * a.NMh + 4u * (uint32_t)g4;
    const uint32_t own = nb_base + irow;
    const uint32_t oth_row = qbase + (uint32_t)(PAR ^ 1) * a.NMh + irow;
    uint32_t X[NW], T[NW];
    fast_own_time<NW, PAR>(a, t, own, oth_row, g4, X, T);
    // weighted count of neighbours per slice byte
    const int e0 = i * D;
    uint32_t acc[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) acc[k] = 0;
    if constexpr (DT > 0) {
        uint32_t offs[DT], wts[DT], ws[DT][NW];
#pragma unroll
        for (int e = 0; e < DT; ++e) fast_entry<EM>(t.ent, e0 + e, offs[e], wts[e]);
#pragma unroll
        for (int e = 0; e < DT; ++e) ldsw<NW>(t.sp, nb_base + offs[e], ws[e]);
#pragma unroll
        for (int e = 0; e < DT; ++e)
#pragma unroll
            for (int k = 0; k < NW; ++k) acc[k] = fast_add<EM>(acc[k], wts[e], ws[e][k]);
    } else {
        for (int e = 0; e < D; ++e) {
            uint32_t off, wt, w[NW];
            fast_entry<EM>(t.ent, e0 + e, off, wt);
            ldsw<NW>(t.sp, nb_base + off, w);
#pragma unroll
            for (int k = 0; k < NW; ++k) acc[k] = fast_add<EM>(acc[k], wt, w[k]);
        }
    }
    const uint32_t ctr = ((uint32_t)(2 * i + PAR) << a.lgG4) + (uint32_t)g4;
    uint32_t out[NW];
    fast_flip<NW>(a, t.tbl + q * a.tbl_words, X, acc, T, t.bias[i],
                  [&](int k) { return philox10(ctr + (uint32_t)k, a.tt, a.c0 + (uint32_t)q, a.n, a.key0, a.key1); },
                  out);
    stsw<NW>(t.sp, own, out);
}

// The items of colour class g of parity PAR, with no closing barrier.  A class holds
// ns sites x P replicas x G4/NW lanes; lanes run over slice groups fastest, so the lanes of
// a site read one neighbour row entry (broadcast) and consecutive words of each neighbour row.
template <int DT, int NW, int PAR, int EM>
__device__ __forceinline__ void fast_class(const FastArgs &a, const InstDesc &d, const TileLds &t,
                                           int lgGW, int lgL, int g)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int Lmask = (1 << lgL) - 1;
    const int D = (DT > 0) ? DT : d.D;
    if ((1 << lgL) <= nt) {
        // every thread keeps one (replica, lane group) and strides over the sites; threads
        // past the last whole site row (block sizes that are not powers of two) stay idle
        const int r = tid & Lmask;
        const int q = r >> lgGW;
        const int g4 = NW * (r & ((1 << lgGW) - 1));
        const int sstep = nt >> lgL;
        const int s_first = (tid < (sstep << lgL)) ? (tid >> lgL) : (1 << 30);
        const int s1 = t.coff[g + 1];
        for (int si = t.coff[g] + s_first; si < s1; si += sstep)
            fast_item<DT, NW, PAR, EM>(a, t, D, t.csite[si], q, g4);
    } else {
        const int s0 = t.coff[g];
        const int items = (t.coff[g + 1] - s0) << lgL;
        for (int it = tid; it < items; it += nt) {
            const int r = it & Lmask;
            fast_item<DT, NW, PAR, EM>(a, t, D, t.csite[s0 + (it >> lgL)], r >> lgGW,
                                       NW * (r & ((1 << lgGW) - 1)));
        }
    }
}

// All colour classes of parity PAR, one barrier after each.
template <int DT, int NW, int PAR, int EM>
__device__ __forceinline__ void fast_phase(const FastArgs &a, const InstDesc &d, const TileLds &t,
                                           int lgGW, int lgL)
{
    for (int g = 0; g < d.n_colors; ++g) {
        fast_class<DT, NW, PAR, EM>(a, d, t, lgGW, lgL, g);
        __syncthreads();
    }
}

// ------------------------------------------------------------------ latency path
//
// A batch of at most one tile per compute unit leaves each tile's sweep a chain of short
// class steps that no other workgroup overlaps.  Two things shorten that chain:
//  * Class k of parity 0 and class k - 1 of parity 1 (k - 1 taken mod the class count, and
//    from the previous sweep when k = 0) touch disjoint words: each writes its own sites'
//    slices of its parity and reads the other parity only at those sites, while the classes
//    are different, so no site is in both.  Every update still reads exactly the values it
//    reads in the plain order (all parity-0 classes, then all parity-1 classes), so the
//    chain is unchanged, and a sweep takes one step per class instead of two.
//  * The spin-independent part of a thread's next item (site, neighbour entries, bias and
//    Philox words) is formed while the current item's loads and lookups are in flight.
// Waves with no item in a step skip it.  Needs two classes at least and every step's
// items within one pass of the workgroup (one item per thread).

// Per-thread constants: replica q and first slice group g4 of the thread's items, its site
// slot within a step, and whether any lane of its wave has an item in a step starting at a
// given site slot (the wave's first slot).
struct LatLane {
    int q, g4, s, wave_s;
    uint32_t qbase;
    const uint32_t *tb;
};

// The spin-independent part of a thread's item: parity par, site row irow, entries, bias
// and draws (on = false: no item; it then stands on site 0 and stores nothing).
template <int DT, int NW>
struct LatItem {
    uint32_t irow, par;
    uint32_t off[DT], wt[DT];
    uint32_t bias;
    Words4 u[NW];
    bool on;
};

// Step (sw, k) holds class k of parity 0 at sweep sw (when sw < n_sweeps) followed, in
// lane order, by class k - 1 of parity 1 at sweep sw - [k == 0] (when that sweep is in
// range).  Sites of the step before the thread's slot: nA of the first part, nB of both.
struct LatStep {
    int a0, nA, b0, nB, swB;
};

__device__ __forceinline__ LatStep lat_step(const TileLds &t, int nc, int n_sweeps, int sw, int k)
{
    LatStep z;
    const int kB = (k == 0 ? nc : k) - 1;
    z.swB = sw - (k == 0 ? 1 : 0);
    // class bounds are the same in every lane: keep them scalar
    z.a0 = __builtin_amdgcn_readfirstlane(t.coff[k]);
    const int a1 = __builtin_amdgcn_readfirstlane(t.coff[k + 1]);
    z.b0 = __builtin_amdgcn_readfirstlane(t.coff[kB]);
    const int b1 = __builtin_amdgcn_readfirstlane(t.coff[kB + 1]);
    z.nA = sw < n_sweeps ? a1 - z.a0 : 0;
    z.nB = (z.swB >= 0 && z.swB < n_sweeps) ? b1 - z.b0 : 0;
    return z;
}

template <int DT, int NW, int EM>
__device__ __forceinline__ void lat_prep(const FastArgs &a, const TileLds &t, const LatLane &ln,
                                         const LatStep &z, uint64_t t0, int sw, LatItem<DT, NW> &p)
{
    const bool inA = ln.s < z.nA;
    p.on = ln.s < z.nA + z.nB;
    p.par = inA ? 0u : 1u;
    const int i = t.csite[inA ? z.a0 + ln.s : p.on ? z.b0 + ln.s - z.nA : 0];
    const uint32_t tt = (uint32_t)(t0 + (uint64_t)(inA ? sw : z.swB));
    p.irow = (uint32_t)i << a.lgMh;
#pragma unroll
    for (int e = 0; e < DT; ++e) fast_entry<EM>(t.ent, i * DT + e, p.off[e], p.wt[e]);
    p.bias = t.bias[i];
    const uint32_t ctr = (((uint32_t)(2 * i) + p.par) << a.lgG4) + (uint32_t)ln.g4;
#pragma unroll
    for (int k = 0; k < NW; ++k)
        p.u[k] = philox10(ctr + (uint32_t)k, tt, a.c0 + (uint32_t)ln.q, a.n, a.key0, a.key1);
}

// The spin-dependent part: fast_item's update, with the parity taken per lane.
template <int DT, int NW, int EM>
__device__ __forceinline__ void lat_apply(const FastArgs &a, const TileLds &t, const LatLane &ln,
                                          const LatItem<DT, NW> &p)
{
    const int G4 = a.G4, g4 = ln.g4;
    const uint32_t nb_base = ln.qbase + (p.par ? a.NMh : 0u) + 4u * (uint32_t)g4;
    const uint32_t own = nb_base + p.irow;
    const uint32_t oth_row = ln.qbase + (p.par ? 0u : a.NMh) + p.irow;
    uint32_t X[NW], Wc[NW], T[NW], acc[NW], ws[DT][NW], out[NW];
    ldsw<NW>(t.sp, own, X);
    ldsw<NW>(t.sp, oth_row + 4u * (uint32_t)g4, Wc);
    // the other parity's word before the lane's (parity 0) or after it (parity 1)
    const uint32_t Wx = lds32(t.sp, oth_row + 4u * (uint32_t)((g4 + (p.par ? NW : -1)) & (G4 - 1)));
#pragma unroll
    for (int e = 0; e < DT; ++e) ldsw<NW>(t.sp, nb_base + p.off[e], ws[e]);
    if constexpr (NW == 2) {
        T[0] = (p.par ? __builtin_amdgcn_alignbyte(Wc[1], Wc[0], 1)
                      : __builtin_amdgcn_alignbyte(Wc[0], Wx, 3)) + Wc[0];
        T[1] = (p.par ? __builtin_amdgcn_alignbyte(Wx, Wc[1], 1)
                      : __builtin_amdgcn_alignbyte(Wc[1], Wc[0], 3)) + Wc[1];
    } else {
        T[0] = (p.par ? __builtin_amdgcn_alignbyte(Wx, Wc[0], 1)
                      : __builtin_amdgcn_alignbyte(Wc[0], Wx, 3)) + Wc[0];
    }
#pragma unroll
    for (int k = 0; k < NW; ++k) acc[k] = 0;
#pragma unroll
    for (int e = 0; e < DT; ++e)
#pragma unroll
        for (int k = 0; k < NW; ++k) acc[k] = fast_add<EM>(acc[k], p.wt[e], ws[e][k]);
    fast_flip<NW>(a, ln.tb, X, acc, T, p.bias, [&](int k) { return p.u[k]; }, out);
    if (p.on) stsw<NW>(t.sp, own, out);
}

// n_sweeps sweeps of a tile on the latency path (the caller checked that it applies).
template <int DT, int NW, int EM>
__device__ __forceinline__ void lat_sweeps(const FastArgs &a, const InstDesc &d, const TileLds &t,
                                           int lgGW, int lgL, int n_sweeps, uint64_t t0)
{
    const int tid = threadIdx.x;
    LatLane ln;
    const int r = tid & ((1 << lgL) - 1);
    ln.q = r >> lgGW;
    ln.g4 = NW * (r & ((1 << lgGW) - 1));
    ln.s = tid >> lgL;
    ln.wave_s = __builtin_amdgcn_readfirstlane(tid >> lgL);  // lane 0's slot: the wave's first
    ln.qbase = (uint32_t)ln.q * a.rs;
    ln.tb = t.tbl + ln.q * a.tbl_words;
    const int nc = d.n_colors;
    const int steps = nc * n_sweeps + 1;
    LatItem<DT, NW> cur, nxt;
    LatStep z = lat_step(t, nc, n_sweeps, 0, 0);
    bool wcur = ln.wave_s < z.nA + z.nB;
    if (wcur) lat_prep<DT, NW, EM>(a, t, ln, z, t0, 0, cur);
    int sw = 0, k = 0;
    for (int step = 0; step < steps; ++step) {
        if (++k == nc) {
            k = 0;
            ++sw;
        }
        z = lat_step(t, nc, n_sweeps, sw, k);
        const bool wnext = ln.wave_s < z.nA + z.nB;
        if (wcur && wnext) {
            lat_prep<DT, NW, EM>(a, t, ln, z, t0, sw, nxt);
            lat_apply<DT, NW, EM>(a, t, ln, cur);
        } else if (wcur) {
            lat_apply<DT, NW, EM>(a, t, ln, cur);
        } else if (wnext) {
            lat_prep<DT, NW, EM>(a, t, ln, z, t0, sw, nxt);
        }
        __syncthreads();
        cur = nxt;
        wcur = wnext;
    }
}

// Whether a tile takes the latency path with this workgroup: two classes at least, and
// every step's sites (class k plus class k - 1, cyclically) within one pass.
__device__ __forceinline__ bool lat_fits(const InstDesc &d, const TileLds &t, int lgL)
{
    const int nc = d.n_colors;
    if (nc < 2 || (1 << lgL) > (int)blockDim.x) return false;
    int most = 0;
    for (int k = 0; k < nc; ++k) {
        const int kB = (k == 0 ? nc : k) - 1;
        most = max(most, t.coff[k + 1] - t.coff[k] + t.coff[kB + 1] - t.coff[kB]);
    }
    return most <= ((int)blockDim.x >> lgL);
}

template <int DT, int NW, bool WIDE, bool LAT>
__device__ __forceinline__ void fast_sweeps(const SweepLaunch &L, const InstDesc &d,
                                            const Tile &tile, const TileLds &t, uint64_t t0)
{
    FastArgs a;
    a.key0 = L.key0;
    a.key1 = L.key1;
    a.n = (uint32_t)tile.inst;
    a.c0 = (uint32_t)tile.c0;
    a.NMh = (uint32_t)(d.N * d.Mh);
    a.rs = (uint32_t)rep_lds_bytes(d);
    a.sel_x = (uint32_t)(2 * d.F + 1) << 8;
    a.G4 = d.G4;
    a.lgG4 = ilog2(d.G4);
    a.lgMh = ilog2(d.Mh);
    a.tbl_words = d.tbl_words;
    const int lgGW = ilog2(d.G4 / NW);
    const int lgL = ilog2(tile.P) + lgGW;  // lanes per site: P * G4 / NW
    bool lat = false;
    if constexpr (LAT && DT > 0) lat = lat_fits(d, t, lgL);
    auto run = [&](auto em) {
        constexpr int EM = decltype(em)::value;
        if constexpr (LAT && DT > 0) {
            if (lat) {
                lat_sweeps<DT, NW, EM>(a, d, t, lgGW, lgL, L.n_sweeps, t0);
                return;
            }
        }
        const int nc = d.n_colors;
        if (nc < 2) {
            for (int sw = 0; sw < L.n_sweeps; ++sw) {
                a.tt = (uint32_t)(t0 + (uint64_t)sw);
                fast_phase<DT, NW, 0, EM>(a, d, t, lgGW, lgL);
                fast_phase<DT, NW, 1, EM>(a, d, t, lgGW, lgL);
            }
            return;
        }
        // class k of parity 0 with class k - 1 of parity 1 (from the previous sweep when
        // k = 0; the order of the latency path below), one barrier per step; the step after
        // the last sweep finishes its last parity-1 class
        FastArgs b = a;
        for (int sw = 0; sw <= L.n_sweeps; ++sw) {
            const bool tail = sw == L.n_sweeps;
            for (int k = 0; k < (tail ? 1 : nc); ++k) {
                if (!tail) {
                    a.tt = (uint32_t)(t0 + (uint64_t)sw);
                    fast_class<DT, NW, 0, EM>(a, d, t, lgGW, lgL, k);
                }
                if (k > 0 || sw > 0) {
                    b.tt = (uint32_t)(t0 + (uint64_t)(sw - (k == 0)));
                    fast_class<DT, NW, 1, EM>(b, d, t, lgGW, lgL, k > 0 ? k - 1 : nc - 1);
                }
                __syncthreads();
            }
        }
    };
    // 16-bit entries are only used with two words per lane and rows of at least four
    // entries (the large replicas they are meant for; the host guarantees it), so only
    // those instantiations carry them
    constexpr bool k16 = WIDE && NW == 2 && (DT == 0 || DT >= 4);
    if (k16 && d.ent_mode == kEntXad16)
        run(IntC<k16 ? kEntXad16 : kEntPerm>{});
    else
        run(IntC<kEntPerm>{});
}

// WIDE: the instantiation carries the kEntXad16 form.  The multi-cycle kernel does not
// (with it it would need more registers than its four waves per SIMD allow): its instances
// fit one tile each, which kEntXad16 instances never do.
template <int NW, bool WIDE, bool LAT = false>
__device__ __forceinline__ void fast_dispatch(const SweepLaunch &L, const InstDesc &d,
                                              const Tile &tile, const TileLds &t, uint64_t t0)
{
    switch (d.D) {
    case 1: fast_sweeps<1, NW, WIDE, LAT>(L, d, tile, t, t0); break;
    case 2: fast_sweeps<2, NW, WIDE, LAT>(L, d, tile, t, t0); break;
    case 3: fast_sweeps<3, NW, WIDE, LAT>(L, d, tile, t, t0); break;
    case 4: fast_sweeps<4, NW, WIDE, LAT>(L, d, tile, t, t0); break;
    case 5: fast_sweeps<5, NW, WIDE, LAT>(L, d, tile, t, t0); break;
    case 6: fast_sweeps<6, NW, WIDE, LAT>(L, d, tile, t, t0); break;
    case 7: fast_sweeps<7, NW, WIDE, LAT>(L, d, tile, t, t0); break;
    case 8: fast_sweeps<8, NW, WIDE, LAT>(L, d, tile, t, t0); break;
    default: fast_sweeps<0, NW, WIDE, LAT>(L, d, tile, t, t0); break;
    }
}

// Entry idx of a fast tile's neighbour rows in the 32-bit form (offset << 16 | w1 << 8 | w0)
// whatever the instance's EntMode (a uniform branch; the energy pass runs once per call).
__device__ __forceinline__ uint32_t fast_entry32(const InstDesc &d, const uint32_t *ent, int idx)
{
    if (d.ent_mode == kEntXad16) {
        const uint32_t v = reinterpret_cast<const uint16_t *>(ent)[idx];
        return ((v & 0x7FFFu) << 16) | ((v >> 15) ? 0x0001u : 0x0100u);
    }
    return ent[idx];
}

// E_cl and C of every replica of a fast tile from its final spins.  Per site and group of
// eight slices (two words, one per parity) the byte field g = f + F = 2 A + bias is formed
// as in the sweep, and 2E over the eight slices is sum_b (2 x_b - 1)(g_b - F + h), taken with
// two v_dot4_u32_u8; h - F = bias - 2F + sum |J|, and each entry's two weight bytes sum to
// its |J|.  C comes from popcounts of x xor (x shifted one slice in time).  Replicas are
// dealt to groups of waves (one wave each when the tile has at least as many replicas as
// the workgroup has waves), so the reductions need at most one workgroup barrier.
template <int DT>
__device__ __forceinline__ void fast_energy(const DevState &st, const InstDesc &d, const Tile &tile,
                                            const TileLds &t)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int N = d.N, Mh = d.Mh, G4 = d.G4, F = d.F;
    const int D = (DT > 0) ? DT : d.D;
    const uint32_t RSq = (uint32_t)rep_lds_bytes(d), NMh = (uint32_t)(N * Mh);
    const int lgG4 = ilog2(G4);
    const int lane = tid & (kWave - 1), wid = tid / kWave, nw = nt / kWave;
    const int wpr = nw > tile.P ? nw / tile.P : 1;   // waves per replica
    const int ngroups = nw / wpr;
    const int grp = wid / wpr, sub = wid - grp * wpr;
    for (int q = grp; q < tile.P; q += ngroups) {
        // per lane in 32 bits (a replica of the fast path holds at most 2^14 items of
        // eight slices, each contributing |2E| <= 8 * 6F and |C| <= 8)
        int e2 = 0, c1 = 0;
        const uint32_t qbase = (uint32_t)q * RSq;
        for (int it = sub * kWave + lane; it < N * G4; it += wpr * kWave) {
            const int i = it >> lgG4;
            const int g4 = it & (G4 - 1);
            const uint32_t row = qbase + (uint32_t)(i * Mh);
            const uint32_t X0 = lds32(t.sp, row + 4u * (uint32_t)g4);
            const uint32_t X1 = lds32(t.sp, row + NMh + 4u * (uint32_t)g4);
            const uint32_t X0n = lds32(t.sp, row + 4u * (uint32_t)((g4 + 1) & (G4 - 1)));
            // time bonds (2m, 2m+1) and (2m+1, 2m+2): 8 per group
            const int dis_t = (int)(popc(X0 ^ X1) + popc(X1 ^ __builtin_amdgcn_alignbyte(X0n, X0, 1)));
            c1 += 8 - 2 * dis_t;
            const uint32_t nb = qbase + 4u * (uint32_t)g4;
            uint32_t A0 = 0, A1 = 0, sumJ = 0;
            if constexpr (DT > 0) {
                uint32_t ents[DT], y0[DT], y1[DT];
#pragma unroll
                for (int e = 0; e < DT; ++e) ents[e] = fast_entry32(d, t.ent, i * D + e);
#pragma unroll
                for (int e = 0; e < DT; ++e) {
                    y0[e] = lds32(t.sp, nb + (ents[e] >> 16));
                    y1[e] = lds32(t.sp, nb + (ents[e] >> 16) + NMh);
                }
#pragma unroll
                for (int e = 0; e < DT; ++e) {
                    A0 += __builtin_amdgcn_perm(0u, ents[e], y0[e]);
                    A1 += __builtin_amdgcn_perm(0u, ents[e], y1[e]);
                    sumJ = __builtin_amdgcn_udot4(ents[e], 0x00000101u, sumJ, false);
                }
            } else {
                for (int e = 0; e < D; ++e) {
                    const uint32_t ent = fast_entry32(d, t.ent, i * D + e);
                    A0 += __builtin_amdgcn_perm(0u, ent, lds32(t.sp, nb + (ent >> 16)));
                    A1 += __builtin_amdgcn_perm(0u, ent, lds32(t.sp, nb + (ent >> 16) + NMh));
                    sumJ = __builtin_amdgcn_udot4(ent, 0x00000101u, sumJ, false);
                }
            }
            const uint32_t bias = t.bias[i];
            const uint32_t G0 = (A0 << 1) + bias, G1 = (A1 << 1) + bias;
            const int hF = (int)(bias & 0xFFu) + (int)sumJ - 2 * F;  // h - F
            const int dot = (int)__builtin_amdgcn_udot4(X0, G0, __builtin_amdgcn_udot4(X1, G1, 0u, false), false);
            const int gs = (int)__builtin_amdgcn_udot4(0x01010101u, G0,
                                                       __builtin_amdgcn_udot4(0x01010101u, G1, 0u, false), false);
            const int pc = (int)(popc(X0) + popc(X1));
            e2 += 2 * dot + 2 * hF * pc - gs - 8 * hF;
        }
        long long ee = wave_sum((long long)e2), cc = wave_sum((long long)c1);
        if (wpr == 1) {
            if (lane == 0) {
                st.E[d.rep_base + tile.c0 + q] = ee / 2;
                st.C[d.rep_base + tile.c0 + q] = cc;
            }
        } else if (lane == 0) {
            t.red[2 * wid] = ee;
            t.red[2 * wid + 1] = cc;
        }
    }
    if (wpr > 1) {
        // every group holds exactly one replica here (tile.P < nw)
        __syncthreads();
        if (sub == 0 && lane == 0 && grp < tile.P) {
            long long ee = 0, cc = 0;
            for (int w = wid; w < wid + wpr; ++w) {
                ee += t.red[2 * w];
                cc += t.red[2 * w + 1];
            }
            st.E[d.rep_base + tile.c0 + grp] = ee / 2;
            st.C[d.rep_base + tile.c0 + grp] = cc;
        }
    }
}

// MULTI: a fused launch of L.cycles PT cycles (its own instantiation, bounded at four
// waves per SIMD: the exchange step in the loop needs more registers than eight allow).
// LAT: the latency path for tiles whose colour classes fit one pass of the workgroup (its
// own instantiation at four waves per SIMD, for batches of at most one tile per unit).
template <bool FUSE, bool MULTI = false, bool LAT = false>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(MULTI || LAT ? 4 : 8))) sweep_fast_kernel(SweepLaunch L)
{
    extern __shared__ __align__(16) char lds[];
    const DevState &st = L.st;
    const Tile tile = st.tiles[L.tile0 + blockIdx.x];
    const int n = tile.inst;
    const InstDesc d = st.inst[n];
    TileLds t = carve(lds, d, 0, tile.P);
    stage_common(st, d, n, tile, t, 0);
    uint64_t t0 = st.ctr[n].t;
    __syncthreads();

    // With MULTI (fused launches whose tiles each hold a whole instance) the workgroup
    // runs L.cycles PT cycles: after each but the last it does the instance's exchange
    // step itself, with the replicas still in LDS, then stages the threshold tables of
    // the replicas' new rungs and reads the advanced sweep counter.
    for (int cyc = 0;; ++cyc) {
        if (L.lane_words == 2 && d.G4 >= 2)
            fast_dispatch<2, !MULTI, LAT>(L, d, tile, t, t0);
        else
            fast_dispatch<1, !MULTI, LAT>(L, d, tile, t, t0);

        switch (d.D) {
        case 1: fast_energy<1>(st, d, tile, t); break;
        case 2: fast_energy<2>(st, d, tile, t); break;
        case 3: fast_energy<3>(st, d, tile, t); break;
        case 4: fast_energy<4>(st, d, tile, t); break;
        case 5: fast_energy<5>(st, d, tile, t); break;
        case 6: fast_energy<6>(st, d, tile, t); break;
        case 7: fast_energy<7>(st, d, tile, t); break;
        case 8: fast_energy<8>(st, d, tile, t); break;
        default: fast_energy<0>(st, d, tile, t); break;
        }
        if (!(FUSE && MULTI) || cyc + 1 >= L.cycles) break;
        // only this workgroup reads what the exchange writes: its barriers order it; the
        // counters are re-read with vector loads (a scalar-cache copy would be stale)
        __syncthreads();
        exchange_instance(st, n, L.swap_key0, L.swap_key1, L.t_add);
        __syncthreads();
        stage_tables(st, d, tile.c0, tile.P, t.tbl);
        t0 = __hip_atomic_load(&st.ctr[n].t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
    }
    write_back(st, d, tile, t);
    if constexpr (FUSE) finish_tile(L, st, n, t.red);
}

// ------------------------------------------------------------------ slice-block sweep
//
// A replica too large for one workgroup's LDS (or whose rows need offsets beyond 16 bits)
// is split into blocks of ng four-slice groups of both parities.  One launch runs one whole
// sweep of every block.  Parity-0 attempts read only parity 1 in time and parity-1 attempts
// only parity 0, so a sweep of groups [g0, g0+ng) needs:
//   phase 0 over groups [g0, g0+ng], one group more than the block owns: that extra group
//     is the next block's first group, recomputed here from the same draws and the same
//     pre-sweep values, hence bit-identical to what that block computes;
//   phase 1 over [g0, g0+ng), whose time neighbours are parity-0 groups [g0, g0+ng].
// The halos (parity-1 groups g0-1 and g0+ng, parity-0 group g0+ng) belong to the
// neighbouring blocks, which write their groups back during the same launch, so they are
// read from boundary records instead: at the end of sweep t each block records its first
// group of both parities and its last group of parity 1 in buffer (t+1) mod 2, and sweep t
// reads its neighbours' records from buffer t mod 2 (filled from the spins before the
// first sweep of a call).  Slot s of a row stands for group g0 - 1 + s (mod G4); a block
// owns slots 1..ng.  Parity-1 rows hold slots 0..ng+1 (ng + 2 words); parity-0 rows hold
// slots 1..ng+1 (ng + 1 words), slot 0 of parity 0 being never read.

// A thread's position (x, y, z) in a linear walk over [z][y][x] (x < nx, y < ny) that
// advances by a fixed stride per step, with carries instead of divisions.
struct Walk3 {
    int x, y, z, sx, sy, sz, nx, ny;
    __device__ __forceinline__ Walk3(int start, int stride, int nx_, int ny_) : nx(nx_), ny(ny_)
    {
        x = start % nx;
        const int r = start / nx;
        y = r % ny;
        z = r / ny;
        sx = stride % nx;
        const int rs = stride / nx;
        sy = rs % ny;
        sz = rs / ny;
    }
    __device__ __forceinline__ void step()
    {
        x += sx;
        int c = 0;
        if (x >= nx) {
            x -= nx;
            c = 1;
        }
        y += sy + c;
        z += sz;
        if (y >= ny) {
            y -= ny;
            ++z;
        }
    }
};

struct BlockLds {
    uint8_t *sp;       // P replicas x (N rows of ng + 1 words, N rows of ng + 2 words)
    uint32_t *ent;     // N * D entries
    uint32_t *bias;    // N
    uint16_t *csite;   // N
    int32_t *coff;     // n_colors + 1
    uint32_t *tbl;     // P tables
    long long *red;    // reduction scratch
};

__host__ __device__ __forceinline__ int64_t block_offsets(const InstDesc &d, int P, int ng,
                                                          int64_t o[7])
{
    int64_t x = 0;
    o[0] = x; x = a16(x + (int64_t)P * d.N * (2 * ng + 3) * 4);
    o[1] = x; x = a16(x + (int64_t)d.N * d.D * 4);
    o[2] = x; x = a16(x + (int64_t)d.N * 4);
    o[3] = x; x = a16(x + (int64_t)d.N * 2);
    o[4] = x; x = a16(x + (int64_t)(d.n_colors + 1) * 4);
    o[5] = x; x = a16(x + (int64_t)P * d.tbl_words * 4);
    o[6] = x; x = a16(x + 2 * 16 * 8);
    return x;
}

// Global four-slice group held by LDS slot s of a block starting at g0.
__device__ __forceinline__ int block_slot_group(int s, int g0, int G4)
{
    return (g0 - 1 + s + G4) & (G4 - 1);
}

// Per-launch constants of a block tile.
struct BlockArgs {
    uint32_t key0, key1, tt, n, c0;
    uint32_t RS[2];       // bytes of one LDS row of parity 0 (ng + 1 words) and 1 (ng + 2)
    uint32_t base[2];     // start of each parity's rows within a replica
    uint32_t QS;          // bytes of one replica
    uint32_t sel_x;       // v_perm selector: x -> x * (2F + 1)
    int G4, g0, esh, tbl_words;
};

// LDS byte offset of slot s of site i's row of parity p in replica q.  The per-parity
// constants are chosen with selects: an index into the two-element arrays by a run-time
// parity would place the arguments in scratch memory.
__device__ __forceinline__ uint32_t block_at(const BlockArgs &a, int p, int q, int i, int s)
{
    const uint32_t base = p ? a.base[1] : a.base[0];
    const uint32_t rs = p ? a.RS[1] : a.RS[0];
    return (uint32_t)q * a.QS + base + __umul24((uint32_t)i, rs) + 4u * (uint32_t)(s - 1 + p);
}

// One lane's update of site i, replica q, the group in slot s of parity PAR: four
// Metropolis attempts served by one Philox call.
template <int DT, int PAR>
__device__ __forceinline__ void block_item(const BlockArgs &a, const BlockLds &t, int D, int i,
                                           int q, int s)
{
    const uint32_t nb_base = block_at(a, PAR, q, 0, s);
    const uint32_t own = nb_base + __umul24((uint32_t)i, a.RS[PAR]);
    const uint32_t oth = block_at(a, PAR ^ 1, q, i, s);
    const uint32_t X = lds32(t.sp, own);
    const uint32_t Wc = lds32(t.sp, oth);
    uint32_t T;
    if constexpr (PAR == 0)
        T = __builtin_amdgcn_alignbyte(Wc, lds32(t.sp, oth - 4u), 3) + Wc;
    else
        T = __builtin_amdgcn_alignbyte(lds32(t.sp, oth + 4u), Wc, 1) + Wc;
    // the entry holds j << esh in its top half; a block row is RS bytes
    const uint32_t *er = t.ent + i * D;
    const int shift = 16 + a.esh;
    uint32_t acc = 0;
    if constexpr (DT > 0) {
        uint32_t ents[DT], ws[DT];
#pragma unroll
        for (int e = 0; e < DT; ++e) ents[e] = er[e];
#pragma unroll
        for (int e = 0; e < DT; ++e) ws[e] = lds32(t.sp, nb_base + __umul24(ents[e] >> shift, a.RS[PAR]));
#pragma unroll
        for (int e = 0; e < DT; ++e) acc += __builtin_amdgcn_perm(0u, ents[e], ws[e]);
    } else {
        for (int e = 0; e < D; ++e) {
            const uint32_t ent = er[e];
            acc += __builtin_amdgcn_perm(0u, ent, lds32(t.sp, nb_base + __umul24(ent >> shift, a.RS[PAR])));
        }
    }
    const int g = block_slot_group(s, a.g0, a.G4);
    const Words4 u = philox10((uint32_t)(2 * i + PAR) * (uint32_t)a.G4 + (uint32_t)g, a.tt,
                              a.c0 + (uint32_t)q, a.n, a.key0, a.key1);
    const uint32_t V = __builtin_amdgcn_perm(0u, a.sel_x, X) + (acc << 1) + t.bias[i];
    const uint32_t IDX = V + (V << 1) + T;
    const uint32_t *tb = t.tbl + q * a.tbl_words;
    uint32_t flip = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint32_t thr = tb[(IDX >> (8 * b)) & 0xFFu];
        flip |= (u.w[b] <= thr ? 1u : 0u) << (8 * b);
    }
    *reinterpret_cast<uint32_t *>(t.sp + own) = X ^ flip;
}


// The slots a phase runs: ns of them, slot s0 + r for r < cut and s0 + r + jump beyond
// (two runs of consecutive slots).
struct SlotSet {
    int s0, ns, cut, jump;
    __device__ __forceinline__ int at(int r) const { return s0 + r + (r >= cut ? jump : 0); }
};

// A thread's share of a slot set whose P * ns (replica, slot) pairs per site fit the
// workgroup: it keeps pair (q, sl) and runs sites s_first, s_first + sstep, ... of each
// class.  It depends only on the thread and the slot set, so a resident block computes
// it once per call, not once per sweep (the divisions would cost as much as a few
// attempts).
struct PhaseLane {
    int q, sl, sstep, s_first;
};

__device__ __forceinline__ PhaseLane phase_lane(const Tile &tile, const SlotSet &S, int nt)
{
    const int tid = threadIdx.x;
    const int lanes = tile.P * S.ns;
    PhaseLane L;
    if (lanes > nt) {
        L.q = L.sl = L.sstep = 0;
        L.s_first = 1 << 30;
        return L;
    }
    const int r = tid % lanes;
    L.q = r / S.ns;
    L.sl = S.at(r - L.q * S.ns);
    L.sstep = nt / lanes;
    L.s_first = (tid < L.sstep * lanes) ? tid / lanes : (1 << 30);
    return L;
}

// All colour classes of parity PAR over the slots of S (a whole sweep: phase 0 over slots
// 1..ng+1, phase 1 over 1..ng).  Slots of one parity are independent of each other within
// a phase, so a phase may be run as several slot sets in any order.  When the pairs fit
// the workgroup each thread keeps one (replica, slot) pair, given by PL, and strides over
// the sites of a class; otherwise the items of a class are dealt out one by one.
template <int DT, int PAR>
__device__ __forceinline__ void block_phase(const BlockArgs &a, const InstDesc &d, const Tile &tile,
                                            const BlockLds &t, const SlotSet &S, const PhaseLane &PL,
                                            int nt, int g_lo = 0, int g_hi = 1 << 30)
{
    const int tid = threadIdx.x;
    const int D = (DT > 0) ? DT : d.D;
    const int ns = S.ns;
    const int lanes = tile.P * ns;  // per site
    g_hi = min(g_hi, d.n_colors);
    if (lanes <= nt) {
        for (int g = g_lo; g < g_hi; ++g) {
            const int s1 = t.coff[g + 1];
            for (int si = t.coff[g] + PL.s_first; si < s1; si += PL.sstep)
                block_item<DT, PAR>(a, t, D, t.csite[si], PL.q, PL.sl);
            __syncthreads();
        }
    } else {
        for (int g = g_lo; g < g_hi; ++g) {
            const int s0 = t.coff[g];
            const int items = (t.coff[g + 1] - s0) * lanes;
            for (int it = tid; it < items; it += nt) {
                const int si = it / lanes, r = it - si * lanes;
                const int q = r / ns;
                block_item<DT, PAR>(a, t, D, t.csite[s0 + si], q, S.at(r - q * ns));
            }
            __syncthreads();
        }
    }
}

// The slot sets of a whole sweep (phase 0, then phase 1) or of the split sweep below, with
// the workgroup size nt.
struct SweepSets {
    SlotSet s[4];
    PhaseLane l[4];
    int nt;
};

__device__ __forceinline__ SweepSets whole_sweep_sets(const Tile &tile, int nt)
{
    const int ng = tile.ng;
    SweepSets w;
    w.nt = nt;
    w.s[0] = SlotSet{1, ng + 1, ng + 1, 0};
    w.s[1] = SlotSet{1, ng, ng, 0};
    w.s[2] = w.s[3] = w.s[1];
    for (int k = 0; k < 2; ++k) w.l[k] = phase_lane(tile, w.s[k], nt);
    w.l[2] = w.l[3] = w.l[1];
    return w;
}

template <int DT>
__device__ __forceinline__ void block_sweep(const BlockArgs &a, const InstDesc &d, const Tile &tile,
                                            const BlockLds &t, const SweepSets &w)
{
    block_phase<DT, 0>(a, d, tile, t, w.s[0], w.l[0], w.nt);
    block_phase<DT, 1>(a, d, tile, t, w.s[1], w.l[1], w.nt);
}

__device__ __forceinline__ SweepSets split_sweep_sets(const Tile &tile, int nt)
{
    const int ng = tile.ng;
    SweepSets w;
    w.nt = nt;
    w.s[0] = SlotSet{2, ng - 1, ng - 1, 0};  // phase 0: 2..ng
    w.s[1] = SlotSet{1, 2, 1, ng - 1};       // phase 0: 1 and ng + 1
    w.s[2] = SlotSet{1, 2, 1, ng - 2};       // phase 1: 1 and ng
    w.s[3] = SlotSet{2, ng - 2, ng - 2, 0};  // phase 1: 2..ng - 1
    for (int k = 0; k < 4; ++k) w.l[k] = phase_lane(tile, w.s[k], nt);
    return w;
}

// A sweep of a resident block (ng >= 6) ordered so that the exchange with the neighbours
// overlaps work: phase 0 first over slots 2..ng, which read no halo; then halos_in() (the
// neighbours' parity-1 groups of the previous sweep into the halo slots); phase 0 over
// slots 1 and ng+1; phase 1 over slots 1 and ng, the groups the neighbours need; then
// records() stores them; phase 1 over slots 2..ng-1 while the neighbours go on, with
// commit() after its first colour class, when the record stores have long completed.
template <int DT, class HalosIn, class Records, class Commit>
__device__ __forceinline__ void block_sweep_split(const BlockArgs &a, const InstDesc &d,
                                                  const Tile &tile, const BlockLds &t,
                                                  const SweepSets &w, HalosIn &&halos_in,
                                                  Records &&records, Commit &&commit)
{
    block_phase<DT, 0>(a, d, tile, t, w.s[0], w.l[0], w.nt);
    halos_in();
    block_phase<DT, 0>(a, d, tile, t, w.s[1], w.l[1], w.nt);
    block_phase<DT, 1>(a, d, tile, t, w.s[2], w.l[2], w.nt);
    records();
    block_phase<DT, 1>(a, d, tile, t, w.s[3], w.l[3], w.nt, 0, 1);
    commit();
    block_phase<DT, 1>(a, d, tile, t, w.s[3], w.l[3], w.nt, 1);
}

// The slice blocks of one replica share every cache line of its spin rows (a block owns a
// few words of each row), so the launches map workgroups to tiles with xcd_tile: runs of
// consecutive tiles share an XCD.

// Before the first slice-block launch of a call: every block's boundary record of the
// current spins into buffer (t mod 2), its progress count zeroed, and E_cl, C of its
// replica cleared by the block at g0 = 0 (the blocks add their partial sums on the call's
// last launch).  One workgroup per block, mapped to tiles as in the sweep launches.
__global__ void block_prepare_kernel(SweepLaunch L)
{
    const DevState &st = L.st;
    const Tile tile = st.tiles[L.tile0 + xcd_tile(blockIdx.x, gridDim.x)];
    const InstDesc d = st.inst[tile.inst];
    const int N = d.N, ng = tile.ng, g0 = tile.g0;
    uint32_t *rec = st.halo + (int64_t)(st.ctr[tile.inst].t & 1) * st.halo_words + tile.hb;
    const uint8_t *rep = st.spins + d.spin_base + (int64_t)tile.c0 * d.rep_bytes;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const uint8_t *r0 = rep + (int64_t)i * d.Mh;
        const uint8_t *r1 = rep + (int64_t)N * d.Mh + (int64_t)i * d.Mh;
        rec[i] = *reinterpret_cast<const uint32_t *>(r0 + 4 * g0);
        rec[N + i] = *reinterpret_cast<const uint32_t *>(r1 + 4 * g0);
        rec[2 * N + i] = *reinterpret_cast<const uint32_t *>(r1 + 4 * (g0 + ng - 1));
    }
    if (threadIdx.x == 0) st.prog[xcd_tile(blockIdx.x, gridDim.x)] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) st.xseen[1] = 0u;
    if (g0 == 0 && threadIdx.x == 0)
        for (int q = 0; q < tile.P; ++q) {
            st.E[d.rep_base + tile.c0 + q] = 0;
            st.C[d.rep_base + tile.c0 + q] = 0;
        }
}

// Resident slice blocks pass boundary records and progress counts between workgroups on
// different XCDs, whose L2 caches are not coherent with one another.  Both are read and
// written only with agent-scope atomic operations, which the hardware performs coherently
// for the whole device, so no L2 write-back or invalidation is needed: every wave waits for
// its record stores to complete before the barrier that precedes the count's store, and a
// block issues its halo loads only after it has seen the counts.  When every replica's
// ring of blocks runs on one XCD (local), the stores are plain: they land in that XCD's L2,
// where the same device-scope loads find them, without the trip to the coherence point.
__device__ __forceinline__ uint32_t rec_ld(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void rec_st(uint32_t *p, uint32_t v, bool local)
{
    if (local)
        *p = v;
    else
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Stage a slice block into LDS: the owned groups of both planes from the spins (16-byte
// pieces when VEC, i.e. ng is a multiple of 4), the halos from the neighbours' boundary
// records, then rows, biases, colour lists and the rung table (a slice block holds one
// replica).
template <bool VEC>
__device__ __forceinline__ void block_stage(const DevState &st, const InstDesc &d, const Tile &tile,
                                            const BlockArgs &a, const BlockLds &t,
                                            const uint32_t *rec_in)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int P = tile.P, ng = tile.ng, g0 = tile.g0, N = d.N;
    uint32_t *sp32 = reinterpret_cast<uint32_t *>(t.sp);
    const uint8_t *rep0 = st.spins + d.spin_base + (int64_t)tile.c0 * d.rep_bytes;
    const Tile tp = st.tiles[tile.prev], tn = st.tiles[tile.next];
    const int ND = N * d.D, tw = d.tbl_words;
    const uint32_t *tbl_src = st.tbl + d.tbl_base + (int64_t)st.rung_of[d.rep_base + tile.c0] * tw;

    // Staging is bound by device-memory latency, not bandwidth: the first round of every
    // stream (owned groups, halos, neighbour rows, biases, colour lists, rung table) is
    // loaded before any of it is stored, so the workgroup waits for memory about once.
    // Halos: parity 1 slot 0 <- previous block's last parity-1 group; parity 1 slot ng+1
    // and parity 0 slot ng+1 <- next block's first groups (P = 1 for slice blocks).
    constexpr int kEnt0 = 8;   // neighbour-row words per thread in the first round
    const int nv = VEC ? ng >> 2 : ng;
    Walk3 wk(tid, nt, nv, N);  // (vector or group, site, q * 2 + plane)
    uint4 val[4];
    int dst[4];
    bool ok[4];
    auto load_owned = [&]() {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ok[u] = wk.z < 2 * P;
            if (ok[u]) {
                const int v = wk.x, i = wk.y, pl = wk.z & 1, q = wk.z >> 1;
                const uint8_t *row = rep0 + (int64_t)q * d.rep_bytes + (int64_t)pl * N * d.Mh +
                                     (int64_t)i * d.Mh;
                if constexpr (VEC) {
                    val[u] = *reinterpret_cast<const uint4 *>(row + 4 * (g0 + 4 * v));
                    dst[u] = (int)(block_at(a, pl, q, i, 1 + 4 * v) >> 2);
                } else {
                    val[u].x = *reinterpret_cast<const uint32_t *>(row + 4 * (g0 + v));
                    dst[u] = (int)(block_at(a, pl, q, i, 1 + v) >> 2);
                }
                wk.step();
            }
        }
    };
    auto store_owned = [&]() {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (!ok[u]) continue;
            sp32[dst[u]] = val[u].x;
            if constexpr (VEC) {
                sp32[dst[u] + 1] = val[u].y;
                sp32[dst[u] + 2] = val[u].z;
                sp32[dst[u] + 3] = val[u].w;
            }
        }
    };
    load_owned();
    const bool row0 = tid < N;
    uint32_t h1p = 0, h0n = 0, h1n = 0, bias0 = 0, tbl0 = 0;
    uint16_t cs0 = 0;
    int32_t co0 = 0;
    if (row0) {
        h1p = rec_ld(rec_in + tp.hb + 2 * N + tid);
        h0n = rec_ld(rec_in + tn.hb + tid);
        h1n = rec_ld(rec_in + tn.hb + N + tid);
        bias0 = st.bias[d.site_base + tid];
        cs0 = st.csite[d.site_base + tid];
    }
    uint32_t e0[kEnt0];
#pragma unroll
    for (int u = 0; u < kEnt0; ++u)
        if (tid + u * nt < ND) e0[u] = st.ent[d.ent_base + tid + u * nt];
    if (tid <= d.n_colors) co0 = st.cls_off[d.cls_base + tid];
    if (tid < tw) tbl0 = tbl_src[tid];

    store_owned();
    if (row0) {
        sp32[block_at(a, 1, 0, tid, 0) >> 2] = h1p;
        sp32[block_at(a, 1, 0, tid, ng + 1) >> 2] = h1n;
        sp32[block_at(a, 0, 0, tid, ng + 1) >> 2] = h0n;
        t.bias[tid] = bias0;
        t.csite[tid] = cs0;
    }
#pragma unroll
    for (int u = 0; u < kEnt0; ++u)
        if (tid + u * nt < ND) t.ent[tid + u * nt] = e0[u];
    if (tid <= d.n_colors) t.coff[tid] = co0;
    if (tid < tw) t.tbl[tid] = tbl0;

    // the remaining rounds, if any
    while (wk.z < 2 * P) {
        load_owned();
        store_owned();
    }
    for (int i = tid + nt; i < N; i += nt) {
        const uint32_t x1p = rec_ld(rec_in + tp.hb + 2 * N + i);
        const uint32_t x0n = rec_ld(rec_in + tn.hb + i);
        const uint32_t x1n = rec_ld(rec_in + tn.hb + N + i);
        sp32[block_at(a, 1, 0, i, 0) >> 2] = x1p;
        sp32[block_at(a, 1, 0, i, ng + 1) >> 2] = x1n;
        sp32[block_at(a, 0, 0, i, ng + 1) >> 2] = x0n;
        t.bias[i] = st.bias[d.site_base + i];
        t.csite[i] = st.csite[d.site_base + i];
    }
    for (int base = tid + kEnt0 * nt; base < ND; base += 4 * nt) {
        uint32_t e[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (base + u * nt < ND) e[u] = st.ent[d.ent_base + base + u * nt];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (base + u * nt < ND) t.ent[base + u * nt] = e[u];
    }
    for (int g = tid + nt; g <= d.n_colors; g += nt) t.coff[g] = st.cls_off[d.cls_base + g];
    for (int k = tid + nt; k < tw; k += nt) t.tbl[k] = tbl_src[k];
}

// Wait until both neighbouring blocks have published `need` sweeps (their boundary records
// of sweep need - 1 are then complete): thread 0 polls while the workgroup waits at a
// barrier.  The wait is bounded, and a block that gives up sets the error word and carries
// on, so every wave of the launch always exits (the host then reports the call as failed).
constexpr int kWaitPolls = 1 << 18;  // the host may lower it (SweepLaunch::wait_polls)
__device__ __forceinline__ void block_wait(const DevState &st, int ip, int in, int need,
                                           int max_polls)
{
    if (threadIdx.x == 0) {
        int polls = 0;
        while (__hip_atomic_load(&st.prog[ip], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need ||
               __hip_atomic_load(&st.prog[in], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
            // once any block has given up, the others stop waiting too
            if (++polls > max_polls ||
                __hip_atomic_load(st.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                atomicOr(st.err, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
}

// Eight waves per SIMD bound the registers (at most 64 VGPRs and few enough SGPRs) so that
// two 1024-thread workgroups fit on a compute unit when their LDS does: without it the
// kernel takes over 100 SGPRs, seven waves per SIMD, and one such workgroup per unit.  The
// resident variant (below) is bounded at four: its sweep loop carries more state, and at
// eight it would spill to scratch memory.
//
// PERSIST: one launch runs all n_sweeps sweeps of the call with every block resident (the
// host launches it only when the device can hold all blocks at once).  The owned groups
// stay in LDS; in each sweep, once its two parity-1 boundary groups are final, a block
// writes them to the records of the next sweep and publishes its progress, and before the
// slots next to its edges in the next sweep it waits for both neighbours and takes their
// parity-1 groups as its halos (with ng >= 6 the interior slots run around these steps,
// see block_sweep_split).  The parity-0 halo (the next block's first group) needs no
// exchange: the block recomputes it bit for bit.  The records alternate between two
// buffers: a neighbour can rewrite a buffer only after it has seen this block's progress
// of the sweep that read it.
template <bool FUSE, bool PERSIST>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(PERSIST ? 4 : 8))) sweep_block_kernel(SweepLaunch L)
{
    extern __shared__ __align__(16) char lds[];
    const DevState &st = L.st;
    const int bt = xcd_tile(blockIdx.x, gridDim.x);
    // resident blocks with L.xcd_local: every replica's ring of blocks lies in one run of
    // xcd_tile, so it runs on one XCD; a launch whose workgroups did not keep to that fails
    // the call (checked at the end; the host recovers), each block running to its end, its
    // waits bounded
    const bool local = PERSIST && L.xcd_local != 0;
    const Tile tile = st.tiles[L.tile0 + bt];
    const int n = tile.inst;
    const InstDesc d = st.inst[n];
    const int tid = threadIdx.x;
    // The workgroup size is kept in a register the compiler cannot see through: otherwise,
    // short of registers, it re-reads it from the dispatch packet in every phase of every
    // sweep, a global load waited for in full.
    int nt = blockDim.x;
    __asm__ volatile("" : "+s"(nt));
    const int P = tile.P, ng = tile.ng, g0 = tile.g0, G4 = d.G4, N = d.N;
    int64_t o[7];
    block_offsets(d, P, ng, o);
    BlockLds t;
    t.sp = reinterpret_cast<uint8_t *>(lds + o[0]);
    t.ent = reinterpret_cast<uint32_t *>(lds + o[1]);
    t.bias = reinterpret_cast<uint32_t *>(lds + o[2]);
    t.csite = reinterpret_cast<uint16_t *>(lds + o[3]);
    t.coff = reinterpret_cast<int32_t *>(lds + o[4]);
    t.tbl = reinterpret_cast<uint32_t *>(lds + o[5]);
    t.red = reinterpret_cast<long long *>(lds + o[6]);

    uint32_t *sp32 = reinterpret_cast<uint32_t *>(t.sp);
    const uint64_t tsw = st.ctr[n].t + (uint64_t)L.sweep_off;
    BlockArgs a;
    a.key0 = L.key0;
    a.key1 = L.key1;
    a.tt = (uint32_t)tsw;
    a.n = (uint32_t)n;
    a.c0 = (uint32_t)tile.c0;
    a.RS[0] = 4u * (uint32_t)(ng + 1);
    a.RS[1] = 4u * (uint32_t)(ng + 2);
    a.base[0] = 0;
    a.base[1] = (uint32_t)N * a.RS[0];
    a.QS = (uint32_t)N * (a.RS[0] + a.RS[1]);
    a.sel_x = (uint32_t)(2 * d.F + 1) << 8;
    a.G4 = G4;
    a.g0 = g0;
    a.esh = d.ent_sh;
    a.tbl_words = d.tbl_words;
    const uint32_t *rec_in = st.halo + (int64_t)(tsw & 1) * st.halo_words;
    if ((ng & 3) == 0)
        block_stage<true>(st, d, tile, a, t, rec_in);
    else
        block_stage<false>(st, d, tile, a, t, rec_in);
    __syncthreads();

    const int n_sw = PERSIST ? L.n_sweeps : 1;
    const int ip = tile.prev - L.tile0, in = tile.next - L.tile0;
    const int hbp = st.tiles[tile.prev].hb, hbn = st.tiles[tile.next].hb;
    const int polls = L.wait_polls > 0 ? L.wait_polls : kWaitPolls;
    // resident blocks: wait for both neighbours' previous sweep and take their parity-1
    // boundary groups as halos
    auto wait_halos = [&](int sw) {
        block_wait(st, ip, in, sw + L.wait_extra, polls);
        const uint32_t *rin = st.halo + (int64_t)((tsw + sw) & 1) * st.halo_words;
        for (int i = tid; i < N; i += nt) {
            const uint32_t h1p = rec_ld(rin + hbp + 2 * N + i);
            const uint32_t h1n = rec_ld(rin + hbn + N + i);
            sp32[block_at(a, 1, 0, i, 0) >> 2] = h1p;
            sp32[block_at(a, 1, 0, i, ng + 1) >> 2] = h1n;
        }
        __syncthreads();
    };
    // With at most one site per thread the halos of sweep sw are fetched into registers at
    // the end of sweep sw - 1 (fetch_halos) and stored to LDS only before the edge slots of
    // sweep sw (store_halos), so the load latency overlaps phase 0's interior slots.  The
    // parity-1 halo slots are read by no slot of the interior.
    const bool early = PERSIST && ng >= 6 && N <= nt;
    uint32_t hreg_p = 0, hreg_n = 0;
    // The loads are issued after every sweep of a resident block, also when their values go
    // unused (the last sweep of the call, or no early halos), and by every thread (past N,
    // of site N - 1): loads under a branch would be waited for where the branch ends.  They
    // stay inside the record buffers.
    auto fetch_halos = [&](int sw, bool wait) {
        if (wait) block_wait(st, ip, in, sw + L.wait_extra, polls);
        const uint32_t *rin = st.halo + (int64_t)((tsw + sw) & 1) * st.halo_words;
        const int i = min(tid, N - 1);
        hreg_p = rec_ld(rin + hbp + 2 * N + i);
        hreg_n = rec_ld(rin + hbn + N + i);
    };
    auto store_halos = [&]() {
        if (tid < N) {
            sp32[block_at(a, 1, 0, tid, 0) >> 2] = hreg_p;
            sp32[block_at(a, 1, 0, tid, ng + 1) >> 2] = hreg_n;
        }
        __syncthreads();
    };
    // resident blocks: the parity-1 boundary groups for the neighbours' next sweep, then
    // progress.  Every wave waits for its record stores to complete (vmcnt 0; a workgroup
    // barrier does not wait for them) before thread 0 stores the progress count.
    auto store_records = [&](int sw) {
        uint32_t *rout = st.halo + (int64_t)((tsw + sw + 1) & 1) * st.halo_words + tile.hb;
        for (int i = tid; i < N; i += nt) {
            rec_st(rout + N + i, sp32[block_at(a, 1, 0, i, 1) >> 2], local);
            rec_st(rout + 2 * N + i, sp32[block_at(a, 1, 0, i, ng) >> 2], local);
        }
    };
    auto commit = [&](int sw) {
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        __syncthreads();
        if (tid == 0) rec_st(reinterpret_cast<uint32_t *>(&st.prog[bt]), (uint32_t)(sw + 1), local);
    };
    auto publish = [&](int sw) {
        store_records(sw);
        commit(sw);
    };
    // the sweep loop, instantiated per degree (the switch stays outside the loop, so only one
    // degree's phase set-up is live in it)
    const bool split = PERSIST && ng >= 6;
    const SweepSets sets = split ? split_sweep_sets(tile, nt) : whole_sweep_sets(tile, nt);
    auto sweeps = [&](auto dt) {
        constexpr int DT = decltype(dt)::value;
        for (int sw = 0; sw < n_sw; ++sw) {
            a.tt = (uint32_t)(tsw + sw);
            if (split) {
                block_sweep_split<DT>(
                    a, d, tile, t, sets,
                    [&]() {
                        if (sw > 0) {
                            if (early)
                                store_halos();
                            else
                                wait_halos(sw);
                        }
                    },
                    [&]() {
                        if (sw + 1 < n_sw) store_records(sw);
                    },
                    [&]() {
                        if (sw + 1 < n_sw) commit(sw);
                    });
            } else {
                if (PERSIST && sw > 0) wait_halos(sw);
                block_sweep<DT>(a, d, tile, t, sets);
                if (PERSIST && sw + 1 < n_sw) publish(sw);
            }
            if (PERSIST) fetch_halos(sw + 1, early && sw + 1 < n_sw);
        }
    };
    switch (d.D) {
    case 1: sweeps(IntC<1>{}); break;
    case 2: sweeps(IntC<2>{}); break;
    case 3: sweeps(IntC<3>{}); break;
    case 4: sweeps(IntC<4>{}); break;
    case 5: sweeps(IntC<5>{}); break;
    case 6: sweeps(IntC<6>{}); break;
    case 7: sweeps(IntC<7>{}); break;
    case 8: sweeps(IntC<8>{}); break;
    default: sweeps(IntC<0>{}); break;
    }

    // partial E_cl and C of the block's owned slices after the last sweep of the call
    if (L.last) {
        const int D = d.D, F = d.F;
        for (int q = 0; q < P; ++q) {
            long long ee = 0, cc = 0;
            for (Walk3 wk(tid, nt, ng, N); wk.z < 1; wk.step()) {  // (owned group, site)
                const int lg = wk.x, i = wk.y;
                const uint32_t X0 = lds32(t.sp, block_at(a, 0, q, i, lg + 1));
                const uint32_t X1 = lds32(t.sp, block_at(a, 1, q, i, lg + 1));
                const uint32_t X0n = lds32(t.sp, block_at(a, 0, q, i, lg + 2));
                const uint32_t dis_t = popc(X0 ^ X1) + popc(X1 ^ __builtin_amdgcn_alignbyte(X0n, X0, 1));
                cc += 8 - 2 * (long long)dis_t;
                const int hval = (int)(t.bias[i] & 0xFFu) - F;
                int sumJ = 0;
                long long eterm = 0;
                for (int e = 0; e < D; ++e) {
                    const uint32_t ent = t.ent[i * D + e];
                    const int w0 = (int)(ent & 0xFFu), w1 = (int)((ent >> 8) & 0xFFu);
                    const int J = w1 - w0;
                    sumJ += w0 + w1;
                    const int j = (int)((ent >> 16) >> d.ent_sh);
                    if (J != 0 && j > i) {
                        const uint32_t Y0 = lds32(t.sp, block_at(a, 0, q, j, lg + 1));
                        const uint32_t Y1 = lds32(t.sp, block_at(a, 1, q, j, lg + 1));
                        eterm += (long long)J * (8 - 2 * (long long)(popc(X0 ^ Y0) + popc(X1 ^ Y1)));
                    }
                }
                eterm += (long long)(hval + sumJ) * (2 * (long long)(popc(X0) + popc(X1)) - 8);
                ee += eterm;
            }
            ee = block_sum(ee, t.red);
            cc = block_sum(cc, t.red);
            if (tid == 0) {
                atomicAdd(reinterpret_cast<unsigned long long *>(&st.E[d.rep_base + tile.c0 + q]),
                          (unsigned long long)ee);
                atomicAdd(reinterpret_cast<unsigned long long *>(&st.C[d.rep_base + tile.c0 + q]),
                          (unsigned long long)cc);
            }
        }
    }

    // write back the owned groups of both parities (16-byte stores for whole vectors)
    if ((ng & 3) == 0) {
        for (Walk3 wk(tid, nt, ng >> 2, N); wk.z < 2 * P; wk.step()) {  // (vector, site, q * 2 + plane)
            const int v = wk.x, i = wk.y, pl = wk.z & 1, q = wk.z >> 1;
            const int w = (int)(block_at(a, pl, q, i, 1 + 4 * v) >> 2);
            const uint4 val = make_uint4(sp32[w], sp32[w + 1], sp32[w + 2], sp32[w + 3]);
            *reinterpret_cast<uint4 *>(st.spins + d.spin_base + (int64_t)(tile.c0 + q) * d.rep_bytes +
                                       (int64_t)pl * N * d.Mh + (int64_t)i * d.Mh + 4 * (g0 + 4 * v)) = val;
        }
    } else {
        for (Walk3 wk(tid, nt, ng, N); wk.z < 2 * P; wk.step()) {  // (group, site, q * 2 + plane)
            const int lg = wk.x, i = wk.y, pl = wk.z & 1, q = wk.z >> 1;
            *reinterpret_cast<uint32_t *>(st.spins + d.spin_base + (int64_t)(tile.c0 + q) * d.rep_bytes +
                                          (int64_t)pl * N * d.Mh + (int64_t)i * d.Mh + 4 * (g0 + lg)) =
                sp32[block_at(a, pl, q, i, 1 + lg) >> 2];
        }
    }
    // boundary records for the next launch: first group of both parities, last of parity 1
    if constexpr (!PERSIST) {
        uint32_t *rec_out = st.halo + (int64_t)((tsw + 1) & 1) * st.halo_words + tile.hb;
        for (int i = tid; i < N; i += nt) {
            rec_out[i] = sp32[block_at(a, 0, 0, i, 1) >> 2];
            rec_out[N + i] = sp32[block_at(a, 1, 0, i, 1) >> 2];
            rec_out[2 * N + i] = sp32[block_at(a, 1, 0, i, ng) >> 2];
        }
    }
    if (local) xcd_check(st, st.xseen + 1, (int)blockIdx.x, kErrPlace, L.xcd_local == 2);
    if constexpr (FUSE)
        if (L.last) finish_tile(L, st, n, t.red);
}

// ------------------------------------------------------------------ generic sweep

__device__ __forceinline__ int lds_x(const uint8_t *rep, const InstDesc &d, int k, int i)
{
    const int p = (d.M >= 2) ? (k & 1) : 0;
    const int m = (d.M >= 2) ? (k >> 1) : 0;
    return rep[p * d.N * d.Mh + i * d.Mh + m];
}

template <bool FUSE>
__global__ void __launch_bounds__(1024) sweep_generic_kernel(SweepLaunch L)
{
    extern __shared__ __align__(16) char lds[];
    const DevState &st = L.st;
    const Tile tile = st.tiles[L.tile0 + blockIdx.x];
    const int n = tile.inst;
    const InstDesc d = st.inst[n];
    const int n_adj = st.adj_off[d.off_base + d.N];
    TileLds t = carve(lds, d, n_adj, tile.P);
    stage_common(st, d, n, tile, t, n_adj);
    const uint64_t t0 = st.ctr[n].t;
    __syncthreads();

    const int tid = threadIdx.x, nt = blockDim.x;
    const int N = d.N, M = d.M, Mh = d.Mh, G4 = d.G4, F = d.F;
    const int rep_lds = (int)rep_lds_bytes(d);
    const int Lq = tile.P * G4;  // lanes per site
    const int bstride = 2 * F + 1;

    for (int sw = 0; sw < L.n_sweeps; ++sw) {
        const uint32_t tt = (uint32_t)(t0 + (uint64_t)sw);
        for (int p = 0; p < d.parities; ++p) {
            for (int g = 0; g < d.n_colors; ++g) {
                const int s0 = t.coff[g];
                const int items = (t.coff[g + 1] - s0) * Lq;
                for (int it = tid; it < items; it += nt) {
                    const int si = it / Lq;
                    const int r = it - si * Lq;
                    const int q = r / G4;
                    const int g4 = r - q * G4;
                    const int i = t.csite[s0 + si];
                    uint8_t *rep = t.sp + q * rep_lds;
                    const Words4 u = philox10(spin_ctr0(i, p, G4, g4), tt,
                                              (uint32_t)(tile.c0 + q), (uint32_t)n, L.key0, L.key1);
                    const uint32_t *tb = t.tbl + q * d.tbl_words;
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int m = 4 * g4 + b;
                        if (m >= Mh) break;
                        const int k = (M >= 2) ? 2 * m + p : 0;
                        uint8_t *cell = rep + p * N * Mh + i * Mh + m;
                        const int x = *cell;
                        int f = t.h[i];
                        for (int e = t.off[i]; e < t.off[i + 1]; ++e) {
                            const int a = t.adj[e];
                            f += (a >> 16) * (2 * (int)rep[p * N * Mh + (a & 0xFFFF) * Mh + m] - 1);
                        }
                        int tau = 1;
                        if (M >= 2)
                            tau = lds_x(rep, d, (k == 0) ? M - 1 : k - 1, i) +
                                  lds_x(rep, d, (k + 1 == M) ? 0 : k + 1, i);
                        const int idx = (x * bstride + f + F) * 3 + tau;
                        if (u.w[b] <= tb[idx]) *cell = (uint8_t)(x ^ 1);
                    }
                }
                __syncthreads();
            }
        }
    }

    for (int q = 0; q < tile.P; ++q) {
        long long e2 = 0, cc = 0;
        const uint8_t *rep = t.sp + q * rep_lds;
        for (int it = tid; it < M * N; it += nt) {
            const int k = it / N;
            const int i = it - k * N;
            const int s = 2 * lds_x(rep, d, k, i) - 1;
            int f = 2 * t.h[i];
            for (int e = t.off[i]; e < t.off[i + 1]; ++e) {
                const int a = t.adj[e];
                f += (a >> 16) * (2 * lds_x(rep, d, k, a & 0xFFFF) - 1);
            }
            e2 += (long long)s * f;
            if (M >= 2) cc += (long long)s * (2 * lds_x(rep, d, (k + 1 == M) ? 0 : k + 1, i) - 1);
        }
        e2 = block_sum(e2, t.red);
        cc = block_sum(cc, t.red);
        if (tid == 0) {
            st.E[d.rep_base + tile.c0 + q] = e2 / 2;
            st.C[d.rep_base + tile.c0 + q] = cc;
        }
    }
    write_back(st, d, tile, t);
    if constexpr (FUSE) finish_tile(L, st, n, t.red);
}

// ------------------------------------------------------------------ exchange

__global__ void exchange_kernel(DevState st, uint32_t key0, uint32_t key1, uint32_t t_add)
{
    exchange_instance(st, blockIdx.x, key0, key1, t_add);
}

// ------------------------------------------------------------------ imaginary time

// Lag l of the imaginary-time correlations, in slices: max(1, floor((l + 1) M / 16)).
__device__ __forceinline__ int tau_lag(int M, int l)
{
    const int d = (l + 1) * M / 16;
    return d < 1 ? 1 : d;
}

// Ct_l = sum_k sum_i s_i^k s_i^{(k + lag_l) mod M} of replica (blockIdx.x) over the
// positions of chunk blockIdx.y (of gridDim.y), added to sumCt of the replica's rung.  A lane takes the
// four slices m = 4 g4 .. 4 g4 + 3 of one (parity, site) row; slice k = 2m + p meets
// slice k + lag in the row of parity (p + lag) mod 2 at m + (p + lag) / 2 (cyclically).
//
// When a site's two rows fit one wave (Mh % 4 == 0 and 2 Wr <= 64 words, Wr = Mh / 4), a
// wave holds both rows of 64 / (2 Wr) sites, one word per lane, and takes every lagged
// word from the lane that loaded it (ds_bpermute): one load per four slices, one lane read
// of the row's next word, and per lag a byte alignment, one lane read, an xor and a
// popcount.  A lane's sources and byte shifts depend only on the lane, so they are set up
// once.  The loop runs per wave (every
// lane stays active for the lane reads); lanes past the last site only mask their sums.
// Other rows fall back to loads: neighbouring lanes read neighbouring bytes at every lag.
__global__ void __launch_bounds__(256) tau_corr_kernel(DevState st)
{
    __shared__ long long red[4][kTauLags];
    const int g = blockIdx.x;
    const int n = st.rep_inst[g];
    const InstDesc d = st.inst[n];
    const int c = g - d.rep_base;
    const uint8_t *rep = st.spins + d.spin_base + (int64_t)c * d.rep_bytes;
    const int N = d.N, M = d.M, Mh = d.Mh, G4 = d.G4;
    int lag[kTauLags];
#pragma unroll
    for (int l = 0; l < kTauLags; ++l) lag[l] = tau_lag(M, l) % M;
    int acc[kTauLags];
#pragma unroll
    for (int l = 0; l < kTauLags; ++l) acc[l] = 0;
    const int total = d.parities * N * G4;
    const int Wr4 = Mh >> 2;
    if (M >= 2 && (Mh & 3) == 0 && 2 * Wr4 <= 64) {
        const uint32_t *rep32 = reinterpret_cast<const uint32_t *>(rep);
        const int Wr = Wr4, gw = 2 * Wr, spw = 64 / gw;
        const int lane = threadIdx.x & 63;
        const int sl = lane / gw, rem = lane - sl * gw;
        const int p = rem >= Wr ? 1 : 0, g4 = rem - p * Wr;
        const bool used = sl < spw;
        // A lane reads lag l's word from lane j of row (p + lag) mod 2 of its site.  Every
        // lane that reads row P' at lag l has the same parity, (P' + lag) mod 2, and so
        // the same byte shift: the source lane shifts its own word by it (joining it with
        // the next word of its row), and one lane read per lag suffices.
        const int nxt = used ? 4 * (sl * gw + p * Wr + ((g4 + 1 == Wr) ? 0 : g4 + 1)) : 4 * lane;
        int src[kTauLags];
        uint32_t ssh[kTauLags];
#pragma unroll
        for (int l = 0; l < kTauLags; ++l) {
            const int q = p + lag[l];
            const int sh = q >> 1;                 // slices to move along the row
            int j = g4 + (sh >> 2);                // sh / 4 <= Mh / 8 < Wr
            if (j >= Wr) j -= Wr;
            src[l] = used ? 4 * (sl * gw + (q & 1) * Wr + j) : 4 * lane;
            const int pr = (p + lag[l]) & 1;       // the parity of the lanes that read this row
            ssh[l] = (uint32_t)(((pr + lag[l]) >> 1) & 3);
        }
        const int waves = gridDim.y * (blockDim.x >> 6);
        const int w0 = blockIdx.y * (blockDim.x >> 6) + (threadIdx.x >> 6);
        uint32_t pc[kTauLags];
#pragma unroll
        for (int l = 0; l < kTauLags; ++l) pc[l] = 0;
        int npos = 0;
        // four site groups per step, their loads issued together
        constexpr int kU = 4;
        const int step = waves * spw;
        const uint32_t row0 = (uint32_t)p * (uint32_t)N;
        for (int s0 = w0 * spw; s0 < N; s0 += kU * step) {
            uint32_t X[kU];
            bool ok[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = s0 + u * step + sl;
                ok[u] = used && i < N;
                X[u] = ok[u] ? rep32[(row0 + (uint32_t)i) * (uint32_t)Wr + (uint32_t)g4] : 0u;
                npos += ok[u] ? 1 : 0;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const uint32_t Xn = (uint32_t)__builtin_amdgcn_ds_bpermute(nxt, (int)X[u]);
#pragma unroll
                for (int l = 0; l < kTauLags; ++l) {
                    const uint32_t V = __builtin_amdgcn_alignbyte(Xn, X[u], ssh[l]);
                    const uint32_t Y = (uint32_t)__builtin_amdgcn_ds_bpermute(src[l], (int)V);
                    pc[l] += ok[u] ? (uint32_t)__popc(X[u] ^ Y) : 0u;
                }
            }
        }
        // Four products per position; a differing byte pair contributes -1 instead of +1.
        // The wave's sums (32-bit: a replica holds at most 2 N M < 2^31 products) go
        // straight to the rung's accumulators, one lag per lane of lanes 0..7; waves
        // without sites add nothing.
        if (w0 * spw >= N) return;
        int v[kTauLags];
#pragma unroll
        for (int l = 0; l < kTauLags; ++l) v[l] = 4 * npos - 2 * (int)pc[l];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
            for (int l = 0; l < kTauLags; ++l) v[l] += __shfl_xor(v[l], o);
        if (lane < kTauLags) {
            int mine = v[0];
#pragma unroll
            for (int l = 1; l < kTauLags; ++l) mine = (lane == l) ? v[l] : mine;
            const int r = st.rung_of[g];
            atomicAdd(reinterpret_cast<unsigned long long *>(&st.sumCt[((int64_t)d.rep_base + r) * kTauLags + lane]),
                      (unsigned long long)(long long)mine);
        }
        return;
    } else if (M >= 2 && (Mh & 3) == 0) {
        // whole words: the four bytes from slice m2 on are two aligned words joined by a
        // byte alignment (rows hold Mh / 4 words, cyclically), and a byte pair differs
        // iff its xor is 1, so one popcount counts four products at once
        const uint32_t *rep32 = reinterpret_cast<const uint32_t *>(rep);
        const int Wr = Mh >> 2;
        for (int pos = blockIdx.y * blockDim.x + threadIdx.x; pos < total; pos += gridDim.y * blockDim.x) {
            const int g4 = pos % G4;
            const int pi = pos / G4;
            const int i = pi % N, p = pi / N;
            const uint32_t X = rep32[((int64_t)p * N + i) * Wr + g4];
#pragma unroll
            for (int l = 0; l < kTauLags; ++l) {
                const int q = p + lag[l];
                int m2 = 4 * g4 + (q >> 1);
                if (m2 >= Mh) m2 -= Mh;
                const uint32_t *row2 = rep32 + ((int64_t)(q & 1) * N + i) * Wr;
                const int j = m2 >> 2;
                const uint32_t lo = row2[j], hi = row2[(j + 1 == Wr) ? 0 : j + 1];
                const uint32_t Y = __builtin_amdgcn_alignbyte(hi, lo, (uint32_t)(m2 & 3));
                acc[l] += 4 - 2 * (int)__popc(X ^ Y);
            }
        }
    } else {
    for (int pos = blockIdx.y * blockDim.x + threadIdx.x; pos < total; pos += gridDim.y * blockDim.x) {
        const int g4 = pos % G4;
        const int pi = pos / G4;
        const int i = pi % N, p = pi / N;
        const uint8_t *row = rep + (int64_t)p * N * Mh + (int64_t)i * Mh;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int m = 4 * g4 + b;
            if (m >= Mh) break;
            const int x = row[m];
#pragma unroll
            for (int l = 0; l < kTauLags; ++l) {
                int y = x;  // M == 1: the slice meets itself
                if (M >= 2) {
                    const int q = p + lag[l];
                    int m2 = m + (q >> 1);
                    if (m2 >= Mh) m2 -= Mh;
                    y = rep[(int64_t)(q & 1) * N * Mh + (int64_t)i * Mh + m2];
                }
                acc[l] += 1 - 2 * (x ^ y);
            }
        }
    }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int l = 0; l < kTauLags; ++l) {
        const long long v = wave_sum((long long)acc[l]);
        if (lane == 0) red[wave][l] = v;
    }
    __syncthreads();
    if (threadIdx.x < kTauLags) {
        long long v = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += red[w][threadIdx.x];
        const int r = st.rung_of[g];
        atomicAdd(reinterpret_cast<unsigned long long *>(&st.sumCt[((int64_t)d.rep_base + r) * kTauLags + threadIdx.x]),
                  (unsigned long long)v);
    }
}

__global__ void advance_kernel(DevState st, int32_t n_inst, uint32_t t_add)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n < n_inst) st.ctr[n].t += t_add;
}

__global__ void threshold_eval_kernel(const double *dS, uint32_t *out, int32_t n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = threshold(dS[i]);
}

}  // namespace

// ------------------------------------------------------------------ launchers

int32_t sweep_tile_lds_bytes(const InstDesc &d, int32_t n_adj, int32_t P)
{
    int64_t o[10];
    const int64_t x = carve_offsets(d, n_adj, P, o);
    return (int32_t)(x > 0x7fffffff ? 0x7fffffff : x);
}

int32_t block_tile_lds_bytes(const InstDesc &d, int32_t P, int32_t ng)
{
    int64_t o[7];
    const int64_t x = block_offsets(d, P, ng, o);
    return (int32_t)(x > 0x7fffffff ? 0x7fffffff : x);
}

hipError_t sweep_kernels_set_lds(int32_t fast_bytes, int32_t generic_bytes, int32_t block_bytes)
{
    const struct {
        const void *fn;
        int32_t bytes;
    } k[] = {
        {reinterpret_cast<const void *>(&sweep_block_kernel<false, false>), block_bytes},
        {reinterpret_cast<const void *>(&sweep_block_kernel<true, false>), block_bytes},
        {reinterpret_cast<const void *>(&sweep_block_kernel<false, true>), block_bytes},
        {reinterpret_cast<const void *>(&sweep_block_kernel<true, true>), block_bytes},
        {reinterpret_cast<const void *>(&sweep_fast_kernel<false>), fast_bytes},
        {reinterpret_cast<const void *>(&sweep_fast_kernel<true>), fast_bytes},
        {reinterpret_cast<const void *>(&sweep_fast_kernel<true, true>), fast_bytes},
        {reinterpret_cast<const void *>(&sweep_fast_kernel<false, false, true>), fast_bytes},
        {reinterpret_cast<const void *>(&sweep_fast_kernel<true, false, true>), fast_bytes},
        {reinterpret_cast<const void *>(&sweep_generic_kernel<false>), generic_bytes},
        {reinterpret_cast<const void *>(&sweep_generic_kernel<true>), generic_bytes},
    };
    for (const auto &x : k) {
        if (x.bytes <= 0) continue;
        const hipError_t e = hipFuncSetAttribute(x.fn, hipFuncAttributeMaxDynamicSharedMemorySize, x.bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t block_resident_per_cu(int32_t threads, int32_t lds_bytes, int32_t *per_cu)
{
    int a = 0, b = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &a, reinterpret_cast<const void *>(&sweep_block_kernel<false, true>), threads, lds_bytes);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &b, reinterpret_cast<const void *>(&sweep_block_kernel<true, true>), threads, lds_bytes);
    if (e != hipSuccess) return e;
    *per_cu = a < b ? a : b;
    return hipSuccess;
}

hipError_t launch_init_spins(const DevState &st, int32_t n_reps, uint32_t key0, uint32_t key1,
                             hipStream_t s)
{
    if (n_reps <= 0) return hipSuccess;
    hipLaunchKernelGGL(init_spins_kernel, dim3(n_reps), dim3(256), 0, s, st, key0, key1);
    return hipGetLastError();
}

hipError_t launch_energy(const DevState &st, int32_t rep_first, int32_t n_reps, hipStream_t s)
{
    if (n_reps <= 0) return hipSuccess;
    hipLaunchKernelGGL(energy_kernel, dim3(n_reps), dim3(256), 0, s, st, rep_first);
    return hipGetLastError();
}

hipError_t launch_sweep(const SweepLaunch &L, int kind, hipStream_t s)
{
    if (L.n_tiles <= 0) return hipSuccess;
    const dim3 grid(L.n_tiles), block(L.block_threads);
    const bool fuse = L.fuse_exchange != 0;
    if (kind == kTileFast) {
        if (fuse && L.cycles > 1)
            hipLaunchKernelGGL((sweep_fast_kernel<true, true>), grid, block, L.lds_bytes, s, L);
        else if (L.lat && fuse)
            hipLaunchKernelGGL((sweep_fast_kernel<true, false, true>), grid, block, L.lds_bytes, s, L);
        else if (L.lat)
            hipLaunchKernelGGL((sweep_fast_kernel<false, false, true>), grid, block, L.lds_bytes, s, L);
        else if (fuse)
            hipLaunchKernelGGL(sweep_fast_kernel<true>, grid, block, L.lds_bytes, s, L);
        else
            hipLaunchKernelGGL(sweep_fast_kernel<false>, grid, block, L.lds_bytes, s, L);
    } else if (kind == kTileBlock) {
        if (L.persist) {
            if (fuse)
                hipLaunchKernelGGL((sweep_block_kernel<true, true>), grid, block, L.lds_bytes, s, L);
            else
                hipLaunchKernelGGL((sweep_block_kernel<false, true>), grid, block, L.lds_bytes, s, L);
        } else {
            if (fuse)
                hipLaunchKernelGGL((sweep_block_kernel<true, false>), grid, block, L.lds_bytes, s, L);
            else
                hipLaunchKernelGGL((sweep_block_kernel<false, false>), grid, block, L.lds_bytes, s, L);
        }
    } else {
        if (fuse)
            hipLaunchKernelGGL(sweep_generic_kernel<true>, grid, block, L.lds_bytes, s, L);
        else
            hipLaunchKernelGGL(sweep_generic_kernel<false>, grid, block, L.lds_bytes, s, L);
    }
    return hipGetLastError();
}

hipError_t launch_block_prepare(const SweepLaunch &L, hipStream_t s)
{
    if (L.n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(block_prepare_kernel, dim3(L.n_tiles), dim3(256), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_exchange(const DevState &st, int32_t n_inst, uint32_t key0, uint32_t key1,
                           uint32_t t_add, hipStream_t s)
{
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(exchange_kernel, dim3(n_inst), dim3(64), 0, s, st, key0, key1, t_add);
    return hipGetLastError();
}

hipError_t launch_tau_corr(const DevState &st, int32_t n_reps, int32_t chunks, hipStream_t s)
{
    if (n_reps <= 0 || chunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(tau_corr_kernel, dim3(n_reps, chunks), dim3(256), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_advance(const DevState &st, int32_t n_inst, uint32_t t_add, hipStream_t s)
{
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(advance_kernel, dim3((n_inst + 255) / 256), dim3(256), 0, s, st, n_inst, t_add);
    return hipGetLastError();
}

hipError_t launch_threshold_eval(const double *dS, uint32_t *out, int32_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(threshold_eval_kernel, dim3((n + 255) / 256), dim3(256), 0, s, dS, out, n);
    return hipGetLastError();
}

}  // namespace ptq
