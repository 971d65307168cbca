// pt_bitpack.hip -- kernels of the bit-packed spin encoding (PT_BITPACK32).
//
// The spins of 32 replica slots share one 32-bit word: bit (c mod 32) of word group
// w = c / 32 holds x = (s + 1) / 2 of slot c.  An instance's words are laid out
// [w][p][i][m'] (parity p, site i, same-parity slice m' < 4 * G4): rows are padded to whole
// four-slice groups, and padding words and the bits of slots >= R stay 0.  The chain is
// the one of the byte-per-spin encoding: every attempt draws its own Philox word and
// reads its own rung's threshold table, so packing changes where the bits live, not what
// is computed.
//
//   bp_init          initial spins from INIT-domain Philox words
//   bp_sweep         one colour class (p, g) of one sweep of every instance
//   bp_energy_part   E_cl and C partial sums per block of positions
//   bp_energy_sum    E_cl and C of every replica slot from the partial sums
//
// Work items.  A lane serves a part j of one word group at one four-slice group; the lanes
// of a word are neighbours, combine their results with lane shuffles, and lane j = 0
// writes the word.
//   sweep:  per instance and colour g, item = ((w * Sg + si) * G4 + g4) * 8 + j (4 slots
//           per lane) for the si-th of the class's Sg sites; a sweep block is 256
//           consecutive items.
//   init, energy: per (instance, word group) the positions (p, i, g4) in the order
//           pos = (p * N + i) * G4 + g4, four lanes of 8 slots each; position block
//           `chunk` of `chunks` takes pos = chunk * 64 + lane / 4 + k * 64 * chunks.
#include "pt_internal.h"

#pragma clang fp contract(off)

namespace ptq {
namespace {

constexpr int kBpThreads = 256;   // threads of every bit-packed kernel's workgroup
constexpr int kBpPositions = 64;  // positions per workgroup pass (four lanes each)

__device__ __forceinline__ uint32_t *bp_rowp(const DevState &st, const InstDesc &d, int w, int p, int i)
{
    return reinterpret_cast<uint32_t *>(st.spins + d.spin_base) +
           ((int64_t)(w * d.parities + p) * d.N + i) * d.bp_row;
}

__device__ __forceinline__ uint32_t word_of(const uint4 &v, int b)
{
    return b == 0 ? v.x : b == 1 ? v.y : b == 2 ? v.z : v.w;
}

// OR over the four lanes of a quad (lanes 4q .. 4q+3); every lane of the quad must call it.
__device__ __forceinline__ uint32_t quad_or(uint32_t v)
{
    v |= __shfl_xor(v, 1, 64);
    v |= __shfl_xor(v, 2, 64);
    return v;
}

// Other-parity word at same-parity index idx (0 <= idx < Mh) of a row whose words
// 4*g4 .. 4*g4+3 are already in `o`.
__device__ __forceinline__ uint32_t other_word(const uint32_t *row, const uint4 &o, int g4, int idx)
{
    const int k = idx - 4 * g4;
    return (k >= 0 && k < 4) ? word_of(o, k) : row[idx];
}

// Time neighbours of same-parity slice m (slice k = 2m + p) in the other parity's row:
// k - 1 and k + 1 are other-parity indices (m - 1, m) for p = 0 and (m, m + 1) for p = 1,
// cyclically in Mh.
__device__ __forceinline__ void time_words(const uint32_t *orow, const uint4 &o, int g4, int p,
                                           int Mh, int m, uint32_t &lo, uint32_t &hi)
{
    if (p == 0) {
        lo = other_word(orow, o, g4, (m == 0) ? Mh - 1 : m - 1);
        hi = other_word(orow, o, g4, m);
    } else {
        lo = other_word(orow, o, g4, m);
        hi = other_word(orow, o, g4, (m + 1 == Mh) ? 0 : m + 1);
    }
}

// ------------------------------------------------------------------ init

__global__ void __launch_bounds__(kBpThreads) bp_init_kernel(DevState st, uint32_t key0, uint32_t key1)
{
    const int4 blk = reinterpret_cast<const int4 *>(st.bp_eblk)[blockIdx.x];
    const int n = blk.x, w = blk.y, chunk = blk.z, chunks = blk.w;
    const InstDesc d = st.inst[n];
    const int j = threadIdx.x & 3;
    const int Q = d.parities * d.N * d.G4;
    for (int pos = chunk * kBpPositions + (threadIdx.x >> 2); pos < Q; pos += kBpPositions * chunks) {
        const int g4 = pos % d.G4;
        const int pi = pos / d.G4;
        const int i = pi % d.N, p = pi / d.N;
        uint32_t x[4] = {0u, 0u, 0u, 0u};
        for (int r = 0; r < 8; ++r) {
            const int c = 32 * w + 8 * j + r;
            if (c >= d.R) break;
            const Words4 u = philox10((uint32_t)(2 * i + p) * (uint32_t)d.G4 + (uint32_t)g4, 0u,
                                      (uint32_t)c, (uint32_t)n, key0, key1);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (4 * g4 + b < d.Mh) x[b] |= (u.w[b] >> 31) << (8 * j + r);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) x[b] = quad_or(x[b]);
        if (j == 0)
            *reinterpret_cast<uint4 *>(bp_rowp(st, d, w, p, i) + 4 * g4) = make_uint4(x[0], x[1], x[2], x[3]);
    }
}

// ------------------------------------------------------------------ sweep

// OR over the eight lanes of an octet (lanes 8q .. 8q+7); every lane of it must call it.
__device__ __forceinline__ uint32_t octet_or(uint32_t v)
{
    v |= __shfl_xor(v, 1, 64);
    v |= __shfl_xor(v, 2, 64);
    v |= __shfl_xor(v, 4, 64);
    return v;
}

// Byte spread of 4 bits: bit r of v becomes bit 0 of byte r (v * (1 + 2^7 + 2^14 + 2^21)
// moves bit r by 7r, and only r = k lands on bit 8k).
__device__ __forceinline__ uint32_t spread4(uint32_t v)
{
    return (v * 0x00204081u) & 0x01010101u;
}

// One colour class (p, g) of one sweep.  A lane serves kBpSweepLanes-th of a word group
// (kBpSlots = 4 slots) at one four-slice group: item = ((w * Sg + si) * G4 + g4) * 8 + j,
// the eight lanes of a word are neighbouring and OR their flip masks together.
constexpr int kBpSlots = 32 / kBpSweepLanes;
// Sites of at most this degree load all their neighbours' words at once.
constexpr int kBpMaxDegree = 8;

__global__ void __launch_bounds__(kBpThreads) bp_sweep_kernel(BpLaunch L)
{
    const DevState &st = L.st;
    const int2 blk = reinterpret_cast<const int2 *>(st.bp_sblk)[L.blk0 + blockIdx.x];
    const int n = blk.x;
    const InstDesc d = st.inst[n];
    if (L.p >= d.parities) return;  // the whole block: M == 1 has one parity
    const int p = L.p, g = L.g;
    const int cls0 = st.cls_off[d.cls_base + g];
    const int Sg = st.cls_off[d.cls_base + g + 1] - cls0;
    const int G4 = d.G4, Mh = d.Mh, F = d.F;
    const int item = blk.y + (int)threadIdx.x;
    const bool valid = item < d.bp_W * Sg * G4 * kBpSweepLanes;  // a whole octet or none
    const int j = item % kBpSweepLanes;
    int rest = item / kBpSweepLanes;
    const int g4 = rest % G4;
    rest /= G4;
    const int si = rest % Sg;
    const int w = rest / Sg;
    uint32_t flip[4] = {0u, 0u, 0u, 0u};
    uint4 X = make_uint4(0u, 0u, 0u, 0u);
    uint32_t *own = nullptr;
    if (valid) {
        const int i = st.csite[d.site_base + cls0 + si];
        own = bp_rowp(st, d, w, p, i) + 4 * g4;
        X = *reinterpret_cast<const uint4 *>(own);
        // time field: tau = x(k-1) + x(k+1) per slot and slice (1 when M == 1)
        uint32_t tlo[4] = {0u, 0u, 0u, 0u}, thi[4] = {0u, 0u, 0u, 0u};
        if (d.M >= 2) {
            const uint32_t *orow = bp_rowp(st, d, w, 1 - p, i);
            const uint4 o = *reinterpret_cast<const uint4 *>(orow + 4 * g4);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (4 * g4 + b < Mh) time_words(orow, o, g4, p, Mh, 4 * g4 + b, tlo[b], thi[b]);
        }
        // spatial field f = h_i + sum_j J_ij s_j for the 4 slots x 4 slices of this lane
        const int32_t *off = st.adj_off + d.off_base;
        const int32_t *adj = st.adj + d.adj_base;
        const int sh = kBpSlots * j;
        const uint32_t tt = (uint32_t)(st.ctr[n].t + (uint64_t)L.sweep_off);
        const uint32_t ctr0 = (uint32_t)(2 * i + p) * (uint32_t)G4 + (uint32_t)g4;
        const int bstride = 2 * F + 1;
        int f[4][kBpSlots];
        // table index (x (2F+1) + f + F) * 3 + tau of every (slice, slot): with F <= 20 it
        // is below 256 and is formed for the lane's 4 slots at once, one byte each
        uint32_t idx4[4] = {0u, 0u, 0u, 0u};
        const bool byte_index = F <= 20;
        if (F <= 127) {
            // f = h_i - sum_j |J_ij| + 2 sum_j |J_ij| [x_j == (J_ij > 0)]: the sum runs in
            // one byte per slot (it is at most F), the lane's 4 slots in one word per slice
            int base = st.hfield[d.site_base + i];
            uint32_t acc[4] = {0u, 0u, 0u, 0u};
            auto add_neighbour = [&](int a, const uint4 &Y) {
                const int J = a >> 16;
                const uint32_t aJ = (uint32_t)(J < 0 ? -J : J);
                const uint32_t neg = J < 0 ? 0xFu : 0u;
                base -= (int)aJ;
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[b] += aJ * spread4(((word_of(Y, b) >> sh) & 0xFu) ^ neg);
            };
            const int e0 = off[i], deg = off[i + 1] - e0;
            if (deg <= kBpMaxDegree) {
                // All entries, then all neighbour words, in flight together (integer sums:
                // the order cannot matter).  Slots past the degree hold the site itself with
                // J = 0, so every word load is unconditional (a load under a branch would be
                // waited for where the branch ends) and adds nothing.
                int av[kBpMaxDegree];
                uint4 Yv[kBpMaxDegree];
#pragma unroll
                for (int k = 0; k < kBpMaxDegree; ++k) av[k] = (k < deg) ? adj[e0 + k] : i;
#pragma unroll
                for (int k = 0; k < kBpMaxDegree; ++k)
                    Yv[k] = *reinterpret_cast<const uint4 *>(bp_rowp(st, d, w, p, av[k] & 0xFFFF) + 4 * g4);
#pragma unroll
                for (int k = 0; k < kBpMaxDegree; ++k) add_neighbour(av[k], Yv[k]);
            } else {
                for (int e = e0; e < e0 + deg; ++e) {
                    const int a = adj[e];
                    add_neighbour(a, *reinterpret_cast<const uint4 *>(bp_rowp(st, d, w, p, a & 0xFFFF) + 4 * g4));
                }
            }
            if (byte_index) {
                // V = x (2F+1) + f + F = x (2F+1) + (base + F) + 2 acc, with base + F >= 0
                // (|h_i| + sum_j |J_ij| <= F) and V <= 4F + 1, so no byte carries over
                const uint32_t bF = (uint32_t)(base + F) * 0x01010101u;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const uint32_t xb = spread4((word_of(X, b) >> sh) & 0xFu);
                    const uint32_t tb4 = (d.M >= 2) ? spread4((tlo[b] >> sh) & 0xFu) + spread4((thi[b] >> sh) & 0xFu)
                                                    : 0x01010101u;
                    const uint32_t V = xb * (uint32_t)bstride + bF + 2u * acc[b];
                    idx4[b] = V * 3u + tb4;
                }
            } else {
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int r = 0; r < kBpSlots; ++r) f[b][r] = base + 2 * (int)((acc[b] >> (8 * r)) & 0xFFu);
            }
        } else {
            // f = h_i - sum_j J_ij + 2 sum_j J_ij x_j, slot by slot
            int base = st.hfield[d.site_base + i];
            for (int e = off[i]; e < off[i + 1]; ++e) base -= adj[e] >> 16;
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int r = 0; r < kBpSlots; ++r) f[b][r] = base;
            for (int e = off[i]; e < off[i + 1]; ++e) {
                const int a = adj[e];
                const int J2 = 2 * (a >> 16);
                const uint4 Y = *reinterpret_cast<const uint4 *>(bp_rowp(st, d, w, p, a & 0xFFFF) + 4 * g4);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const uint32_t y = word_of(Y, b) >> sh;
#pragma unroll
                    for (int r = 0; r < kBpSlots; ++r) f[b][r] += J2 * (int)((y >> r) & 1u);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < kBpSlots; ++r) {
            const int c = 32 * w + sh + r;
            if (c >= d.R) break;
            const uint32_t *tb = st.tbl + d.tbl_base + (int64_t)st.rung_of[d.rep_base + c] * d.tbl_words;
            const Words4 u = philox10(ctr0, tt, (uint32_t)c, (uint32_t)n, L.key0, L.key1);
            const int bit = sh + r;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (4 * g4 + b >= Mh) break;
                int idx;
                if (byte_index) {
                    idx = (int)((idx4[b] >> (8 * r)) & 0xFFu);
                } else {
                    const int x = (int)((word_of(X, b) >> bit) & 1u);
                    const int tau = (d.M >= 2) ? (int)((tlo[b] >> bit) & 1u) + (int)((thi[b] >> bit) & 1u) : 1;
                    idx = (x * bstride + f[b][r] + F) * 3 + tau;
                }
                if (u.w[b] <= tb[idx]) flip[b] |= 1u << bit;
            }
        }
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) flip[b] = octet_or(flip[b]);
    if (valid && j == 0 && (flip[0] | flip[1] | flip[2] | flip[3]))
        *reinterpret_cast<uint4 *>(own) = make_uint4(X.x ^ flip[0], X.y ^ flip[1], X.z ^ flip[2], X.w ^ flip[3]);
}

// ------------------------------------------------------------------ energies

// Partial sums of 2 E_cl and C over one position block, for the 32 slots of its word
// group: 2 E_cl = sum_{k,i} s_i^k (2 h_i + sum_j J_ij s_j^k), C = sum_{k,i} s_i^k s_i^{k+1}.
__global__ void __launch_bounds__(kBpThreads) bp_energy_part_kernel(DevState st)
{
    __shared__ long long red[kBpThreads / 64][32][2];
    const int4 blk = reinterpret_cast<const int4 *>(st.bp_eblk)[blockIdx.x];
    const int n = blk.x, w = blk.y, chunk = blk.z, chunks = blk.w;
    const InstDesc d = st.inst[n];
    const int j = threadIdx.x & 3;
    const int sh = 8 * j;
    const int Q = d.parities * d.N * d.G4;
    const int32_t *off = st.adj_off + d.off_base;
    const int32_t *adj = st.adj + d.adj_base;
    int e2[8], cc[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) e2[r] = cc[r] = 0;
    for (int pos = chunk * kBpPositions + (threadIdx.x >> 2); pos < Q; pos += kBpPositions * chunks) {
        const int g4 = pos % d.G4;
        const int pi = pos / d.G4;
        const int i = pi % d.N, p = pi / d.N;
        const uint4 X = *reinterpret_cast<const uint4 *>(bp_rowp(st, d, w, p, i) + 4 * g4);
        // 2 h_i + sum_j J_ij s_j = 2 h_i - sum_j J_ij + 2 sum_j J_ij x_j
        int base = 2 * st.hfield[d.site_base + i];
        for (int e = off[i]; e < off[i + 1]; ++e) base -= adj[e] >> 16;
        int f[4][8];
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 8; ++r) f[b][r] = base;
        auto add_neighbour = [&](int a, const uint4 &Y) {
            const int J2 = 2 * (a >> 16);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const uint32_t y = word_of(Y, b) >> sh;
#pragma unroll
                for (int r = 0; r < 8; ++r) f[b][r] += J2 * (int)((y >> r) & 1u);
            }
        };
        const int e0 = off[i], deg = off[i + 1] - e0;
        if (deg <= kBpMaxDegree) {
            // as in the sweep: every word load unconditional, empty slots are the site
            // itself with J = 0
            int av[kBpMaxDegree];
            uint4 Yv[kBpMaxDegree];
#pragma unroll
            for (int k = 0; k < kBpMaxDegree; ++k) av[k] = (k < deg) ? adj[e0 + k] : i;
#pragma unroll
            for (int k = 0; k < kBpMaxDegree; ++k)
                Yv[k] = *reinterpret_cast<const uint4 *>(bp_rowp(st, d, w, p, av[k] & 0xFFFF) + 4 * g4);
#pragma unroll
            for (int k = 0; k < kBpMaxDegree; ++k) add_neighbour(av[k], Yv[k]);
        } else {
            for (int e = e0; e < e0 + deg; ++e) {
                const int a = adj[e];
                add_neighbour(a, *reinterpret_cast<const uint4 *>(bp_rowp(st, d, w, p, a & 0xFFFF) + 4 * g4));
            }
        }
        // the next slice k + 1 of slice k = 2m + p: parity 1 index m (p = 0), parity 0
        // index m + 1 cyclically (p = 1)
        uint32_t nx[4] = {0u, 0u, 0u, 0u};
        if (d.M >= 2) {
            const uint32_t *orow = bp_rowp(st, d, w, 1 - p, i);
            const uint4 o = *reinterpret_cast<const uint4 *>(orow + 4 * g4);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int m = 4 * g4 + b;
                if (m < d.Mh) nx[b] = other_word(orow, o, g4, (p == 0) ? m : ((m + 1 == d.Mh) ? 0 : m + 1));
            }
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (4 * g4 + b >= d.Mh) break;
            const uint32_t xs = word_of(X, b) >> sh;
            const uint32_t ys = nx[b] >> sh;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int s = 2 * (int)((xs >> r) & 1u) - 1;
                e2[r] += s * f[b][r];
                if (d.M >= 2) cc[r] += s * (2 * (int)((ys >> r) & 1u) - 1);
            }
        }
    }
    // sum over the lanes of one quarter (lanes 4q + j of the wave), then over the waves
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        long long a = e2[r], b = cc[r];
#pragma unroll
        for (int o = 4; o < 64; o <<= 1) {
            a += __shfl_xor(a, o, 64);
            b += __shfl_xor(b, o, 64);
        }
        if (lane < 4) {
            red[wave][sh + r][0] = a;
            red[wave][sh + r][1] = b;
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int slot = threadIdx.x >> 1, k = threadIdx.x & 1;
        long long v = 0;
        for (int wv = 0; wv < kBpThreads / 64; ++wv) v += red[wv][slot][k];
        st.bp_part[((int64_t)blockIdx.x * 32 + slot) * 2 + k] = v;
    }
}

// One wave per replica slot: its lanes stride over the word group's position blocks.
__global__ void __launch_bounds__(kBpThreads) bp_energy_sum_kernel(DevState st, int32_t n_reps)
{
    const int gr = blockIdx.x * (kBpThreads / 64) + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (gr >= n_reps) return;  // the whole wave
    const int n = st.rep_inst[gr];
    const InstDesc d = st.inst[n];
    const int c = gr - d.rep_base;
    const int2 wg = reinterpret_cast<const int2 *>(st.bp_wg)[d.bp_wg_base + c / 32];
    long long e2 = 0, cc = 0;
    for (int b = lane; b < wg.y; b += 64) {
        const int64_t at = ((int64_t)(wg.x + b) * 32 + (c & 31)) * 2;
        e2 += st.bp_part[at];
        cc += st.bp_part[at + 1];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        e2 += __shfl_xor(e2, o, 64);
        cc += __shfl_xor(cc, o, 64);
    }
    if (lane == 0) {
        st.E[gr] = e2 / 2;
        st.C[gr] = cc;
    }
}

}  // namespace

hipError_t launch_bp_init(const DevState &st, int32_t n_eblk, uint32_t key0, uint32_t key1,
                          hipStream_t s)
{
    if (n_eblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(bp_init_kernel, dim3(n_eblk), dim3(kBpThreads), 0, s, st, key0, key1);
    return hipGetLastError();
}

hipError_t launch_bp_sweep(const BpLaunch &L, hipStream_t s)
{
    if (L.n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(bp_sweep_kernel, dim3(L.n_blocks), dim3(kBpThreads), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_bp_energy(const DevState &st, int32_t n_eblk, int32_t n_reps, hipStream_t s)
{
    if (n_eblk <= 0 || n_reps <= 0) return hipSuccess;
    hipLaunchKernelGGL(bp_energy_part_kernel, dim3(n_eblk), dim3(kBpThreads), 0, s, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int per_block = kBpThreads / 64;
    hipLaunchKernelGGL(bp_energy_sum_kernel, dim3((n_reps + per_block - 1) / per_block),
                       dim3(kBpThreads), 0, s, st, n_reps);
    return hipGetLastError();
}

}  // namespace ptq
