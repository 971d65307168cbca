// pt_kernels.hip -- gfx950 kernels of the parallel-tempering sampler.
//
//   init_spins   draws the initial spins (INIT-domain Philox words)
//   energy       E_cl and C of replicas from their spins in device memory
//   sweep_tile   n Metropolis sweeps of a tile of replicas held in LDS, colour class by
//                colour class, then E_cl and C of each replica from the final spins
//   exchange     one even/odd replica-exchange step per instance (one workgroup each)
//   advance      t += n
#include "pt_internal.h"

#pragma clang fp contract(off)

namespace ptq {

namespace {

constexpr int kWave = 64;

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

__device__ __forceinline__ size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// ------------------------------------------------------------------ init

__global__ void init_spins_kernel(DevState st, const int32_t *rep_inst, uint32_t key0,
                                  uint32_t key1)
{
    const int g = blockIdx.x;  // global replica
    const int n = rep_inst[g];
    const InstDesc d = st.inst[n];
    const int c = g - d.rep_base;
    int8_t *base = st.spins + d.spin_base + (int64_t)c * d.M * d.Npad;
    const int items = d.M * d.Nq;
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
        const int k = it / d.Nq;
        const int q = it - k * d.Nq;
        const Words4 u = philox10((uint32_t)k * (uint32_t)d.Nq + (uint32_t)q, 0u, (uint32_t)c,
                                  (uint32_t)n, key0, key1);
        uint32_t packed = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = 4 * q + b;
            const uint32_t v = (i < d.N) ? ((u.w[b] >> 31) ? 0x01u : 0xFFu) : 0u;
            packed |= v << (8 * b);
        }
        *reinterpret_cast<uint32_t *>(base + (int64_t)k * d.Npad + 4 * q) = packed;
    }
}

// ------------------------------------------------------------------ energy from global

__global__ void energy_kernel(DevState st, const int32_t *rep_inst, int32_t rep_first)
{
    __shared__ long long scratch[16];
    const int g = rep_first + blockIdx.x;
    const int n = rep_inst[g];
    const InstDesc d = st.inst[n];
    const int c = g - d.rep_base;
    const int8_t *base = st.spins + d.spin_base + (int64_t)c * d.M * d.Npad;
    const int32_t *off = st.adj_off + d.site_base + n;
    const int32_t *adj = st.adj + d.adj_base;
    const int16_t *hf = st.hfield + d.site_base;
    long long e2 = 0, cc = 0;
    for (int it = threadIdx.x; it < d.M * d.N; it += blockDim.x) {
        const int k = it / d.N;
        const int i = it - k * d.N;
        const int8_t *row = base + (int64_t)k * d.Npad;
        const int s = row[i];
        int f = 2 * hf[i];
        for (int e = off[i]; e < off[i + 1]; ++e) {
            const int a = adj[e];
            f += (a >> 16) * row[a & 0xFFFF];
        }
        e2 += (long long)s * f;
        if (d.M >= 2) {
            const int8_t *nxt = base + (int64_t)((k + 1 == d.M) ? 0 : k + 1) * d.Npad;
            cc += (long long)s * nxt[i];
        }
    }
    e2 = block_sum(e2, scratch);
    cc = block_sum(cc, scratch);
    if (threadIdx.x == 0) {
        st.E[g] = e2 / 2;
        st.C[g] = cc;
    }
}

// ------------------------------------------------------------------ sweep

struct TileLds {
    int8_t *sp;
    int32_t *adj;
    int32_t *off;
    int16_t *h;
    uint32_t *blk;
    int32_t *cls;
    uint32_t *tbl;
    long long *red;
};

__device__ __forceinline__ TileLds carve(char *lds, const InstDesc &d, int n_adj, int n_blk,
                                         int P)
{
    TileLds t;
    size_t o = 0;
    t.sp = reinterpret_cast<int8_t *>(lds + o);
    o = align16(o + (size_t)P * d.M * d.Npad);
    t.adj = reinterpret_cast<int32_t *>(lds + o);
    o = align16(o + (size_t)n_adj * 4);
    t.off = reinterpret_cast<int32_t *>(lds + o);
    o = align16(o + (size_t)(d.N + 1) * 4);
    t.h = reinterpret_cast<int16_t *>(lds + o);
    o = align16(o + (size_t)d.N * 2);
    t.blk = reinterpret_cast<uint32_t *>(lds + o);
    o = align16(o + (size_t)n_blk * 4);
    t.cls = reinterpret_cast<int32_t *>(lds + o);
    o = align16(o + (size_t)(d.n_colors + 1) * 4);
    t.tbl = reinterpret_cast<uint32_t *>(lds + o);
    o = align16(o + (size_t)P * d.tbl_words * 4);
    t.red = reinterpret_cast<long long *>(lds + o);
    return t;
}

__global__ void __launch_bounds__(1024) sweep_tile_kernel(SweepLaunch L)
{
    extern __shared__ __align__(16) char lds[];
    const DevState &st = L.st;
    const Tile tile = st.tiles[blockIdx.x];
    const int n = tile.inst;
    const InstDesc d = st.inst[n];
    const int P = tile.P;
    const int c0 = tile.c0;
    const int32_t *goff = st.adj_off + d.site_base + n;
    const int n_adj = goff[d.N] - goff[0];
    const int32_t *gcls = st.cls_off + d.cls_base;
    const int n_blk = gcls[d.n_colors] - gcls[0];
    TileLds t = carve(lds, d, n_adj, n_blk, P);
    const int tid = threadIdx.x;
    const int nt = blockDim.x;

    // stage the tile: spins, neighbour lists, fields, colour blocks, rung tables
    {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(
            st.spins + d.spin_base + (int64_t)c0 * d.M * d.Npad);
        uint32_t *dst = reinterpret_cast<uint32_t *>(t.sp);
        const int words = P * d.M * d.Npad / 4;
        for (int w = tid; w < words; w += nt) dst[w] = src[w];
        const int a0 = goff[0];
        for (int e = tid; e < n_adj; e += nt) t.adj[e] = st.adj[d.adj_base + e];
        for (int i = tid; i <= d.N; i += nt) t.off[i] = goff[i] - a0;
        for (int i = tid; i < d.N; i += nt) t.h[i] = st.hfield[d.site_base + i];
        const int b0 = gcls[0];
        for (int e = tid; e < n_blk; e += nt) t.blk[e] = st.blk[d.blk_base + e];
        for (int g = tid; g <= d.n_colors; g += nt) t.cls[g] = gcls[g] - b0;
        for (int q = 0; q < P; ++q) {
            const int rung = st.rung_of[d.rep_base + c0 + q];
            const uint32_t *tsrc = st.tbl + d.tbl_base + (int64_t)rung * d.tbl_words;
            for (int w = tid; w < d.tbl_words; w += nt) t.tbl[q * d.tbl_words + w] = tsrc[w];
        }
    }
    const uint64_t t0 = st.ctr[n].t;
    __syncthreads();

    const int M = d.M, N = d.N, Npad = d.Npad, F = d.F;
    const int parities = (M >= 2) ? 2 : 1;
    const int Mc = (M >= 2) ? M / 2 : 1;
    const int bstride = 2 * F + 1;

    for (int sw = 0; sw < L.n_sweeps; ++sw) {
        const uint32_t tt = (uint32_t)(t0 + (uint64_t)sw);
        for (int p = 0; p < parities; ++p) {
            for (int g = 0; g < d.n_colors; ++g) {
                const int e0 = t.cls[g];
                const int nb = t.cls[g + 1] - e0;
                const int per_rep = Mc * nb;
                const int items = P * per_rep;
                for (int it = tid; it < items; it += nt) {
                    const int q = it / per_rep;
                    const int rem = it - q * per_rep;
                    const int mi = rem / nb;
                    const int ei = rem - mi * nb;
                    const int k = (M >= 2) ? 2 * mi + p : 0;
                    const uint32_t ent = t.blk[e0 + ei];
                    const int bq = (int)(ent >> 4);
                    const uint32_t mask = ent & 15u;
                    const Words4 u = philox10((uint32_t)k * (uint32_t)d.Nq + (uint32_t)bq, tt,
                                              (uint32_t)(c0 + q), (uint32_t)n, L.key0, L.key1);
                    int8_t *row = t.sp + (q * M + k) * Npad;
                    const int8_t *prv = t.sp + (q * M + (k == 0 ? M - 1 : k - 1)) * Npad;
                    const int8_t *nxt = t.sp + (q * M + (k + 1 == M ? 0 : k + 1)) * Npad;
                    const uint32_t *tb = t.tbl + q * d.tbl_words;
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        if (!((mask >> b) & 1u)) continue;
                        const int i = 4 * bq + b;
                        const int s = row[i];
                        int f = t.h[i];
                        for (int e = t.off[i]; e < t.off[i + 1]; ++e) {
                            const int a = t.adj[e];
                            f += (a >> 16) * row[a & 0xFFFF];
                        }
                        const int tau = (M >= 2) ? ((prv[i] + nxt[i]) >> 1) + 1 : 1;
                        const int idx = ((s > 0 ? bstride : 0) + f + F) * 3 + tau;
                        if (u.w[b] <= tb[idx]) row[i] = (int8_t)(-s);
                    }
                }
                __syncthreads();
            }
        }
    }
    (void)N;

    // energies of the final configuration, then write the spins back
    for (int q = 0; q < P; ++q) {
        long long e2 = 0, cc = 0;
        for (int it = tid; it < M * N; it += nt) {
            const int k = it / N;
            const int i = it - k * N;
            const int8_t *row = t.sp + (q * M + k) * Npad;
            const int s = row[i];
            int f = 2 * t.h[i];
            for (int e = t.off[i]; e < t.off[i + 1]; ++e) {
                const int a = t.adj[e];
                f += (a >> 16) * row[a & 0xFFFF];
            }
            e2 += (long long)s * f;
            if (M >= 2) cc += (long long)s * t.sp[(q * M + (k + 1 == M ? 0 : k + 1)) * Npad + i];
        }
        e2 = block_sum(e2, t.red);
        cc = block_sum(cc, t.red);
        if (tid == 0) {
            st.E[d.rep_base + c0 + q] = e2 / 2;
            st.C[d.rep_base + c0 + q] = cc;
        }
    }
    {
        uint32_t *dst = reinterpret_cast<uint32_t *>(st.spins + d.spin_base +
                                                     (int64_t)c0 * d.M * d.Npad);
        const uint32_t *src = reinterpret_cast<const uint32_t *>(t.sp);
        const int words = P * d.M * d.Npad / 4;
        for (int w = tid; w < words; w += nt) dst[w] = src[w];
    }
}

// ------------------------------------------------------------------ exchange

__global__ void exchange_kernel(DevState st, uint32_t key0, uint32_t key1, uint32_t t_add)
{
    const int n = blockIdx.x;
    const InstDesc d = st.inst[n];
    const int R = d.R;
    const int base = d.rep_base;
    const int pb = d.pair_base;
    const uint64_t e = st.ctr[n].e;
    const int par = (int)(e & 1u);
    for (int j = threadIdx.x;; j += blockDim.x) {
        const int r = par + 2 * j;
        if (r + 1 >= R) break;
        const int x = st.replica_of[base + r];
        const int y = st.replica_of[base + r + 1];
        const double dE = (double)(st.E[base + x] - st.E[base + y]);
        const double dC = (double)(st.C[base + x] - st.C[base + y]);
        const double D = st.db[pb + r] * dE - st.dK[pb + r] * dC;
        const uint32_t thr = threshold(-D);
        const uint32_t u = philox10((uint32_t)r, (uint32_t)e, 0u, (uint32_t)n, key0, key1).w[0];
        st.att[pb + r] += 1;
        if (u <= thr) {
            st.replica_of[base + r] = y;
            st.replica_of[base + r + 1] = x;
            st.rung_of[base + y] = r;
            st.rung_of[base + x] = r + 1;
            st.acc[pb + r] += 1;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int cold = st.replica_of[base];
        const int hot = st.replica_of[base + R - 1];
        const int lc = st.label[base + cold];
        if (lc == 2) {
            st.rt[base + cold] += 1;
            st.label[base + cold] = 1;
        } else if (lc == 0) {
            st.label[base + cold] = 1;
        }
        if (st.label[base + hot] == 1) st.label[base + hot] = 2;
    }
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        const int c = st.replica_of[base + r];
        const long long E = st.E[base + c];
        const long long C = st.C[base + c];
        st.sumE[base + r] += E;
        st.sumC[base + r] += C;
        st.sumE2[base + r] += E * E;
        st.sumC2[base + r] += C * C;
    }
    if (threadIdx.x == 0) {
        st.ctr[n].e = e + 1;
        st.ctr[n].n_acc += 1;
        st.ctr[n].t += t_add;
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

int32_t sweep_tile_lds_bytes(const InstDesc &d, int32_t n_adj, int32_t n_blk, int32_t P)
{
    auto a16 = [](int64_t x) { return (x + 15) & ~(int64_t)15; };
    int64_t o = 0;
    o = a16(o + (int64_t)P * d.M * d.Npad);
    o = a16(o + (int64_t)n_adj * 4);
    o = a16(o + (int64_t)(d.N + 1) * 4);
    o = a16(o + (int64_t)d.N * 2);
    o = a16(o + (int64_t)n_blk * 4);
    o = a16(o + (int64_t)(d.n_colors + 1) * 4);
    o = a16(o + (int64_t)P * d.tbl_words * 4);
    o = a16(o + 16 * 8);
    return (int32_t)(o > 0x7fffffff ? 0x7fffffff : o);
}

hipError_t sweep_kernel_set_lds(int32_t bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&sweep_tile_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t launch_init_spins(const DevState &st, const int32_t *rep_inst, int32_t n_reps,
                             uint32_t key0, uint32_t key1, hipStream_t s)
{
    if (n_reps <= 0) return hipSuccess;
    hipLaunchKernelGGL(init_spins_kernel, dim3(n_reps), dim3(256), 0, s, st, rep_inst, key0, key1);
    return hipGetLastError();
}

hipError_t launch_energy(const DevState &st, const int32_t *rep_inst, int32_t rep_first,
                         int32_t n_reps, hipStream_t s)
{
    if (n_reps <= 0) return hipSuccess;
    hipLaunchKernelGGL(energy_kernel, dim3(n_reps), dim3(256), 0, s, st, rep_inst, rep_first);
    return hipGetLastError();
}

hipError_t launch_sweep(const SweepLaunch &L, hipStream_t s)
{
    if (L.n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(sweep_tile_kernel, dim3(L.n_tiles), dim3(L.block_threads), L.lds_bytes, s, L);
    return hipGetLastError();
}

hipError_t launch_exchange(const DevState &st, int32_t n_inst, uint32_t key0, uint32_t key1,
                           uint32_t t_add, hipStream_t s)
{
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(exchange_kernel, dim3(n_inst), dim3(64), 0, s, st, key0, key1, t_add);
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
