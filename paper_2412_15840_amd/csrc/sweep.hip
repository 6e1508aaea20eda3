// The triangular sweep on gfx950 (Section 2: eq. e:yi1i2iN, solved in any
// order that computes every dependency first).
//
// Entry y_i depends only on entries that are larger in exactly one index
// (i_j -> k > i_j).  The (non-singleton) modes are cut into blocks of b_j
// indices; a tile is a product of blocks and holds at most ~8k entries, so it
// lives in LDS.  A tile P depends on the tiles P + (q - P_j) e_j, q > P_j, so
// all tiles with the same block-index sum are independent: they form one
// launch, and launches run from the largest block-index sum down (a wavefront
// over tile hyperplanes).  Inside a workgroup:
//   1. the tile of C and the diagonal blocks of every T_j go to LDS;
//   2. for every mode j, the part of the sum over k > i_j that lies in tiles
//      above along j is a small contraction
//        C_tile -= T_j[rows of P_j, k >= end of P_j] x_j Y[..., k, ...],
//      computed by lanes that each own one cross-section position: they load
//      each needed Y entry once from HBM and update all b_j rows in registers,
//      with the T_j coefficients wave-uniform;
//   3. the tile itself is solved by local hyperplanes (sum of local indices,
//      descending), one barrier per local level, dividing by the eigenvalue
//      sums t_{1,i_1 i_1} + ... + t_{N,i_N i_N} (+ the singleton scalars);
//   4. the tile is written back in place.
// The adjoint operator (sum_j T_j^* x_j, lower triangular) runs the same
// machinery mirrored: ascending block sums, pulls from tiles below, conjugated
// coefficients.
#include "sylt_internal.h"

namespace sylt {
namespace {

constexpr int kThreads = kSweepThreads;
constexpr int kBmax = 8;   // largest block of a partially tiled mode
constexpr int kPrefetch = 8;  // pulled entries loaded before they are used
constexpr int kXcds = 8;   // workgroups are dealt to the XCDs round-robin
constexpr int kPerLane = (kSweepTileCap + kThreads - 1) / kThreads;  // tile entries per lane
constexpr int kMaxRounds = kSweepMaxRounds;
// packed local-solve work item: local entry t in the low bits, its local
// coordinates (the same bit layout as the code table) above
constexpr int kPackShift = 14;
constexpr int kPackMask = (1 << kPackShift) - 1;
static_assert(kSweepTileCap <= (1 << kPackShift), "tile index must fit the packed word");

// Tiles of a level are stored in Z-order; give each XCD one contiguous chunk
// of that order (workgroup b runs on XCD b % 8), so tiles that share pull
// sources run on the same L2.
__device__ __forceinline__ int tile_slot(int b, int nt)
{
    const int x = b % kXcds, slot = b / kXcds;
    const int full = nt / kXcds, rem = nt % kXcds;
    return x * full + min(x, rem) + slot;
}

struct TileState {
    int o[kMaxModes];
    int e[kMaxModes];
    int64_t base;
    int ragged;
    double2 shift;
};

// MC > 0: the number of tiled modes is the compile-time constant MC, so every
// loop over modes unrolls and the descriptor fields load once into scalar
// registers; MC == 0 handles any count at run time.
template <int MC>
__device__ __forceinline__ bool entry_ok(uint64_t c, const SweepDesc &sd, const TileState &ts)
{
    const int M = MC > 0 ? MC : sd.M;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const int w = sd.bitw[j];
        if (w == 0) continue;
        const int loc = (int)((c >> sd.bitoff[j]) & ((1ull << w) - 1ull));
        if (loc >= ts.e[j]) return false;
    }
    return true;
}

template <typename V, bool ADJ, int MC>
__global__ void __launch_bounds__(kThreads) sweep_tile_kernel(
    V *__restrict__ X, const double2 *__restrict__ Tbuf, SweepDesc sd,
    const int *__restrict__ tiles, const int64_t *__restrict__ goff,
    const uint64_t *__restrict__ code, const int *__restrict__ llist,
    const int *__restrict__ lloff, const int *__restrict__ lanetab)
{
    const int M = MC > 0 ? MC : sd.M;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double2 *tile = reinterpret_cast<double2 *>(smem_raw);
    double2 *tdiag = tile + sd.S;
    __shared__ TileState ts;

    if (threadIdx.x == 0) {
        int rem = tiles[tile_slot(blockIdx.x, gridDim.x)];
        int64_t base = 0;
        int ragged = 0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const int P = rem % sd.nb[j];
            rem /= sd.nb[j];
            ts.o[j] = P * sd.b[j];
            ts.e[j] = min(sd.b[j], sd.d[j] - ts.o[j]);
            ragged |= ts.e[j] < sd.b[j];
            base += (int64_t)ts.o[j] * sd.s[j];
        }
        double2 sh = make_double2(0.0, 0.0);
        for (int i = 0; i < sd.nsing; ++i) sh = cadd(sh, Tbuf[sd.singoff[i]]);
        ts.base = base;
        ts.ragged = ragged;
        ts.shift = ADJ ? cconj(sh) : sh;
    }
    __syncthreads();

    // 1. diagonal blocks of T_j and the tile of C
    for (int j = 0; j < M; ++j) {
        const int b = sd.b[j], e = ts.e[j], o = ts.o[j], d = sd.d[j];
        const double2 *Tj = Tbuf + sd.moff[j];
        for (int idx = threadIdx.x; idx < b * b; idx += blockDim.x) {
            const int r = idx % b, c = idx / b;
            tdiag[sd.tdoff[j] + idx] =
                (r < e && c < e) ? Tj[(o + r) + (int64_t)d * (o + c)] : make_double2(0.0, 0.0);
        }
    }
    // this lane's local-solve work, all levels at once (one memory latency)
    int pk[kMaxRounds];
    if (sd.packed) {
#pragma unroll
        for (int rr = 0; rr < kMaxRounds; ++rr)
            pk[rr] = rr < sd.rounds
                         ? lanetab[(ADJ ? rr : sd.rounds - 1 - rr) * kThreads + threadIdx.x]
                         : -1;
    }
    // tile of C: all table lookups first, then all loads
    {
        int64_t go[kPerLane];
        uint64_t cv[kPerLane];
#pragma unroll
        for (int i = 0; i < kPerLane; ++i) {
            const int t = threadIdx.x + i * kThreads;
            go[i] = t < sd.S ? goff[t] : 0;
            cv[i] = (t < sd.S && ts.ragged) ? code[t] : 0;
        }
        double2 v[kPerLane];
#pragma unroll
        for (int i = 0; i < kPerLane; ++i) {
            const int t = threadIdx.x + i * kThreads;
            const bool ok = t < sd.S && (!ts.ragged || entry_ok<MC>(cv[i], sd, ts));
            v[i] = ok ? to_d2<V>(X[ts.base + go[i]]) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int i = 0; i < kPerLane; ++i) {
            const int t = threadIdx.x + i * kThreads;
            if (t < sd.S) tile[t] = v[i];
        }
    }
    __syncthreads();

    // 2. contributions of the tiles above (below, for the adjoint) along each mode
    for (int j = 0; j < M; ++j) {
        const int o = __builtin_amdgcn_readfirstlane(ts.o[j]);
        const int e = __builtin_amdgcn_readfirstlane(ts.e[j]);
        const int d = sd.d[j];
        const int k0 = ADJ ? 0 : o + e;
        const int k1 = ADJ ? o : d;
        if (k0 >= k1) continue;  // uniform
        const int b = sd.b[j], lsj = sd.ls[j];
        const int64_t sj = sd.s[j];
        const int cs = sd.S / b;
        const double2 *Tj = Tbuf + sd.moff[j];
        for (int c = threadIdx.x; c < cs; c += blockDim.x) {
            // cross-section position c -> local entry t0 (loc_j = 0) and its
            // global offset, by mixed-radix digits over the other tiled modes
            int rem = c, t0 = 0;
            int64_t g0 = ts.base;
            bool ok = true;
#pragma unroll
            for (int i = 0; i < M; ++i) {
                const int bi = sd.b[i];
                if (i == j || bi == 1) continue;
                const int loc = rem % bi;
                rem /= bi;
                t0 += loc * sd.ls[i];
                g0 += (int64_t)loc * sd.s[i];
                ok &= loc < ts.e[i];
            }
            if (!ok) continue;
            double2 acc[kBmax];
#pragma unroll
            for (int r = 0; r < kBmax; ++r) acc[r] = make_double2(0.0, 0.0);
            for (int kb = k0; kb < k1; kb += kPrefetch) {
                double2 y[kPrefetch];
#pragma unroll
                for (int u = 0; u < kPrefetch; ++u)
                    y[u] = kb + u < k1 ? to_d2<V>(X[g0 + (int64_t)(kb + u - o) * sj])
                                       : make_double2(0.0, 0.0);
#pragma unroll
                for (int u = 0; u < kPrefetch; ++u) {
                    const int k = kb + u;
                    if (k >= k1) break;  // uniform
#pragma unroll
                    for (int r = 0; r < kBmax; ++r) {
                        if (r < e) {
                            if (ADJ)
                                acc[r] = cmac_conj(acc[r], Tj[k + (int64_t)d * (o + r)], y[u]);
                            else
                                acc[r] = cmac(acc[r], Tj[(o + r) + (int64_t)d * k], y[u]);
                        }
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < kBmax; ++r)
                if (r < e) tile[t0 + r * lsj] = csub(tile[t0 + r * lsj], acc[r]);
        }
        __syncthreads();
    }

    // 3. local hyperplanes
    auto solve_entry = [&](int t, uint64_t c) {
        if (ts.ragged && !entry_ok<MC>(c, sd, ts)) return;
        double2 num = tile[t];
        double2 den = ts.shift;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const int w = sd.bitw[j];
            const int loc = w ? (int)((c >> sd.bitoff[j]) & ((1ull << w) - 1ull)) : 0;
            const int b = sd.b[j], lsj = sd.ls[j];
            const double2 *Td = tdiag + sd.tdoff[j];
            const double2 lam = Td[loc + b * loc];
            den = cadd(den, ADJ ? cconj(lam) : lam);
            if (ADJ) {
                for (int q = 1; q <= loc; ++q)
                    num = csub(num, cmul(cconj(Td[(loc - q) + b * loc]), tile[t - q * lsj]));
            } else {
                const int qmax = ts.e[j] - 1 - loc;
                for (int q = 1; q <= qmax; ++q)
                    num = csub(num, cmul(Td[loc + b * (loc + q)], tile[t + q * lsj]));
            }
        }
        tile[t] = cdiv(num, den);
    };
    if (sd.packed) {
        // rounds in processing order; a barrier wherever the local level changes
#pragma unroll
        for (int rr = 0; rr < kMaxRounds; ++rr) {
            if (rr >= sd.rounds) break;  // uniform
            const int ri = ADJ ? rr : sd.rounds - 1 - rr;
            if (rr > 0 && sd.round_level[ri] != sd.round_level[ADJ ? ri - 1 : ri + 1]) __syncthreads();
            if (pk[rr] >= 0) solve_entry(pk[rr] & kPackMask, (uint64_t)(pk[rr] >> kPackShift));
        }
        __syncthreads();
    } else {
        for (int step = 0; step < sd.nll; ++step) {
            const int lv = ADJ ? step : sd.nll - 1 - step;
            const int i0 = lloff[lv], i1 = lloff[lv + 1];
            for (int idx = i0 + threadIdx.x; idx < i1; idx += blockDim.x) {
                const int t = llist[idx];
                solve_entry(t, code[t]);
            }
            __syncthreads();
        }
    }

    // 4. write back: all table lookups first, then all stores
    {
        int64_t go[kPerLane];
        uint64_t cv[kPerLane];
#pragma unroll
        for (int i = 0; i < kPerLane; ++i) {
            const int t = threadIdx.x + i * kThreads;
            go[i] = t < sd.S ? goff[t] : 0;
            cv[i] = (t < sd.S && ts.ragged) ? code[t] : 0;
        }
#pragma unroll
        for (int i = 0; i < kPerLane; ++i) {
            const int t = threadIdx.x + i * kThreads;
            if (t < sd.S && (!ts.ragged || entry_ok<MC>(cv[i], sd, ts)))
                X[ts.base + go[i]] = from_d2<V>(tile[t]);
        }
    }
}

template <typename V, bool ADJ>
hipError_t run_sweep(const sylt_plan_s &p, V *X, hipStream_t s)
{
    const SweepPlan &sp = p.sweep;
    decltype(&sweep_tile_kernel<V, ADJ, 0>) ker;
    switch (sp.desc.M) {
        case 1: ker = sweep_tile_kernel<V, ADJ, 1>; break;
        case 2: ker = sweep_tile_kernel<V, ADJ, 2>; break;
        case 3: ker = sweep_tile_kernel<V, ADJ, 3>; break;
        case 4: ker = sweep_tile_kernel<V, ADJ, 4>; break;
        case 5: ker = sweep_tile_kernel<V, ADJ, 5>; break;
        case 6: ker = sweep_tile_kernel<V, ADJ, 6>; break;
        case 7: ker = sweep_tile_kernel<V, ADJ, 7>; break;
        case 8: ker = sweep_tile_kernel<V, ADJ, 8>; break;
        default: ker = sweep_tile_kernel<V, ADJ, 0>; break;
    }
    if (sp.lds_bytes > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)ker,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)sp.lds_bytes);
        if (e != hipSuccess) return e;
    }
    const int nlev = (int)sp.level_off.size() - 1;
    for (int step = 0; step < nlev; ++step) {
        const int lv = ADJ ? step : nlev - 1 - step;
        const int64_t b0 = sp.level_off[lv], b1 = sp.level_off[lv + 1];
        if (b1 <= b0) continue;
        hipLaunchKernelGGL(ker, dim3((unsigned)(b1 - b0)), dim3(kThreads), sp.lds_bytes, s, X,
                           p.dT, sp.desc, sp.d_tiles + b0, sp.d_goff, sp.d_code, sp.d_llist,
                           sp.d_lloff, sp.d_lanetab);
    }
    return hipGetLastError();
}

}  // namespace

int sweep_max_partial_block() { return kBmax; }

hipError_t launch_sweep(const sylt_plan_s &p, int op, int precision, void *X, hipStream_t s)
{
    if (precision == SYLT_FP64) {
        return op == SYLT_OP_N ? run_sweep<double2, false>(p, static_cast<double2 *>(X), s)
                               : run_sweep<double2, true>(p, static_cast<double2 *>(X), s);
    }
    return op == SYLT_OP_N ? run_sweep<float2, false>(p, static_cast<float2 *>(X), s)
                           : run_sweep<float2, true>(p, static_cast<float2 *>(X), s);
}

}  // namespace sylt
