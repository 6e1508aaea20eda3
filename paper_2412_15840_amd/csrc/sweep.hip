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

#include <algorithm>
#include <type_traits>

namespace sylt {
namespace {

constexpr int kThreads = kSweepThreads;
constexpr int kBmax = 8;   // largest block of a partially tiled mode
constexpr int kPen = kSweepPencilMax;  // pencil entries held in registers
constexpr int kChunk0 = 4;    // mode-0 coefficients loaded together
static_assert(kPen % kChunk0 == 0, "pencil length must be whole chunks");
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

// f(std::integral_constant<int, I>{}) for I = B, B + 1, ..., E - 1
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

struct DiagModes {
    int d[kMaxModes];
    int64_t moff[kMaxModes];
    int nsing;
    int64_t singoff[kMaxModes];
};

struct TileState {
    int o[kMaxModes];
    int e[kMaxModes];
    int64_t base;
    int ragged;
    int shape;  // modes 1..M-1 whose block is short in this tile (bit j-1)
    int nll;    // local levels of this tile: 1 + sum_j (e_j - 1)
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

// Pull of one mode for a short k range (at most NP2 terms): every lane takes
// two cross-section positions per round, c and c + blockDim.x, so a round
// keeps as many loads in flight as a full round of the one-position form and
// the mode needs half as many rounds (each round costs about one memory
// latency).  A position outside a ragged tile borrows the other position's
// addresses and its result is dropped.
template <typename V, bool ADJ, int MC, int BJ, int NP2>
__device__ __forceinline__ void pull_mode_pairs(const V *__restrict__ X,
                                                const double2 *__restrict__ Tj,
                                                const int *__restrict__ cj,
                                                const int64_t *__restrict__ goff,
                                                const uint64_t *__restrict__ code,
                                                const SweepDesc &sd, const TileState &ts,
                                                double2 *tile, int o, int e, int d, int k0, int k1,
                                                int lsj, int64_t sj, int cs)
{
    const int step = blockDim.x;
    for (int c = threadIdx.x; c < cs; c += 2 * step) {
        const int ta = cj[c];
        const bool inb = c + step < cs;
        const int tb = inb ? cj[c + step] : ta;
        const bool va = !ts.ragged || entry_ok<MC>(code[ta], sd, ts);
        const bool vb = inb && (!ts.ragged || entry_ok<MC>(code[tb], sd, ts));
        if (!va && !vb) continue;
        const int64_t ga = goff[ta], gb = goff[tb];
        const V *sa = X + ts.base + (va ? ga : gb) - (int64_t)o * sj;
        const V *sb = X + ts.base + (vb ? gb : ga) - (int64_t)o * sj;
        double2 acca[BJ], accb[BJ];
#pragma unroll
        for (int r = 0; r < BJ; ++r) acca[r] = accb[r] = make_double2(0.0, 0.0);
        using L = std::conditional_t<std::is_same<V, double2>::value, double2, V>;
        L ya[NP2], yb[NP2];
#pragma unroll
        for (int u = 0; u < NP2; ++u) {
            if constexpr (std::is_same<V, double2>::value) {
                ya[u] = k0 + u < k1 ? sa[(int64_t)(k0 + u) * sj] : make_double2(0.0, 0.0);
                yb[u] = k0 + u < k1 ? sb[(int64_t)(k0 + u) * sj] : make_double2(0.0, 0.0);
            } else if (k0 + u < k1) {
                ya[u] = sa[(int64_t)(k0 + u) * sj];
                yb[u] = sb[(int64_t)(k0 + u) * sj];
            }
        }
#pragma unroll
        for (int u = 0; u < NP2; ++u) {
            const int k = k0 + u;
            if (k >= k1) break;  // uniform
            const double2 ua = to_d2<V>(ya[u]), ub = to_d2<V>(yb[u]);
#pragma unroll
            for (int r = 0; r < BJ; ++r) {
                if (r < e) {
                    if (ADJ) {
                        const double2 t = Tj[k + (int64_t)d * (o + r)];
                        acca[r] = cmac_conj(acca[r], t, ua);
                        accb[r] = cmac_conj(accb[r], t, ub);
                    } else {
                        const double2 t = Tj[(o + r) + (int64_t)d * k];
                        acca[r] = cmac(acca[r], t, ua);
                        accb[r] = cmac(accb[r], t, ub);
                    }
                }
            }
        }
        if constexpr (!std::is_same<V, double2>::value) __builtin_amdgcn_s_waitcnt(0x0f70);
        if (va) {
#pragma unroll
            for (int r = 0; r < BJ; ++r)
                if (r < e) tile[ta + r * lsj] = csub(tile[ta + r * lsj], acca[r]);
        }
        if (vb) {
#pragma unroll
            for (int r = 0; r < BJ; ++r)
                if (r < e) tile[tb + r * lsj] = csub(tile[tb + r * lsj], accb[r]);
        }
    }
}

// Pull of one mode: for every cross-section position of the tile (one per
// lane and round), the rows of the block receive
//   sum over k outside the block of T_j[row, k] * Y[..., k, ...]
// (k above the block for the upper sweep, below it for the adjoint).  BJ is
// the block size, NP the loads a lane keeps in flight; PAIRS lets a short k
// range take the two-position form.
template <typename V, bool ADJ, int MC, int BJ, int NP, bool PAIRS>
__device__ __forceinline__ void pull_mode(const V *__restrict__ X, const double2 *__restrict__ Tj,
                                          const int *__restrict__ cj,
                                          const int64_t *__restrict__ goff,
                                          const uint64_t *__restrict__ code, const SweepDesc &sd,
                                          const TileState &ts, double2 *tile, int o, int e, int d,
                                          int k0, int k1, int lsj, int64_t sj, int cs)
{
    if constexpr (PAIRS && BJ <= 3) {
        if constexpr (std::is_same<V, double2>::value) {
            if (2 * (k1 - k0) <= NP) {  // uniform
                pull_mode_pairs<V, ADJ, MC, BJ, NP / 2>(X, Tj, cj, goff, code, sd, ts, tile, o, e,
                                                        d, k0, k1, lsj, sj, cs);
                return;
            }
        } else {
            if (2 * (k1 - k0) <= NP) {  // uniform
                pull_mode_pairs<V, ADJ, MC, BJ, NP / 2>(X, Tj, cj, goff, code, sd, ts, tile, o, e,
                                                        d, k0, k1, lsj, sj, cs);
                return;
            }
            if (k1 - k0 <= NP) {  // uniform
                pull_mode_pairs<V, ADJ, MC, BJ, NP>(X, Tj, cj, goff, code, sd, ts, tile, o, e, d,
                                                    k0, k1, lsj, sj, cs);
                return;
            }
        }
    }
    for (int c = threadIdx.x; c < cs; c += blockDim.x) {
        // cross-section position c -> local entry t0 (loc_j = 0), from the
        // plan's table; its global offset and, in a ragged tile, whether it
        // lies inside the tile, from the per-entry tables
        const int t0 = cj[c];
        if (ts.ragged && !entry_ok<MC>(code[t0], sd, ts)) continue;
        const V *src = X + ts.base + goff[t0] - (int64_t)o * sj;
        double2 acc[BJ];
#pragma unroll
        for (int r = 0; r < BJ; ++r) acc[r] = make_double2(0.0, 0.0);
        for (int kb = k0; kb < k1; kb += NP) {
            // the loads of a chunk are issued together and waited for at the
            // first use.  Stored as complex64, the entries stay in that type
            // until they are used: a conversion next to its load would wait
            // for that load alone, one memory latency per entry.
            using L = std::conditional_t<std::is_same<V, double2>::value, double2, V>;
            L y[NP];
#pragma unroll
            for (int u = 0; u < NP; ++u) {
                if constexpr (std::is_same<V, double2>::value)
                    y[u] = kb + u < k1 ? src[(int64_t)(kb + u) * sj] : make_double2(0.0, 0.0);
                else if (kb + u < k1)
                    y[u] = src[(int64_t)(kb + u) * sj];
            }
#pragma unroll
            for (int u = 0; u < NP; ++u) {
                const int k = kb + u;
                if (k >= k1) break;  // uniform
                const double2 yu = to_d2<V>(y[u]);
#pragma unroll
                for (int r = 0; r < BJ; ++r) {
                    if (r < e) {
                        if (ADJ)
                            acc[r] = cmac_conj(acc[r], Tj[k + (int64_t)d * (o + r)], yu);
                        else
                            acc[r] = cmac(acc[r], Tj[(o + r) + (int64_t)d * k], yu);
                    }
                }
            }
            // complex64: every load of the chunk has been used.  Without this
            // wait (vmcnt(0), the other counters left alone) the compiler
            // waits before reusing a load's register in the next chunk.
            if constexpr (!std::is_same<V, double2>::value) __builtin_amdgcn_s_waitcnt(0x0f70);
        }
#pragma unroll
        for (int r = 0; r < BJ; ++r)
            if (r < e) tile[t0 + r * lsj] = csub(tile[t0 + r * lsj], acc[r]);
    }
}

template <typename V, bool ADJ, int MC, bool PEN>
__global__ void __launch_bounds__(kThreads) sweep_tile_kernel(
    V *__restrict__ X, const double2 *__restrict__ Tbuf, const double2 *__restrict__ Ttbuf,
    const SweepDesc *__restrict__ sdp,
    const int *__restrict__ tiles, const int64_t *__restrict__ goff,
    const uint64_t *__restrict__ code, const int *__restrict__ llist,
    const int *__restrict__ lloff, const int *__restrict__ lanetab, const int *__restrict__ cst)
{
    // the descriptor is read from device memory: a by-value kernel argument
    // that lambdas capture would be copied to scratch
    const SweepDesc &sd = *sdp;
    const int M = MC > 0 ? MC : sd.M;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double2 *tile = reinterpret_cast<double2 *>(smem_raw);
    double2 *tdiag = tile + sd.S;
    __shared__ TileState ts;

    if (threadIdx.x == 0) {
        int rem = tiles[tile_slot(blockIdx.x, gridDim.x)];
        int64_t base = 0;
        int ragged = 0, shape = 0, nll = 1;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const int P = rem % sd.nb[j];
            rem /= sd.nb[j];
            ts.o[j] = P * sd.b[j];
            ts.e[j] = min(sd.b[j], sd.d[j] - ts.o[j]);
            ragged |= ts.e[j] < sd.b[j];
            if (j > 0) shape |= (ts.e[j] < sd.b[j]) << (j - 1);
            nll += ts.e[j] - 1;
            base += (int64_t)ts.o[j] * sd.s[j];
        }
        ts.shape = shape;
        ts.nll = nll;
        double2 sh = make_double2(0.0, 0.0);
        for (int i = 0; i < sd.nsing; ++i) sh = cadd(sh, Tbuf[sd.singoff[i]]);
        ts.base = base;
        ts.ragged = ragged;
        ts.shift = ADJ ? cconj(sh) : sh;
    }
    __syncthreads();

    // 1. diagonal blocks of T_j (and a zero entry after them) and the tile of C
    if (threadIdx.x == 0) tdiag[sd.tdiag] = make_double2(0.0, 0.0);
    for (int j = 0; j < M; ++j) {
        const int b = sd.b[j], e = ts.e[j], o = ts.o[j], d = sd.d[j];
        const double2 *Tj = Tbuf + sd.moff[j];
        for (int idx = threadIdx.x; idx < b * b; idx += blockDim.x) {
            const int r = idx % b, c = idx / b;
            tdiag[sd.tdoff[j] + idx] =
                (r < e && c < e) ? Tj[(o + r) + (int64_t)d * (o + c)] : make_double2(0.0, 0.0);
        }
    }
    // this lane's pencil (pencil form of the local solve)
    const int pen_item = PEN ? lanetab[ts.shape * kThreads + threadIdx.x] : -1;
    // this lane's local-solve work, all levels at once (one memory latency)
    int pk[kMaxRounds];
    if (!PEN && sd.packed) {
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
        const int *cj = cst + sd.csoff[j];
        // the block size is a compile-time constant of the pull loop, so the
        // row accumulators take only the registers the block needs and the
        // rest go to loads in flight
        switch (b) {
#define SYLT_PULL(BJ, NP)                                                                         \
    case BJ:                                                                                      \
        pull_mode<V, ADJ, MC, BJ, NP, PEN>(X, Tj, cj, goff, code, sd, ts, tile, o, e, d, k0, k1, lsj, sj, \
                                      cs);                                                        \
        break;
            SYLT_PULL(1, 16) SYLT_PULL(2, 16) SYLT_PULL(3, 16) SYLT_PULL(4, 12)
            SYLT_PULL(5, 12) SYLT_PULL(6, 8) SYLT_PULL(7, 8) SYLT_PULL(8, 8)
#undef SYLT_PULL
            default: break;
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
                    num = cmsub_conj(num, Td[(loc - q) + b * loc], tile[t - q * lsj]);
            } else {
                const int qmax = ts.e[j] - 1 - loc;
                for (int q = 1; q <= qmax; ++q)
                    num = cmsub(num, Td[loc + b * (loc + q)], tile[t + q * lsj]);
            }
        }
        tile[t] = cdiv(num, den);
    };
    if (PEN) {
        // Pencil form: lane = one pencil along mode 0 (the tile's entries that
        // differ only in loc_0), kept in registers as it is solved; a wave holds
        // pencils of one index sum g over the other modes, so at local level L
        // all its lanes solve entry loc_0 = L - g: the mode-0 terms use
        // wave-uniform coefficients T_0[loc_0, k] and the lane's own registers,
        // only the other modes read neighbours from LDS.
        const int lead = __builtin_amdgcn_readfirstlane(pen_item);
        const bool has = pen_item >= 0;
        const int t0 = has ? (pen_item & kPackMask) : 0;
        const uint64_t c = has ? (uint64_t)(pen_item >> kPackShift) : 0;
        const uint64_t cl = lead >= 0 ? (uint64_t)(lead >> kPackShift) : 0;
        constexpr int kD = 2 * (MC > 1 ? MC - 1 : 1);  // first two neighbours per other mode
        int dep[kD];  // per neighbour: coefficient slot << 16 | entry offset (zero slot if none)
        int g = 0;
        bool act = has;
        double2 sigma = ts.shift;  // the diagonal terms of the other modes
#pragma unroll
        for (int j = 1; j < M; ++j) {
            const int w = sd.bitw[j];
            const uint64_t m = (1ull << w) - 1ull;
            g += w ? (int)((cl >> sd.bitoff[j]) & m) : 0;
            const int loc = w ? (int)((c >> sd.bitoff[j]) & m) : 0;
            act = act && loc < ts.e[j];
        }
#pragma unroll
        for (int j = 1; j < M; ++j) {
            const int w = sd.bitw[j];
            const int loc = w ? (int)((c >> sd.bitoff[j]) & ((1ull << w) - 1ull)) : 0;
            const int b = sd.b[j], td = sd.tdoff[j];
            const double2 lam = tdiag[td + loc + b * loc];
            sigma = cadd(sigma, ADJ ? cconj(lam) : lam);
            const int nq = ADJ ? loc : ts.e[j] - 1 - loc;
#pragma unroll
            for (int q = 1; q <= 2; ++q) {
                const bool ok = act && nq >= q;
                const int slot = ok ? td + (ADJ ? (loc - q) + b * loc : loc + b * (loc + q)) : sd.tdiag;
                dep[2 * (j - 1) + q - 1] = (slot << 16) | (ok ? q * sd.ls[j] : 0);
            }
        }
        g = __builtin_amdgcn_readfirstlane(g);
        const int e0 = __builtin_amdgcn_readfirstlane(ts.e[0]);
        const int64_t r0 = __builtin_amdgcn_readfirstlane(ts.o[0]);
        const int64_t d0 = sd.d[0];
        // column K of T_0 (row K, i.e. column K of T_0^T, for the adjoint):
        // the coefficients with which entry K enters the entries solved after
        // it are contiguous there
        const double2 *Tcol = (ADJ ? Ttbuf : Tbuf) + sd.moff[0] + r0;
        // y[K]: minus the mode-0 sum of entry K over the entries already
        // solved, added to as each of them is solved (right-looking), so an
        // entry's own solve does not wait on a chain of multiply-adds
        double2 y[kPen];
#pragma unroll
        for (int i = 0; i < kPen; ++i) y[i] = make_double2(0.0, 0.0);
        // the entry at mode-0 position K, with K a compile-time constant: the
        // pencil registers are then addressed statically
        auto entry = [&](auto kc) __attribute__((always_inline)) {
            constexpr int K = decltype(kc)::value;
            const int t = t0 + K;
            const double2 *cf = Tcol + d0 * (r0 + K);
            double2 num = cadd(tile[t], y[K]);
            double2 yk = make_double2(0.0, 0.0);
            if (act) {
                const double2 lam0 = cf[K];
                const double2 den = cadd(sigma, ADJ ? cconj(lam0) : lam0);
#pragma unroll
                for (int i = 0; i < kD; ++i) {
                    if (i >= 2 * (M - 1)) break;
                    const double2 a = tdiag[dep[i] >> 16];
                    const double2 yn = tile[ADJ ? t - (dep[i] & 0xffff) : t + (dep[i] & 0xffff)];
                    num = ADJ ? cmsub_conj(num, a, yn) : cmsub(num, a, yn);
                }
                if (sd.pen_long) {  // neighbours beyond the second (blocks longer than 3)
#pragma unroll 1
                    for (int j = 1; j < M; ++j) {
                        const int w = sd.bitw[j];
                        const int loc = w ? (int)((c >> sd.bitoff[j]) & ((1ull << w) - 1ull)) : 0;
                        const int b = sd.b[j], lsj = sd.ls[j];
                        const double2 *Td = tdiag + sd.tdoff[j];
                        const int nq = ADJ ? loc : ts.e[j] - 1 - loc;
                        for (int q = 3; q <= nq; ++q)
                            num = ADJ ? cmsub_conj(num, Td[(loc - q) + b * loc], tile[t - q * lsj])
                                      : cmsub(num, Td[loc + b * (loc + q)], tile[t + q * lsj]);
                    }
                }
                yk = cdiv_scaled(num, den);
                tile[t] = yk;
            }
            // pass y_K on to the entries still to be solved (an inactive lane
            // passes zero)
            if (ADJ) {
                // entries past the block end are never solved; the coefficient
                // index stays in the block
#pragma unroll
                for (int kb = (K + 1) & ~(kChunk0 - 1); kb < kPen; kb += kChunk0) {
                    if (kb >= e0) break;  // uniform
#pragma unroll
                    for (int kk = kb; kk < kb + kChunk0; ++kk)
                        if (kk > K) y[kk] = cmsub_conj(y[kk], cf[min(kk, e0 - 1)], yk);
                }
            } else {
#pragma unroll
                for (int kk = 0; kk < K; ++kk) y[kk] = cmsub(y[kk], cf[kk], yk);
            }
        };
        // A wave is active at the e0 local levels g .. g + e0 - 1, one entry
        // each; before and after them it only takes part in the barriers, so
        // every wave passes the same nll barriers.
        const int nll = ts.nll;
        const int before = lead < 0 ? nll : (ADJ ? g : nll - g - e0);
        for (int i = 0; i < before; ++i) __syncthreads();
        if (lead >= 0) {
            if (ADJ) {
                static_for<0, kPen>([&](auto kc) __attribute__((always_inline)) {
                    if (decltype(kc)::value < e0) {
                        entry(kc);
                        __syncthreads();
                    }
                });
            } else {
                static_for<0, kPen>([&](auto kc) __attribute__((always_inline)) {
                    constexpr int K = kPen - 1 - decltype(kc)::value;
                    if (K < e0) {
                        entry(std::integral_constant<int, K>{});
                        __syncthreads();
                    }
                });
            }
            const int after = ADJ ? nll - g - e0 : g;
            for (int i = 0; i < after; ++i) __syncthreads();
        }
    } else if (sd.packed) {
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

template <typename V, bool ADJ, bool PEN>
hipError_t run_sweep_as(const sylt_plan_s &p, V *X, hipStream_t s)
{
    const SweepPlan &sp = p.sweep;
    decltype(&sweep_tile_kernel<V, ADJ, 0, PEN>) ker;
    switch (sp.desc.M) {
        case 1: ker = sweep_tile_kernel<V, ADJ, 1, PEN>; break;
        case 2: ker = sweep_tile_kernel<V, ADJ, 2, PEN>; break;
        case 3: ker = sweep_tile_kernel<V, ADJ, 3, PEN>; break;
        case 4: ker = sweep_tile_kernel<V, ADJ, 4, PEN>; break;
        case 5: ker = sweep_tile_kernel<V, ADJ, 5, PEN>; break;
        case 6: ker = sweep_tile_kernel<V, ADJ, 6, PEN>; break;
        case 7: ker = sweep_tile_kernel<V, ADJ, 7, PEN>; break;
        case 8: ker = sweep_tile_kernel<V, ADJ, 8, PEN>; break;
        default: ker = sweep_tile_kernel<V, ADJ, 0, PEN>; break;
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
                           p.dT, p.dTt, sp.d_desc, sp.d_tiles + b0, sp.d_goff, sp.d_code, sp.d_llist,
                           sp.d_lloff, sp.d_lanetab, sp.d_cst);
    }
    return hipGetLastError();
}

template <typename V, bool ADJ>
hipError_t run_sweep(const sylt_plan_s &p, V *X, hipStream_t s)
{
    if (p.sweep.desc.penc && p.sweep.desc.M > kSweepPencilModes) return hipErrorInvalidValue;
    return p.sweep.desc.penc ? run_sweep_as<V, ADJ, true>(p, X, s) : run_sweep_as<V, ADJ, false>(p, X, s);
}

// Remark 1 (eq. e:yi1i2iNdiag): with every T_j diagonal the sweep is
// y_i = c_i / (lambda_{1,i_1} + ... + lambda_{N,i_N}), one streaming pass.
template <typename V, bool ADJ>
__global__ void __launch_bounds__(256) diag_sweep_kernel(V *__restrict__ X,
                                                         const double2 *__restrict__ slo,
                                                         const double2 *__restrict__ shi, int64_t lo,
                                                         int64_t ntot)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ntot;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t q, r;
        if (ntot <= 0xffffffffll) {  // 32-bit quotient when the index fits
            q = (uint32_t)i / (uint32_t)lo;
            r = (uint32_t)i - (uint32_t)q * (uint32_t)lo;
        } else {
            q = i / lo;
            r = i - q * lo;
        }
        const double2 den = cadd(slo[r], shi[q]);
        X[i] = from_d2<V>(cdiv_scaled(to_d2<V>(X[i]), ADJ ? cconj(den) : den));
    }
}

// table[r] = base + sum over modes [j0, j1) of lambda_{j, i_j(r)}, r < count
__global__ void diag_table_kernel(double2 *table, int64_t count, const double2 *__restrict__ T,
                                  DiagModes dm, int j0, int j1, int with_singletons)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < count;
         r += (int64_t)gridDim.x * blockDim.x) {
        double2 acc = make_double2(0.0, 0.0);
        if (with_singletons)
            for (int i = 0; i < dm.nsing; ++i) acc = cadd(acc, T[dm.singoff[i]]);
        int64_t rem = r;
        for (int j = j0; j < j1; ++j) {
            const int64_t i = rem % dm.d[j];
            rem /= dm.d[j];
            acc = cadd(acc, T[dm.moff[j] + i * (dm.d[j] + 1)]);
        }
        table[r] = acc;
    }
}

template <typename V, bool ADJ>
hipError_t run_diag_sweep(const sylt_plan_s &p, V *X, hipStream_t s)
{
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((p.ntot + 255) / 256, 256 * 32));
    hipLaunchKernelGGL((diag_sweep_kernel<V, ADJ>), dim3((unsigned)blocks), dim3(256), 0, s, X,
                       p.dslo, p.dshi, p.dlo, p.ntot);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_diag_tables(const sylt_plan_s &p, hipStream_t s)
{
    DiagModes dm{};
    for (int j = 0; j < p.M; ++j) {
        dm.d[j] = p.cdim[j];
        dm.moff[j] = p.moff[p.cmode[j]];
    }
    for (int k = 0; k < p.N; ++k)
        if (p.n[k] == 1) dm.singoff[dm.nsing++] = p.moff[k];
    const int split = p.dsplit;  // compressed modes [0, split) make up the low table
    auto grid = [](int64_t n) {
        return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
    };
    hipLaunchKernelGGL(diag_table_kernel, dim3(grid(p.dlo)), dim3(256), 0, s, p.dslo, p.dlo, p.dT, dm,
                       0, split, 1);
    hipLaunchKernelGGL(diag_table_kernel, dim3(grid(p.dhi)), dim3(256), 0, s, p.dshi, p.dhi, p.dT, dm,
                       split, p.M, 0);
    return hipGetLastError();
}

int sweep_max_partial_block() { return kBmax; }

hipError_t launch_sweep(const sylt_plan_s &p, int op, int precision, void *X, hipStream_t s)
{
    if (p.diagT) {
        if (precision == SYLT_FP64)
            return op == SYLT_OP_N ? run_diag_sweep<double2, false>(p, static_cast<double2 *>(X), s)
                                   : run_diag_sweep<double2, true>(p, static_cast<double2 *>(X), s);
        return op == SYLT_OP_N ? run_diag_sweep<float2, false>(p, static_cast<float2 *>(X), s)
                               : run_diag_sweep<float2, true>(p, static_cast<float2 *>(X), s);
    }
    if (precision == SYLT_FP64) {
        return op == SYLT_OP_N ? run_sweep<double2, false>(p, static_cast<double2 *>(X), s)
                               : run_sweep<double2, true>(p, static_cast<double2 *>(X), s);
    }
    return op == SYLT_OP_N ? run_sweep<float2, false>(p, static_cast<float2 *>(X), s)
                           : run_sweep<float2, true>(p, static_cast<float2 *>(X), s);
}

}  // namespace sylt
