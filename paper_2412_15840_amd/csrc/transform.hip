// Mode-product passes on gfx950.
//
// A chain of mode products (eq. e:CUNU2U1B with U_k^*, eq. e:XUNU2U1Y with
// U_k) applies one small dense matrix along every mode.  Products on distinct
// modes commute, so a run of consecutive modes [a, b) is fused into one HBM
// pass: the tensor is viewed as (Lin, G, Rout) with G the product of the run's
// extents, and a workgroup loads an lb x G x rb tile (lb consecutive entries of
// the low modes -- a coalesced run -- times the full extents of the run) into
// LDS, applies the run's products in LDS/registers and writes the tile back in
// place.  Each lane owns whole fibres: it streams the n inputs of a fibre from
// LDS once and accumulates all n outputs in registers, with the matrix entries
// wave-uniform (scalar loads), i.e. n complex multiply-adds per LDS read.
//
// The residual pass (R = B - sum_k A_k x_k X, the operator of eq.
// e:sylvesterND) uses the same tiling but sums the products of the run into an
// LDS accumulator instead of chaining them.
#include "sylt_internal.h"

namespace sylt {
namespace {

constexpr int kThreads = 256;

template <typename V> __device__ __forceinline__ V vzero();
template <> __device__ __forceinline__ double2 vzero<double2>() { return make_double2(0.0, 0.0); }
template <> __device__ __forceinline__ float2 vzero<float2>() { return make_float2(0.f, 0.f); }

template <typename V> __device__ __forceinline__ V vadd(V a, V b)
{
    a.x += b.x;
    a.y += b.y;
    return a;
}

// y = M x along one fibre of length NN held in LDS at base + m*stride; the
// result overwrites the fibre (ACC == false) or is added into acc (ACC == true).
// M is column-major NN x NN, read with wave-uniform addresses.
template <typename V, int NN, bool ACC>
__device__ __forceinline__ void fibre_fixed(V *src, V *acc, int base, int stride,
                                            const V *__restrict__ M)
{
    V y[NN];
#pragma unroll
    for (int i = 0; i < NN; ++i) y[i] = vzero<V>();
#pragma unroll
    for (int m = 0; m < NN; ++m) {
        const V x = src[base + m * stride];
#pragma unroll
        for (int i = 0; i < NN; ++i) y[i] = cmac(y[i], M[i + NN * m], x);
    }
#pragma unroll
    for (int i = 0; i < NN; ++i) {
        if (ACC)
            acc[base + i * stride] = vadd(acc[base + i * stride], y[i]);
        else
            src[base + i * stride] = y[i];
    }
}

// any extent: the outputs ic .. ic+7 of one fibre, written to a separate
// buffer (so the chunks of a fibre are independent work items)
constexpr int kGenericChunk = 8;
template <typename V, bool ACC>
__device__ __forceinline__ void fibre_generic(const V *src, V *dst, int base, int stride, int n,
                                              const V *__restrict__ M, int ic)
{
    V y[kGenericChunk];
#pragma unroll
    for (int i = 0; i < kGenericChunk; ++i) y[i] = vzero<V>();
    for (int m = 0; m < n; ++m) {
        const V x = src[base + m * stride];
#pragma unroll
        for (int i = 0; i < kGenericChunk; ++i)
            if (ic + i < n) y[i] = cmac(y[i], M[ic + i + n * m], x);
    }
#pragma unroll
    for (int i = 0; i < kGenericChunk; ++i) {
        if (ic + i < n) {
            if (ACC)
                dst[base + (ic + i) * stride] = vadd(dst[base + (ic + i) * stride], y[i]);
            else
                dst[base + (ic + i) * stride] = y[i];
        }
    }
}

// Dispatch on the runtime extent for groups of mixed sizes (all <= 24).
template <typename V, bool ACC>
__device__ __forceinline__ void fibre_switch(V *src, V *acc, int base, int stride, int n,
                                             const V *__restrict__ M)
{
    switch (n) {
#define SYLT_CASE(K) \
    case K: fibre_fixed<V, K, ACC>(src, acc, base, stride, M); break;
        SYLT_CASE(2) SYLT_CASE(3) SYLT_CASE(4) SYLT_CASE(5) SYLT_CASE(6) SYLT_CASE(7)
        SYLT_CASE(8) SYLT_CASE(9) SYLT_CASE(10) SYLT_CASE(11) SYLT_CASE(12) SYLT_CASE(13)
        SYLT_CASE(14) SYLT_CASE(15) SYLT_CASE(16) SYLT_CASE(17) SYLT_CASE(18) SYLT_CASE(19)
        SYLT_CASE(20) SYLT_CASE(21) SYLT_CASE(22) SYLT_CASE(23) SYLT_CASE(24)
#undef SYLT_CASE
        default: break;
    }
}

struct TileCoord {
    int64_t l0, r0;
    int lbe, rbe;
};

__device__ __forceinline__ TileCoord tile_coord(const PassDesc &pa)
{
    TileCoord t;
    const int64_t tid = blockIdx.x;
    const int64_t tl = tid % pa.ntl, tr = tid / pa.ntl;
    t.l0 = tl * pa.lb;
    t.r0 = tr * pa.rb;
    t.lbe = (int)min((int64_t)pa.lb, pa.Lin - t.l0);
    t.rbe = (int)min((int64_t)pa.rb, pa.Rout - t.r0);
    return t;
}

// LDS tile layout: index l + lb * (g + G * r) for l < lb, g < G, r < rb.
template <typename VG, typename VL>
__device__ __forceinline__ void load_tile(VL *tile, const VG *__restrict__ X, const PassDesc &pa,
                                          const TileCoord &tc)
{
    const int lbG = pa.lb * (int)pa.G;
    for (int r = 0; r < tc.rbe; ++r) {
        const int64_t gbase = tc.l0 + pa.Lin * pa.G * (tc.r0 + r);
        VL *tb = tile + (int64_t)lbG * r;
        for (int e = threadIdx.x; e < lbG; e += blockDim.x) {
            const int l = e & (pa.lb - 1);
            const int g = e >> pa.lbshift;
            if (l < tc.lbe) {
                const VG v = X[gbase + l + pa.Lin * g];
                tb[e].x = v.x;
                tb[e].y = v.y;
            }
        }
    }
}

template <typename V>
__device__ __forceinline__ void store_tile(V *__restrict__ X, const V *tile, const PassDesc &pa,
                                           const TileCoord &tc)
{
    const int lbG = pa.lb * (int)pa.G;
    for (int r = 0; r < tc.rbe; ++r) {
        const int64_t gbase = tc.l0 + pa.Lin * pa.G * (tc.r0 + r);
        const V *tb = tile + (int64_t)lbG * r;
        for (int e = threadIdx.x; e < lbG; e += blockDim.x) {
            const int l = e & (pa.lb - 1);
            const int g = e >> pa.lbshift;
            if (l < tc.lbe) X[gbase + l + pa.Lin * g] = tb[e];
        }
    }
}

// Fibre f of mode q -> LDS base index (or -1 for a lane outside the tile).
__device__ __forceinline__ int fibre_base(const PassDesc &pa, const TileCoord &tc, int q, int n,
                                          int f)
{
    const int l = f & (pa.lb - 1);
    int rest = f >> pa.lbshift;
    const int gs = pa.gs[q];
    const int ghi_count = (int)(pa.G / ((int64_t)gs * n));
    const int glo = rest % gs;
    rest /= gs;
    const int ghi = rest % ghi_count;
    const int r = rest / ghi_count;
    if (l >= tc.lbe) return -1;
    return l + pa.lb * (glo + gs * n * ghi + (int)pa.G * r);
}

// Table of fibre_base over a full tile, for every mode of the pass: entry
// q * (nfull) + f, nfull = lb * (G / n) * rb fibres per mode.  Built once per
// workgroup so the per-group lookup is one LDS read instead of the divisions
// of fibre_base; a ragged tile masks fibres with l >= lbe or beyond its rows.
__device__ __forceinline__ void build_fibre_table(int *fbt, const PassDesc &pa, int n)
{
    const int nfull = pa.lb * (int)(pa.G / n) * pa.rb;
    TileCoord full;
    full.l0 = full.r0 = 0;
    full.lbe = pa.lb;
    full.rbe = pa.rb;
    for (int idx = threadIdx.x; idx < pa.ng * nfull; idx += blockDim.x) {
        const int q = idx / nfull, f = idx - q * nfull;
        fbt[idx] = fibre_base(pa, full, q, n, f);
    }
}

// ------------------------------------------------------------ transform
// NN > 0: every mode of the group has extent NN.  NN == 0: mixed extents <= 24.
template <typename V, int NN>
__global__ void __launch_bounds__(kThreads) transform_pass_kernel(V *X, const V *Xs,
                                                                  const V *__restrict__ Mbuf,
                                                                  PassDesc pa)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V *tile = reinterpret_cast<V *>(smem_raw);
    const TileCoord tc = tile_coord(pa);
    load_tile<V, V>(tile, Xs, pa, tc);
    __syncthreads();
    for (int q = 0; q < pa.ng; ++q) {
        const int n = NN > 0 ? NN : pa.gd[q];
        const int nfib = pa.lb * (int)(pa.G / n) * tc.rbe;
        const int stride = pa.lb * pa.gs[q];
        const V *M = Mbuf + pa.moff[q];
        for (int f = threadIdx.x; f < nfib; f += blockDim.x) {
            const int base = fibre_base(pa, tc, q, n, f);
            if (base < 0) continue;
            if constexpr (NN > 0)
                fibre_fixed<V, NN, false>(tile, tile, base, stride, M);
            else
                fibre_switch<V, false>(tile, tile, base, stride, n, M);
        }
        __syncthreads();
    }
    store_tile<V>(X, tile, pa, tc);
}

// ------------------------------------------------ pipelined uniform pass
// Persistent workgroups of 512 lanes walk the tiles; while the products of
// tile t run in LDS, the loads of tile t + grid are already in flight into
// registers.  Each fibre's NN outputs are split into P wave-uniform parts of
// NP rows, so every wave has work even when a tile holds few fibres; a round
// covers 512 / P whole fibres: all parts read their inputs, a barrier, then
// all write (the fibre is updated in place).
constexpr int kPipeThreads = 512;
constexpr int kPipeRegs = 16;  // tile entries per lane (tiles <= 8192 entries)

template <typename V, int NN, int NP, int PART>
__device__ __forceinline__ void fibre_part(const V *tile, int base, int stride,
                                           const V *__restrict__ M, V (&y)[NP])
{
    constexpr int I0 = PART * NP;
    constexpr int CNT = NN - I0 < NP ? (NN - I0 > 0 ? NN - I0 : 0) : NP;
#pragma unroll
    for (int i = 0; i < NP; ++i) y[i] = vzero<V>();
    // the column loop stays rolled: each iteration needs only its CNT matrix
    // entries in scalar registers, and the next input is already in flight
    V xn = tile[base];
#pragma unroll 1
    for (int m = 0; m < NN; ++m) {
        const V x = xn;
        if (m + 1 < NN) xn = tile[base + (m + 1) * stride];
        const V *Mm = M + I0 + NN * m;
#pragma unroll
        for (int i = 0; i < CNT; ++i) y[i] = cmac(y[i], Mm[i], x);
    }
}

template <typename V>
__device__ __forceinline__ int64_t elem_addr(const PassDesc &pa, const TileCoord &tc, int e,
                                             bool &valid)
{
    const int l = e & (pa.lb - 1);
    const int rest = e >> pa.lbshift;
    const int g = rest % (int)pa.G, r = rest / (int)pa.G;
    valid = l < tc.lbe && r < tc.rbe;
    return tc.l0 + l + pa.Lin * (g + pa.G * (tc.r0 + r));
}

__device__ __forceinline__ TileCoord tile_coord_of(const PassDesc &pa, int64_t t)
{
    TileCoord c;
    const int64_t tl = t % pa.ntl, tr = t / pa.ntl;
    c.l0 = tl * pa.lb;
    c.r0 = tr * pa.rb;
    c.lbe = (int)min((int64_t)pa.lb, pa.Lin - c.l0);
    c.rbe = (int)min((int64_t)pa.rb, pa.Rout - c.r0);
    return c;
}

// Tile walk of a persistent pass.  Workgroups are dealt to the XCDs
// round-robin (workgroup b runs on XCD b % 8), and tiles t, t + 1 share the
// cache lines at their common edge (runs of lb entries need not start on a
// line).  XCD x therefore owns the contiguous range [x T / 8, (x + 1) T / 8),
// which its workgroups walk together, so neighbouring tiles run at the same
// time behind the same L2.  Grids that are not a multiple of 8 walk with
// stride G.
constexpr int kXcds = 8;
struct TileWalk {
    int64_t t, step, end;
};
__device__ __forceinline__ TileWalk tile_walk(int64_t ntiles)
{
    const int b = blockIdx.x, G = gridDim.x;
    if (G % kXcds != 0) return TileWalk{b, G, ntiles};
    const int x = b % kXcds;
    const int64_t lo = ntiles * x / kXcds, hi = ntiles * (x + 1) / kXcds;
    return TileWalk{lo + b / kXcds, G / kXcds, hi};
}

template <typename V, int NN, int P>
__global__ void __launch_bounds__(kPipeThreads) transform_pipe_kernel(V *X, const V *Xs,
                                                                      const V *__restrict__ Mbuf,
                                                                      PassDesc pa)
{
    constexpr int FR = kPipeThreads / P;  // fibres per round (multiple of 64)
    constexpr int NP = (NN + P - 1) / P;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V *tile = reinterpret_cast<V *>(smem_raw);
    const int total = pa.lb * (int)pa.G * pa.rb;
    const int64_t ntiles = pa.ntl * pa.ntr;
    const int part = threadIdx.x / FR;  // wave-uniform
    const int fl = threadIdx.x % FR;

    using R = typename CTraits<V>::R;
    R pre_re[kPipeRegs], pre_im[kPipeRegs];
    const TileWalk walk = tile_walk(ntiles);
    int64_t t = walk.t;
    if (t >= walk.end) return;
    // this lane's tile entries e = lane + i*512 -> (l, g, r); their offsets
    // from the tile origin are the same for every tile of the pass
    int64_t off[kPipeRegs];
    int lr[kPipeRegs];  // l | r << 16, or -1 beyond the tile
#pragma unroll
    for (int i = 0; i < kPipeRegs; ++i) {
        const int e = threadIdx.x + i * kPipeThreads;
        const int l = e & (pa.lb - 1);
        const int rest = e >> pa.lbshift;
        const int g = rest % (int)pa.G, r = rest / (int)pa.G;
        off[i] = l + pa.Lin * (g + pa.G * r);
        lr[i] = e < total ? (l | (r << 16)) : -1;
    }
    auto load_regs = [&](const TileCoord &c) {
        const int64_t org = c.l0 + pa.Lin * pa.G * c.r0;
        const bool whole = c.lbe == pa.lb && c.rbe == pa.rb;
#pragma unroll
        for (int i = 0; i < kPipeRegs; ++i) {
            const bool ok = lr[i] >= 0 &&
                            (whole || ((lr[i] & 0xffff) < c.lbe && (lr[i] >> 16) < c.rbe));
            if (ok) {
                const V v = Xs[org + off[i]];
                pre_re[i] = v.x;
                pre_im[i] = v.y;
            }
        }
    };
    TileCoord tc = tile_coord_of(pa, t);
    load_regs(tc);
    while (true) {
        // registers -> LDS (the tile of this iteration)
#pragma unroll
        for (int i = 0; i < kPipeRegs; ++i) {
            const int e = threadIdx.x + i * kPipeThreads;
            if (e < total) {
                tile[e].x = pre_re[i];
                tile[e].y = pre_im[i];
            }
        }
        __syncthreads();
        const int64_t tn = t + walk.step;
        const TileCoord tcn = tile_coord_of(pa, tn < walk.end ? tn : t);
        if (tn < walk.end) load_regs(tcn);
        for (int q = 0; q < pa.ng; ++q) {
            const int nfib = pa.lb * (int)(pa.G / NN) * tc.rbe;
            const int stride = pa.lb * pa.gs[q];
            const V *M = Mbuf + pa.moff[q];
            for (int f0 = 0; f0 < nfib; f0 += FR) {
                const int f = f0 + fl;
                const int base = f < nfib ? fibre_base(pa, tc, q, NN, f) : -1;
                V y[NP];
                if (base >= 0) {
                    switch (part) {
#define SYLT_PART(K) \
    case K: if constexpr (K < P) fibre_part<V, NN, NP, K>(tile, base, stride, M, y); break;
                        SYLT_PART(0) SYLT_PART(1) SYLT_PART(2) SYLT_PART(3)
                        SYLT_PART(4) SYLT_PART(5) SYLT_PART(6) SYLT_PART(7)
#undef SYLT_PART
                        default: break;
                    }
                }
                __syncthreads();
                if (base >= 0) {
#pragma unroll
                    for (int i = 0; i < NP; ++i)
                        if (part * NP + i < NN) tile[base + (part * NP + i) * stride] = y[i];
                }
                __syncthreads();
            }
        }
        // LDS -> global
        {
            const int64_t org = tc.l0 + pa.Lin * pa.G * tc.r0;
            const bool whole = tc.lbe == pa.lb && tc.rbe == pa.rb;
#pragma unroll
            for (int i = 0; i < kPipeRegs; ++i) {
                const bool ok = lr[i] >= 0 &&
                                (whole || ((lr[i] & 0xffff) < tc.lbe && (lr[i] >> 16) < tc.rbe));
                if (ok) X[org + off[i]] = tile[threadIdx.x + i * kPipeThreads];
            }
        }
        if (tn >= walk.end) break;
        __syncthreads();
        t = tn;
        tc = tcn;
    }
}

// ------------------------------------------------------ MFMA pass
// The product of one mode is a dense complex GEMM Y = M X over the fibres of
// the tile.  With re/im interleaved along rows and columns it becomes a real
// GEMM with the 2n x 2n matrix R[2i+a][2m+b] = {Re M, -Im M; Im M, Re M}
// (a, b in {0, 1}), zero-padded to 16-row blocks and 4-column steps, run on
// the 16x16x4 matrix cores: R lives in A fragments, 16 fibres of a wave are
// the B operand (each lane reads one real component straight from LDS) and
// the 16x16 result blocks are written back in place.  Lane layouts of
// v_mfma_{f64,f32}_16x16x4: A[i][k] in lane i + 16k, B[k][j] in lane j + 16k,
// result D[i][j] in lane j + 16*(i/4) value i%4 (f32) and in lane j + 16*(i%4)
// value i/4 (f64).
typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));
template <typename R> struct MfmaT;
template <> struct MfmaT<double> {
    using acc = mf_d4;
    static __device__ __forceinline__ acc mma(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // row of the 16-row block held by value v of lane l
    static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
    // block row r -> output (within the block's 8) and part (0 re, 1 im),
    // ordered so that values 2c and 2c + 1 of a lane are one complex output
    static __device__ __forceinline__ int out_of_row(int r) { return (r & 3) + 4 * (r >> 3); }
    static __device__ __forceinline__ int part_of_row(int r) { return (r >> 2) & 1; }
};
template <> struct MfmaT<float> {
    using acc = mf_f4;
    static __device__ __forceinline__ acc mma(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
    static __device__ __forceinline__ int out_of_row(int r) { return r >> 1; }
    static __device__ __forceinline__ int part_of_row(int r) { return r & 1; }
};

// two waves per SIMD; each lane prefetches 16 entries of the next tile
constexpr int kMfmaThreads = 512;
constexpr int kMfmaRegs = 16;  // tile entries per lane (tiles <= 8192 entries)

template <typename V, int NN>
__global__ void __launch_bounds__(kMfmaThreads) transform_mfma_kernel(V *X, const V *Xs,
                                                                      const V *__restrict__ Mbuf,
                                                                      PassDesc pa)
{
    using R = typename CTraits<V>::R;
    using MT = MfmaT<R>;
    constexpr int RB = (NN + 7) / 8;        // 16-row blocks of the real matrix (8 outputs each)
    constexpr int KS = (2 * NN + 3) / 4;    // 4-column steps
    constexpr int WAVES = kMfmaThreads / 64;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V *tile = reinterpret_cast<V *>(smem_raw);
    const int total = pa.lb * (int)pa.G * pa.rb;
    const int64_t ntiles = pa.ntl * pa.ntr;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // A fragments of every mode of the pass, in fragment order, after the tile
    R *afr = reinterpret_cast<R *>(tile + total);
    for (int idx = threadIdx.x; idx < pa.ng * RB * KS * 64; idx += kMfmaThreads) {
        const int l = idx & 63;
        const int frag = idx >> 6;
        const int kk = frag % KS, rb = (frag / KS) % RB, q = frag / (KS * RB);
        const int r = l & 15, k = 4 * kk + (l >> 4);
        const int i = 8 * rb + MT::out_of_row(r), m = k >> 1;
        R v = 0;
        if (i < NN && m < NN) {
            const V c = Mbuf[pa.moff[q] + i + NN * m];
            const int a = MT::part_of_row(r), b = k & 1;
            v = a == b ? c.x : (a ? c.y : -c.y);
        }
        afr[idx] = v;
    }
    int *fbt = reinterpret_cast<int *>(afr + pa.ng * RB * KS * 64);
    build_fibre_table(fbt, pa, NN);
    const int nfull = pa.lb * (int)(pa.G / NN) * pa.rb;
    // one zero operand after the table: lanes outside the tile (or past the
    // matrix edge) read it, so the operand loads need no branches
    R *zslot = reinterpret_cast<R *>(fbt + ((pa.ng * nfull + 3) & ~3));
    if (threadIdx.x == 0) zslot[0] = R(0);
    const int zidx = (int)(zslot - reinterpret_cast<R *>(tile));

    R pre_re[kMfmaRegs], pre_im[kMfmaRegs];
    const TileWalk walk = tile_walk(ntiles);
    int64_t t = walk.t;
    if (t >= walk.end) return;
    // global address of tile entry e (rb == 1 needs no division)
    auto gaddr = [&](const TileCoord &c, int e, bool &ok) -> int64_t {
        const int l = e & (pa.lb - 1);
        const int rest = e >> pa.lbshift;
        int g = rest, r = 0;
        if (pa.rb > 1) {
            g = rest % (int)pa.G;
            r = rest / (int)pa.G;
        }
        ok = e < total && l < c.lbe && r < c.rbe;
        return c.l0 + l + pa.Lin * (g + pa.G * (c.r0 + r));
    };
    auto load_regs = [&](const TileCoord &c) {
#pragma unroll
        for (int i = 0; i < kMfmaRegs; ++i) {
            bool ok;
            const int64_t a = gaddr(c, threadIdx.x + i * kMfmaThreads, ok);
            if (ok) {
                const V v = Xs[a];
                pre_re[i] = v.x;
                pre_im[i] = v.y;
            }
        }
    };
    TileCoord tc = tile_coord_of(pa, t);
    load_regs(tc);
    // every path into the loop has the prefetch registers complete (here and
    // before the last mode), so the refill never waits on result stores
    __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
    while (true) {
        // this tile's entries (loaded during the previous tile) into LDS
#pragma unroll
        for (int i = 0; i < kMfmaRegs; ++i) {
            const int e = threadIdx.x + i * kMfmaThreads;
            if (e < total) {
                tile[e].x = pre_re[i];
                tile[e].y = pre_im[i];
            }
        }
        __syncthreads();
        const int64_t tn = t + walk.step;
        const TileCoord tcn = tile_coord_of(pa, tn < walk.end ? tn : t);
        if (tn < walk.end) load_regs(tcn);
        // one mode of the pass: the products of all fibres of mode q, written
        // back into LDS, or (the last mode) straight to memory
        auto mode = [&](int q, bool last) __attribute__((always_inline)) {
            const R *aq = afr + q * RB * KS * 64 + lane;
            const int nfib = pa.lb * (int)(pa.G / NN) * tc.rbe;
            const int stride = pa.lb * pa.gs[q];
            const int ngroups = (nfib + 15) >> 4;
            const int *fq = fbt + q * nfull;
            const R *tr = reinterpret_cast<const R *>(tile);
            for (int grp = wave; grp < ngroups; grp += WAVES) {
                const int f = 16 * grp + (lane & 15);
                const int base = (f < nfib && (f & (pa.lb - 1)) < tc.lbe) ? fq[min(f, nfull - 1)] : -1;
                const int kb = lane >> 4;  // k within a step
                // all B operands of the group first (branch-free addresses),
                // then the MFMA chain
                R bv[KS];
#pragma unroll
                for (int kk = 0; kk < KS; ++kk) {
                    const int k = 4 * kk + kb;
                    const int m = k >> 1;
                    const int idx = (base >= 0 && m < NN) ? 2 * (base + m * stride) + (k & 1) : zidx;
                    bv[kk] = tr[idx];
                }
                typename MT::acc acc[RB];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) acc[rb] = typename MT::acc{0, 0, 0, 0};
#pragma unroll
                for (int kk = 0; kk < KS; ++kk) {
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
                        acc[rb] = MT::mma(aq[(rb * KS + kk) * 64], bv[kk], acc[rb]);
                }
                __builtin_amdgcn_sched_barrier(0);
                if (base >= 0) {
                    // values (0, 1) and (2, 3) of a lane are two complex outputs
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const int i = 8 * rb + MT::out_of_row(MT::row(lane, 2 * c));
                            if (i < NN) {
                                V y;
                                y.x = acc[rb][2 * c];
                                y.y = acc[rb][2 * c + 1];
                                const int e = base + i * stride;
                                if (last) {
                                    bool ok;
                                    const int64_t a = gaddr(tc, e, ok);
                                    X[a] = y;
                                } else {
                                    tile[e] = y;
                                }
                            }
                        }
                    }
                }
            }
        };
        for (int q = 0; q + 1 < pa.ng; ++q) {
            mode(q, false);
            __syncthreads();
        }
        // the next tile's loads are complete before the last mode, whose
        // results go straight to memory: the LDS refill after it then does
        // not wait on those stores
        __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
        mode(pa.ng - 1, true);
        if (tn >= walk.end) break;
        __syncthreads();  // every wave has read the tile before the refill
        t = tn;
        tc = tcn;
    }
}

// A pass of one mode with extent n > 24 (up to 256) on the matrix cores.  The
// tile (lb x n x rb entries; fibres of stride lb) sits in LDS.  A wave forms
// one 16-row block of the real-form product (the layout of the pass above)
// for 16 fibres at a time: the A fragments come from the matrix in memory
// (cache resident, a handful of lines per k-step), the B operands from LDS.
// Results go straight to memory: the whole tile is in LDS before any of it is
// overwritten, and tiles are disjoint.
constexpr int kLongThreads = 512;
constexpr int kLongUnroll = 8;  // k-steps whose operands are loaded together

template <typename V>
__global__ void __launch_bounds__(kLongThreads) transform_long_mfma_kernel(V *X, const V *Xs,
                                                                           const V *__restrict__ Mbuf,
                                                                           PassDesc pa)
{
    using R = typename CTraits<V>::R;
    using MT = MfmaT<R>;
    const int n = pa.gd[0];
    const int RB = (n + 7) / 8, KS = (2 * n + 3) / 4;
    constexpr int WAVES = kLongThreads / 64;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V *tile = reinterpret_cast<V *>(smem_raw);
    const int total = pa.lb * n * pa.rb;
    R *tr = reinterpret_cast<R *>(tile);
    const int zidx = 2 * total;  // a zero operand after the tile
    if (threadIdx.x == 0) tr[zidx] = R(0);
    const V *M = Mbuf + pa.moff[0];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kb = lane >> 4, r16 = lane & 15, ap = MT::part_of_row(r16);
    const int64_t ntiles = pa.ntl * pa.ntr;
    const TileWalk walk = tile_walk(ntiles);
    for (int64_t t = walk.t; t < walk.end; t += walk.step) {
        const TileCoord tc = tile_coord_of(pa, t);
        __syncthreads();  // every wave is done with the previous tile
        for (int e = threadIdx.x; e < total; e += kLongThreads) {
            const int l = e & (pa.lb - 1), rest = e >> pa.lbshift;
            const int g = rest % n, r = rest / n;
            V v;
            v.x = 0;
            v.y = 0;
            if (l < tc.lbe && r < tc.rbe) v = Xs[tc.l0 + l + pa.Lin * (g + (int64_t)n * (tc.r0 + r))];
            tile[e] = v;
        }
        __syncthreads();
        const int nfib = pa.lb * tc.rbe;
        const int items = ((nfib + 15) >> 4) * RB;
        for (int it = wave; it < items; it += WAVES) {
            const int grp = it / RB, rb = it - grp * RB;
            const int f = 16 * grp + r16;
            const int fl = f & (pa.lb - 1), fr = f >> pa.lbshift;
            const bool fok = f < nfib && fl < tc.lbe;
            const int base = fl + pa.lb * n * fr;
            const int i = 8 * rb + MT::out_of_row(r16);
            typename MT::acc acc = {0, 0, 0, 0};
            for (int kk0 = 0; kk0 < KS; kk0 += kLongUnroll) {
                R a[kLongUnroll], b[kLongUnroll];
#pragma unroll
                for (int u = 0; u < kLongUnroll; ++u) {
                    const int k = 4 * (kk0 + u) + kb;
                    const int m = k >> 1;
                    const bool in = kk0 + u < KS && m < n;
                    const V c = M[(in && i < n) ? i + (int64_t)n * m : 0];
                    a[u] = (in && i < n) ? (ap == (k & 1) ? c.x : (ap ? c.y : -c.y)) : R(0);
                    b[u] = tr[(in && fok) ? 2 * (base + m * pa.lb) + (k & 1) : zidx];
                }
#pragma unroll
                for (int u = 0; u < kLongUnroll; ++u) acc = MT::mma(a[u], b[u], acc);
            }
            if (fok) {
#pragma unroll
                for (int c2 = 0; c2 < 2; ++c2) {
                    const int io = 8 * rb + MT::out_of_row(MT::row(lane, 2 * c2));
                    if (io < n) {
                        V y;
                        y.x = acc[2 * c2];
                        y.y = acc[2 * c2 + 1];
                        X[tc.l0 + fl + pa.Lin * (io + (int64_t)n * (tc.r0 + fr))] = y;
                    }
                }
            }
        }
    }
}

// extents above 24: ping-pong between two LDS tiles; the work items of a mode
// are (fibre, chunk of 8 outputs) pairs
template <typename V>
__global__ void __launch_bounds__(kThreads) transform_pass_generic_kernel(
    V *X, const V *Xs, const V *__restrict__ Mbuf, PassDesc pa)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V *bufA = reinterpret_cast<V *>(smem_raw);
    V *bufB = bufA + (int64_t)pa.lb * pa.G * pa.rb;
    const TileCoord tc = tile_coord(pa);
    load_tile<V, V>(bufA, Xs, pa, tc);
    __syncthreads();
    for (int q = 0; q < pa.ng; ++q) {
        const int n = pa.gd[q];
        const int nfib = pa.lb * (int)(pa.G / n) * tc.rbe;
        const int stride = pa.lb * pa.gs[q];
        const V *M = Mbuf + pa.moff[q];
        const int nchunk = (n + kGenericChunk - 1) / kGenericChunk;
        for (int w = threadIdx.x; w < nfib * nchunk; w += blockDim.x) {
            const int f = w % nfib;
            const int base = fibre_base(pa, tc, q, n, f);
            if (base < 0) continue;
            fibre_generic<V, false>(bufA, bufB, base, stride, n, M, (w / nfib) * kGenericChunk);
        }
        __syncthreads();
        V *t = bufA;
        bufA = bufB;
        bufB = t;
    }
    store_tile<V>(X, bufA, pa, tc);
}

// ------------------------------------------------------------- residual
// pass p of P: R = (p == 0 ? B : R) - sum_{k in run} A_k x_k X on the tile;
// the first pass also subtracts a X for the scalars a of the singleton modes.
// Partial sums of |B|^2 (first pass) and |R|^2 (last pass) per tile.
struct SingletonList {
    int count;
    int64_t off[kMaxModes];  // offsets of the 1x1 A_k in the matrix buffer
};

__device__ __forceinline__ void residual_reduce(double sb, double sr, int first, int last,
                                                double *part_b, double *part_r, int64_t tile,
                                                unsigned char *smem_raw);

// R = src - acc on the tile (src = B in the first pass, R after), written as
// complex128 (and as complex64 r32_scale R in the last pass if R32); per-tile
// partial sums of |B|^2 (first pass) and |R|^2 (last pass) in a fixed order.
__device__ __forceinline__ void residual_finish(const double2 *__restrict__ B, double2 *R, float2 *R32,
                                                const double2 *acc, const PassDesc &pa,
                                                const TileCoord &tc, int first, int last,
                                                double *part_b, double *part_r, int64_t tile,
                                                unsigned char *smem_raw, double r32_scale)
{
    // combine with the source and write; accumulate the norms
    double sb = 0.0, sr = 0.0;
    const double2 *src = first ? B : R;
    const int lbG = pa.lb * (int)pa.G;
    for (int r = 0; r < tc.rbe; ++r) {
        const int64_t gbase = tc.l0 + pa.Lin * pa.G * (tc.r0 + r);
        for (int e = threadIdx.x; e < lbG; e += blockDim.x) {
            const int l = e & (pa.lb - 1);
            const int g = e >> pa.lbshift;
            if (l >= tc.lbe) continue;
            const int64_t gi = gbase + l + pa.Lin * g;
            const double2 s = src[gi];
            const double2 a = acc[e + (int64_t)lbG * r];
            const double2 v = make_double2(s.x - a.x, s.y - a.y);
            if (first) sb += s.x * s.x + s.y * s.y;
            if (last) {
                sr += v.x * v.x + v.y * v.y;
                if (R32) R32[gi] = make_float2((float)(v.x * r32_scale), (float)(v.y * r32_scale));
            }
            if (!last || !R32) R[gi] = v;
        }
    }
    residual_reduce(sb, sr, first, last, part_b, part_r, tile, smem_raw);
}

// per-tile partial sums of |B|^2 and |R|^2: block reduction in a fixed order
// (wave shuffles, then LDS)
__device__ __forceinline__ void residual_reduce(double sb, double sr, int first, int last,
                                                double *part_b, double *part_r, int64_t tile,
                                                unsigned char *smem_raw)
{
    __syncthreads();
    double *red = reinterpret_cast<double *>(smem_raw);
    for (int off = 32; off > 0; off >>= 1) {
        sb += __shfl_down(sb, off, 64);
        sr += __shfl_down(sr, off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        red[2 * wid] = sb;
        red[2 * wid + 1] = sr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tb = 0.0, trr = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            tb += red[2 * w];
            trr += red[2 * w + 1];
        }
        if (first) part_b[tile] = tb;
        if (last) part_r[tile] = trr;
    }
}

template <int NN>
__global__ void __launch_bounds__(kThreads) residual_pass_kernel(
    const double2 *__restrict__ B, const double2 *__restrict__ X, double2 *R, float2 *R32,
    const double2 *__restrict__ Abuf, PassDesc pa, SingletonList sing, int first, int last,
    double *part_b, double *part_r, double r32_scale)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double2 *xt = reinterpret_cast<double2 *>(smem_raw);
    double2 *acc = xt + (int64_t)pa.lb * pa.G * pa.rb;
    const TileCoord tc = tile_coord(pa);
    load_tile<double2, double2>(xt, X, pa, tc);
    __syncthreads();
    double2 shift = make_double2(0.0, 0.0);
    if (first)
        for (int i = 0; i < sing.count; ++i) shift = cadd(shift, Abuf[sing.off[i]]);
    const int total = pa.lb * (int)pa.G * pa.rb;
    for (int e = threadIdx.x; e < total; e += blockDim.x) acc[e] = cmul(shift, xt[e]);
    __syncthreads();
    for (int q = 0; q < pa.ng; ++q) {
        const int n = NN > 0 ? NN : pa.gd[q];
        const int nfib = pa.lb * (int)(pa.G / n) * tc.rbe;
        const int stride = pa.lb * pa.gs[q];
        const double2 *M = Abuf + pa.moff[q];
        // extents above 24: (fibre, chunk of 8 outputs) work items
        const int nchunk = (NN > 0 || n <= 24) ? 1 : (n + kGenericChunk - 1) / kGenericChunk;
        for (int w = threadIdx.x; w < nfib * nchunk; w += blockDim.x) {
            const int f = w % nfib;
            const int base = fibre_base(pa, tc, q, n, f);
            if (base < 0) continue;
            if constexpr (NN > 0)
                fibre_fixed<double2, NN, true>(xt, acc, base, stride, M);
            else if (n <= 24)
                fibre_switch<double2, true>(xt, acc, base, stride, n, M);
            else
                fibre_generic<double2, true>(xt, acc, base, stride, n, M, (w / nfib) * kGenericChunk);
        }
        __syncthreads();
    }
    residual_finish(B, R, R32, acc, pa, tc, first, last, part_b, part_r, blockIdx.x, smem_raw,
                    r32_scale);
}

constexpr int kResidualRegs = kResidualMfmaCap / kMfmaThreads;  // X entries per lane of a tile

// The residual pass on the matrix cores (extents 8, 16 or 19 in the pass):
// the X tile stays in LDS and every mode's product M_q x_q X, formed by the
// same real-ified 16x16x4 MFMA GEMM as the transform pass, is added into an
// LDS accumulator tile instead of overwriting the fibres.
template <int NN>
__global__ void __launch_bounds__(kMfmaThreads) residual_mfma_kernel(
    const double2 *__restrict__ B, const double2 *__restrict__ X, double2 *R, float2 *R32,
    const double2 *__restrict__ Abuf, PassDesc pa, SingletonList sing, int first, int last,
    double *part_b, double *part_r, double r32_scale)
{
    using MT = MfmaT<double>;
    constexpr int RB = (NN + 7) / 8;        // 16-row blocks (8 complex outputs each)
    constexpr int KS = (2 * NN + 3) / 4;
    constexpr int WAVES = kMfmaThreads / 64;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int total = pa.lb * (int)pa.G * pa.rb;
    double2 *xt = reinterpret_cast<double2 *>(smem_raw);
    double2 *acc = xt + total;
    double *afr = reinterpret_cast<double *>(acc + total);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int idx = threadIdx.x; idx < pa.ng * RB * KS * 64; idx += kMfmaThreads) {
        const int l = idx & 63;
        const int frag = idx >> 6;
        const int kk = frag % KS, rb = (frag / KS) % RB, q = frag / (KS * RB);
        const int r = l & 15, k = 4 * kk + (l >> 4);
        const int i = 8 * rb + MT::out_of_row(r), m = k >> 1;
        double v = 0.0;
        if (i < NN && m < NN) {
            const double2 c = Abuf[pa.moff[q] + i + NN * m];
            const int a = MT::part_of_row(r), b = k & 1;
            v = a == b ? c.x : (a ? c.y : -c.y);
        }
        afr[idx] = v;
    }
    int *fbt = reinterpret_cast<int *>(afr + pa.ng * RB * KS * 64);
    build_fibre_table(fbt, pa, NN);
    const int nfull = pa.lb * (int)(pa.G / NN) * pa.rb;
    // a zero operand after the table for lanes outside the tile
    double *zslot = reinterpret_cast<double *>(fbt + ((pa.ng * nfull + 3) & ~3));
    if (threadIdx.x == 0) zslot[0] = 0.0;
    const int zidx = (int)(zslot - reinterpret_cast<double *>(xt));
    double2 shift = make_double2(0.0, 0.0);
    if (first)
        for (int i = 0; i < sing.count; ++i) shift = cadd(shift, Abuf[sing.off[i]]);
    // persistent (tile_walk); the X entries and the combine source (B in the
    // first pass, R after) of the next tile are loaded into registers while
    // this one is multiplied
    const int64_t ntiles = pa.ntl * pa.ntr;
    const TileWalk walk = tile_walk(ntiles);
    int64_t t = walk.t;
    // the norms' partial sums: each lane adds its entries of all the
    // workgroup's tiles (in the fixed order of the walk), and the workgroup
    // reduces them once at the end, into slot blockIdx.x
    double sb_all = 0.0, sr_all = 0.0;
    if (t >= walk.end) {
        residual_reduce(sb_all, sr_all, first, last, part_b, part_r, blockIdx.x, smem_raw);
        return;
    }
    const double2 *src = first ? B : R;
    double pre_re[kResidualRegs], pre_im[kResidualRegs], src_re[kResidualRegs], src_im[kResidualRegs];
    auto gaddr = [&](const TileCoord &c, int e, bool &ok) -> int64_t {
        const int l = e & (pa.lb - 1);
        const int rest = e >> pa.lbshift;
        int g = rest, r = 0;
        if (pa.rb > 1) {
            g = rest % (int)pa.G;
            r = rest / (int)pa.G;
        }
        ok = e < total && l < c.lbe && r < c.rbe;
        return c.l0 + l + pa.Lin * (g + pa.G * (c.r0 + r));
    };
    auto load_regs = [&](const TileCoord &c) {
#pragma unroll
        for (int i = 0; i < kResidualRegs; ++i) {
            bool ok;
            const int64_t gi = gaddr(c, threadIdx.x + i * kMfmaThreads, ok);
            if (ok) {
                const double2 v = X[gi], w = src[gi];
                pre_re[i] = v.x;
                pre_im[i] = v.y;
                src_re[i] = w.x;
                src_im[i] = w.y;
            }
        }
    };
    TileCoord tc = tile_coord_of(pa, t);
    load_regs(tc);
    // the prefetch registers are complete on every path into the loop (here
    // and before the last mode), so refilling the tile never waits on the
    // R stores of the previous tile
    __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
    while (true) {
        double cur_re[kResidualRegs], cur_im[kResidualRegs];
#pragma unroll
        for (int i = 0; i < kResidualRegs; ++i) {
            const int e = threadIdx.x + i * kMfmaThreads;
            cur_re[i] = src_re[i];
            cur_im[i] = src_im[i];
            if (e < total) {
                const double2 x = make_double2(pre_re[i], pre_im[i]);
                xt[e] = x;
                acc[e] = cmul(shift, x);
            }
        }
        __syncthreads();
        const int64_t tn = t + walk.step;
        const TileCoord tcn = tile_coord_of(pa, tn < walk.end ? tn : t);
        if (tn < walk.end) load_regs(tcn);
        const double *tr = reinterpret_cast<const double *>(xt);
        // one mode: acc += A_q x_q (tile), fibre groups of 16 on the matrix cores
        auto mode = [&](int q) __attribute__((always_inline)) {
            const double *aq = afr + q * RB * KS * 64 + lane;
            const int nfib = pa.lb * (int)(pa.G / NN) * tc.rbe;
            const int stride = pa.lb * pa.gs[q];
            const int ngroups = (nfib + 15) >> 4;
            const int *fq = fbt + q * nfull;
            for (int grp = wave; grp < ngroups; grp += WAVES) {
                const int f = 16 * grp + (lane & 15);
                const int base = (f < nfib && (f & (pa.lb - 1)) < tc.lbe) ? fq[min(f, nfull - 1)] : -1;
                const int kb = lane >> 4;
                double bv[KS];
#pragma unroll
                for (int kk = 0; kk < KS; ++kk) {
                    const int k = 4 * kk + kb;
                    const int m = k >> 1;
                    const int idx = (base >= 0 && m < NN) ? 2 * (base + m * stride) + (k & 1) : zidx;
                    bv[kk] = tr[idx];
                }
                typename MT::acc d[RB];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) d[rb] = typename MT::acc{0, 0, 0, 0};
#pragma unroll
                for (int kk = 0; kk < KS; ++kk) {
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) d[rb] = MT::mma(aq[(rb * KS + kk) * 64], bv[kk], d[rb]);
                }
                __builtin_amdgcn_sched_barrier(0);
                if (base >= 0) {
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const int i = 8 * rb + MT::out_of_row(MT::row(lane, 2 * c));
                            if (i < NN) {
                                const int e = base + i * stride;
                                double2 a = acc[e];
                                a.x += d[rb][2 * c];
                                a.y += d[rb][2 * c + 1];
                                acc[e] = a;
                            }
                        }
                    }
                }
            }
        };
        for (int q = 0; q + 1 < pa.ng; ++q) {
            mode(q);
            __syncthreads();
        }
        __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): the next tile is in registers
        mode(pa.ng - 1);
        __syncthreads();
        // R = src - acc, with this tile's source values kept in registers
        // (cur_*) while the next tile's were prefetched
        double sb = 0.0, sr = 0.0;
#pragma unroll
        for (int i = 0; i < kResidualRegs; ++i) {
            const int e = threadIdx.x + i * kMfmaThreads;
            bool ok;
            const int64_t gi = gaddr(tc, e, ok);
            if (ok) {
                const double2 sv = make_double2(cur_re[i], cur_im[i]);
                const double2 a = acc[e];
                const double2 v = make_double2(sv.x - a.x, sv.y - a.y);
                if (first) sb += sv.x * sv.x + sv.y * sv.y;
                if (last) {
                    sr += v.x * v.x + v.y * v.y;
                    if (R32) R32[gi] = make_float2((float)(v.x * r32_scale), (float)(v.y * r32_scale));
                }
                if (!last || !R32) R[gi] = v;
            }
        }
        sb_all += sb;
        sr_all += sr;
        if (tn >= walk.end) break;
        __syncthreads();
        t = tn;
        tc = tcn;
    }
    residual_reduce(sb_all, sr_all, first, last, part_b, part_r, blockIdx.x, smem_raw);
}

// one workgroup of kReduceThreads lanes, fixed order: lane l sums entries
// l + kReduceThreads (8 i + u) into accumulator u (eight loads in flight), the
// accumulators, then the lanes of a wave and the waves are added in a fixed
// order
constexpr int kReduceThreads = 1024;
__global__ void __launch_bounds__(kReduceThreads) reduce_sum_kernel(const double *__restrict__ in,
                                                                    int64_t n, double *out)
{
    __shared__ double red[kReduceThreads / 64];
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t i0 = threadIdx.x; i0 < n; i0 += 8 * (int64_t)kReduceThreads) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t i = i0 + (int64_t)u * kReduceThreads;
            a[u] += i < n ? in[i] : 0.0;
        }
    }
    double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kReduceThreads / 64; ++w) t += red[w];
        *out = t;
    }
}

// LDS bytes of the fibre-base table of a matrix-core pass with extent n
size_t fibre_table_bytes(const PassDesc &pa, int n)
{
    return n > 0 ? (size_t)pa.ng * (size_t)(pa.lb * (pa.G / n) * pa.rb) * sizeof(int) : 0;
}

int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    return cus;
}

template <typename K>
hipError_t allow_lds(K kernel, size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

template <typename V>
hipError_t run_transform_pass(const PassDesc &pa, V *X, const V *Xs, const V *Mbuf, hipStream_t s)
{
    const int64_t tiles = pa.ntl * pa.ntr;
    const bool generic = pa.maxn > 24;
    const size_t lds = pa.lds_bytes(sizeof(V)) * (generic ? 2 : 1);
    hipError_t e;
#define SYLT_LAUNCH(KER)                                                                  \
    do {                                                                                  \
        e = allow_lds(KER, lds);                                                          \
        if (e != hipSuccess) return e;                                                    \
        hipLaunchKernelGGL(KER, dim3((unsigned)tiles), dim3(kThreads), lds, s, X, Xs, Mbuf, pa); \
    } while (0)
    if (generic && pa.ng == 1) {
        // one long mode: the matrix-core pass above
        const size_t ldsl = pa.lds_bytes(sizeof(V)) + 32;
        auto ker = transform_long_mfma_kernel<V>;
        e = allow_lds(ker, ldsl);
        if (e != hipSuccess) return e;
        int occ = 1;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, ker, kLongThreads, ldsl) != hipSuccess ||
            occ < 1)
            occ = 1;
        const int64_t grid = std::min<int64_t>(tiles, (int64_t)device_cus() * occ);
        hipLaunchKernelGGL(ker, dim3((unsigned)grid), dim3(kLongThreads), ldsl, s, X, Xs, Mbuf, pa);
        return hipGetLastError();
    }
    const bool pipe = !generic && pa.lb * pa.G * pa.rb <= kPipeRegs * kPipeThreads &&
                      (pa.uniform_n == 2 || pa.uniform_n == 4 || pa.uniform_n == 8 ||
                       pa.uniform_n == 16 || pa.uniform_n == 19);
    if (pipe) {
        const int cus = device_cus();  // of the current device (attributes are per device)
#define SYLT_PIPE(NNV, PV)                                                                     \
    do {                                                                                       \
        auto ker = transform_pipe_kernel<V, NNV, PV>;                                          \
        e = allow_lds(ker, lds);                                                               \
        if (e != hipSuccess) return e;                                                         \
        int occ = 1;                                                                           \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, ker, kPipeThreads, lds) !=      \
                hipSuccess || occ < 1)                                                         \
            occ = 1;                                                                           \
        const int64_t grid = std::min<int64_t>(tiles, (int64_t)cus * occ);                     \
        hipLaunchKernelGGL(ker, dim3((unsigned)grid), dim3(kPipeThreads), lds, s, X, Xs, Mbuf, pa); \
    } while (0)
        const size_t max_lds = max_lds_bytes();
        // the MFMA variant also keeps the real-form matrix fragments in LDS;
        // if they do not fit next to the tile, the VALU variant runs instead
#define SYLT_MFMA(NNV, PV)                                                                      \
    do {                                                                                        \
        constexpr int RBv = (NNV + 7) / 8, KSv = (2 * NNV + 3) / 4;                             \
        const size_t ldsm = lds + (size_t)pa.ng * RBv * KSv * 64 * sizeof(typename CTraits<V>::R) + \
                            fibre_table_bytes(pa, NNV) + 32;                                    \
        if (ldsm > max_lds) {                                                                   \
            SYLT_PIPE(NNV, PV);                                                                 \
            break;                                                                              \
        }                                                                                       \
        auto ker = transform_mfma_kernel<V, NNV>;                                               \
        e = allow_lds(ker, ldsm);                                                               \
        if (e != hipSuccess) return e;                                                          \
        int occ = 1;                                                                            \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, ker, kMfmaThreads, ldsm) !=      \
                hipSuccess || occ < 1)                                                          \
            occ = 1;                                                                            \
        const int64_t grid = std::min<int64_t>(tiles, (int64_t)cus * occ);                      \
        hipLaunchKernelGGL(ker, dim3((unsigned)grid), dim3(kMfmaThreads), ldsm, s, X, Xs, Mbuf, pa); \
    } while (0)
        switch (pa.uniform_n) {
            case 2: SYLT_PIPE(2, 1); break;
            case 4: SYLT_PIPE(4, 1); break;
            case 8: SYLT_MFMA(8, 2); break;
            case 16: SYLT_MFMA(16, 4); break;
            default: SYLT_MFMA(19, 4); break;
        }
#undef SYLT_PIPE
#undef SYLT_MFMA
    } else if (generic) {
        SYLT_LAUNCH(transform_pass_generic_kernel<V>);
    } else {
        switch (pa.uniform_n) {
            case 2: SYLT_LAUNCH((transform_pass_kernel<V, 2>)); break;
            case 4: SYLT_LAUNCH((transform_pass_kernel<V, 4>)); break;
            case 8: SYLT_LAUNCH((transform_pass_kernel<V, 8>)); break;
            case 16: SYLT_LAUNCH((transform_pass_kernel<V, 16>)); break;
            case 19: SYLT_LAUNCH((transform_pass_kernel<V, 19>)); break;
            default: SYLT_LAUNCH((transform_pass_kernel<V, 0>)); break;
        }
    }
#undef SYLT_LAUNCH
    return hipGetLastError();
}

}  // namespace

hipError_t launch_transform(const sylt_plan_s &p, int dir, int precision, void *X, hipStream_t s)
{
    for (const PassDesc &pa : p.passes) {
        hipError_t e;
        if (precision == SYLT_FP64) {
            const double2 *M = dir == SYLT_TO_SCHUR ? p.dUh : p.dU;
            double2 *Xd = static_cast<double2 *>(X);
            e = run_transform_pass<double2>(pa, Xd, Xd, M, s);
        } else {
            const float2 *M = dir == SYLT_TO_SCHUR ? p.dUh32 : p.dU32;
            float2 *Xf = static_cast<float2 *>(X);
            e = run_transform_pass<float2>(pa, Xf, Xf, M, s);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_transform_from(const sylt_plan_s &p, int dir, const double2 *src, double2 *X,
                                 hipStream_t s)
{
    if (p.passes.empty()) return src == X ? hipSuccess : launch_copy_c128(X, src, p.ntot, s);
    const double2 *M = dir == SYLT_TO_SCHUR ? p.dUh : p.dU;
    for (size_t i = 0; i < p.passes.size(); ++i) {
        const hipError_t e = run_transform_pass<double2>(p.passes[i], X, i == 0 ? src : X, M, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t residual_mfma_lds(const PassDesc &pa)
{
    const int n = pa.uniform_n;
    const size_t frags = (size_t)pa.ng * ((n + 7) / 8) * ((2 * n + 3) / 4) * 64;
    return pa.lds_bytes(sizeof(double2)) * 2 + frags * sizeof(double) + fibre_table_bytes(pa, n) + 32;
}

hipError_t launch_transform_with(const sylt_plan_s &p, const double2 *M, double2 *X, hipStream_t s)
{
    for (const PassDesc &pa : p.passes) {
        const hipError_t e = run_transform_pass<double2>(pa, X, X, M, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_residual(const sylt_plan_s &p, const double2 *B, const double2 *X, double2 *R64,
                           float2 *R32, double *norms2_dev, hipStream_t s, double r32_scale)
{
    return launch_residual_with(p, p.dA, B, X, R64, R32, norms2_dev, s, r32_scale);
}

hipError_t launch_residual_with(const sylt_plan_s &p, const double2 *Mbuf, const double2 *B,
                                const double2 *X, double2 *R64, float2 *R32, double *norms2_dev,
                                hipStream_t s, double r32_scale)
{
    const std::vector<PassDesc> &passes = p.residual_mfma ? p.mrpasses : p.rpasses;
    const int P = (int)passes.size();
    // plan scratch: [part_b (max tiles)] [part_r (max tiles)]
    int64_t maxt = 1;
    for (const PassDesc &pa : passes) maxt = std::max<int64_t>(maxt, pa.ntl * pa.ntr);
    double *part_b = p.dScratch;
    double *part_r = p.dScratch + maxt;
    if (P == 0) return hipErrorInvalidValue;  // all modes singleton: not supported here
    SingletonList sing{};
    for (int k = 0; k < p.N; ++k)
        if (p.n[k] == 1) sing.off[sing.count++] = p.moff[k];
    for (int i = 0; i < P; ++i) {
        const PassDesc &pa = passes[i];
        const int64_t tiles = pa.ntl * pa.ntr;
        const size_t lds = std::max<size_t>(pa.lds_bytes(sizeof(double2)) * 2, 64);
        const int first = i == 0, last = i == P - 1;
        hipError_t e;
        if (p.residual_mfma) {
            int64_t mgrid = 0;  // workgroups of the pass: one partial sum each
#define SYLT_MRLAUNCH(NNV)                                                                        \
    do {                                                                                          \
        const size_t mlds = residual_mfma_lds(pa);                                                \
        e = allow_lds(residual_mfma_kernel<NNV>, mlds);                                           \
        if (e != hipSuccess) return e;                                                            \
        int occ = 1;                                                                              \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, residual_mfma_kernel<NNV>,         \
                                                         kMfmaThreads, mlds) != hipSuccess ||     \
            occ < 1)                                                                              \
            occ = 1;                                                                              \
        const int64_t grid = std::min<int64_t>(tiles, (int64_t)device_cus() * occ);              \
        mgrid = grid;                                                                             \
        hipLaunchKernelGGL(residual_mfma_kernel<NNV>, dim3((unsigned)grid), dim3(kMfmaThreads),   \
                           mlds, s, B, X, R64, last ? R32 : nullptr, Mbuf, pa, sing, first, last, \
                           part_b, part_r, r32_scale);                                            \
    } while (0)
            switch (pa.uniform_n) {
                case 8: SYLT_MRLAUNCH(8); break;
                case 16: SYLT_MRLAUNCH(16); break;
                case 19: SYLT_MRLAUNCH(19); break;
                default: return hipErrorInvalidValue;
            }
#undef SYLT_MRLAUNCH
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            if (first && norms2_dev)
                hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(kReduceThreads), 0, s, part_b, mgrid,
                                   norms2_dev + 1);
            if (last && norms2_dev)
                hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(kReduceThreads), 0, s, part_r, mgrid,
                                   norms2_dev + 0);
            continue;
        }
#define SYLT_RLAUNCH(KER)                                                                       \
    do {                                                                                        \
        e = allow_lds(KER, lds);                                                                \
        if (e != hipSuccess) return e;                                                          \
        hipLaunchKernelGGL(KER, dim3((unsigned)tiles), dim3(kThreads), lds, s, B, X, R64,       \
                           last ? R32 : nullptr, Mbuf, pa, sing, first, last, part_b, part_r,   \
                           r32_scale);                                                          \
    } while (0)
        switch (pa.uniform_n) {
            case 2: SYLT_RLAUNCH(residual_pass_kernel<2>); break;
            case 4: SYLT_RLAUNCH(residual_pass_kernel<4>); break;
            case 8: SYLT_RLAUNCH(residual_pass_kernel<8>); break;
            case 16: SYLT_RLAUNCH(residual_pass_kernel<16>); break;
            case 19: SYLT_RLAUNCH(residual_pass_kernel<19>); break;
            default: SYLT_RLAUNCH(residual_pass_kernel<0>); break;
        }
#undef SYLT_RLAUNCH
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (first && norms2_dev)
            hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(kReduceThreads), 0, s, part_b, tiles,
                               norms2_dev + 1);
        if (last && norms2_dev)
            hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(kReduceThreads), 0, s, part_r, tiles,
                               norms2_dev + 0);
    }
    return hipGetLastError();
}

}  // namespace sylt
