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

// any extent n <= 64: outputs in chunks of 8, written to a separate buffer
template <typename V, bool ACC>
__device__ __forceinline__ void fibre_generic(const V *src, V *dst, int base, int stride, int n,
                                              const V *__restrict__ M)
{
    for (int ic = 0; ic < n; ic += 8) {
        V y[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) y[i] = vzero<V>();
        for (int m = 0; m < n; ++m) {
            const V x = src[base + m * stride];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (ic + i < n) y[i] = cmac(y[i], M[ic + i + n * m], x);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (ic + i < n) {
                if (ACC)
                    dst[base + (ic + i) * stride] = vadd(dst[base + (ic + i) * stride], y[i]);
                else
                    dst[base + (ic + i) * stride] = y[i];
            }
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

// ------------------------------------------------------------ transform
// NN > 0: every mode of the group has extent NN.  NN == 0: mixed extents <= 24.
template <typename V, int NN>
__global__ void __launch_bounds__(kThreads) transform_pass_kernel(V *__restrict__ X,
                                                                  const V *__restrict__ Mbuf,
                                                                  PassDesc pa)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V *tile = reinterpret_cast<V *>(smem_raw);
    const TileCoord tc = tile_coord(pa);
    load_tile<V, V>(tile, X, pa, tc);
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

// extents up to 64: ping-pong between two LDS tiles
template <typename V>
__global__ void __launch_bounds__(kThreads) transform_pass_generic_kernel(
    V *__restrict__ X, const V *__restrict__ Mbuf, PassDesc pa)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V *bufA = reinterpret_cast<V *>(smem_raw);
    V *bufB = bufA + (int64_t)pa.lb * pa.G * pa.rb;
    const TileCoord tc = tile_coord(pa);
    load_tile<V, V>(bufA, X, pa, tc);
    __syncthreads();
    for (int q = 0; q < pa.ng; ++q) {
        const int n = pa.gd[q];
        const int nfib = pa.lb * (int)(pa.G / n) * tc.rbe;
        const int stride = pa.lb * pa.gs[q];
        const V *M = Mbuf + pa.moff[q];
        for (int f = threadIdx.x; f < nfib; f += blockDim.x) {
            const int base = fibre_base(pa, tc, q, n, f);
            if (base < 0) continue;
            fibre_generic<V, false>(bufA, bufB, base, stride, n, M);
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

template <int NN>
__global__ void __launch_bounds__(kThreads) residual_pass_kernel(
    const double2 *__restrict__ B, const double2 *__restrict__ X, double2 *R, float2 *R32,
    const double2 *__restrict__ Abuf, PassDesc pa, SingletonList sing, int first, int last,
    double *part_b, double *part_r)
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
        for (int f = threadIdx.x; f < nfib; f += blockDim.x) {
            const int base = fibre_base(pa, tc, q, n, f);
            if (base < 0) continue;
            if constexpr (NN > 0)
                fibre_fixed<double2, NN, true>(xt, acc, base, stride, M);
            else if (n <= 24)
                fibre_switch<double2, true>(xt, acc, base, stride, n, M);
            else
                fibre_generic<double2, true>(xt, acc, base, stride, n, M);
        }
        __syncthreads();
    }
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
                if (R32) R32[gi] = make_float2((float)v.x, (float)v.y);
            }
            if (!last || !R32) R[gi] = v;
        }
    }
    // block reduction (fixed order: wave shuffles then LDS)
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
        if (first) part_b[blockIdx.x] = tb;
        if (last) part_r[blockIdx.x] = trr;
    }
}

__global__ void reduce_sum_kernel(const double *__restrict__ in, int64_t n, double *out)
{
    // one workgroup, fixed order
    __shared__ double red[kThreads / 64];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += in[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        *out = t;
    }
}

template <typename K>
hipError_t allow_lds(K kernel, size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

template <typename V>
hipError_t run_transform_pass(const PassDesc &pa, V *X, const V *Mbuf, hipStream_t s)
{
    const int64_t tiles = pa.ntl * pa.ntr;
    const bool generic = pa.maxn > 24;
    const size_t lds = pa.lds_bytes(sizeof(V)) * (generic ? 2 : 1);
    hipError_t e;
#define SYLT_LAUNCH(KER)                                                                  \
    do {                                                                                  \
        e = allow_lds(KER, lds);                                                          \
        if (e != hipSuccess) return e;                                                    \
        hipLaunchKernelGGL(KER, dim3((unsigned)tiles), dim3(kThreads), lds, s, X, Mbuf, pa); \
    } while (0)
    if (generic) {
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
            e = run_transform_pass<double2>(pa, static_cast<double2 *>(X), M, s);
        } else {
            const float2 *M = dir == SYLT_TO_SCHUR ? p.dUh32 : p.dU32;
            e = run_transform_pass<float2>(pa, static_cast<float2 *>(X), M, s);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_residual(const sylt_plan_s &p, const double2 *B, const double2 *X, double2 *R64,
                           float2 *R32, double *norms2_dev, hipStream_t s)
{
    const int P = (int)p.rpasses.size();
    // plan scratch: [part_b (max tiles)] [part_r (max tiles)]
    int64_t maxt = 1;
    for (const PassDesc &pa : p.rpasses) maxt = std::max<int64_t>(maxt, pa.ntl * pa.ntr);
    double *part_b = p.dScratch;
    double *part_r = p.dScratch + maxt;
    if (P == 0) return hipErrorInvalidValue;  // all modes singleton: not supported here
    SingletonList sing{};
    for (int k = 0; k < p.N; ++k)
        if (p.n[k] == 1) sing.off[sing.count++] = p.moff[k];
    for (int i = 0; i < P; ++i) {
        const PassDesc &pa = p.rpasses[i];
        const int64_t tiles = pa.ntl * pa.ntr;
        const size_t lds = std::max<size_t>(pa.lds_bytes(sizeof(double2)) * 2, 64);
        const int first = i == 0, last = i == P - 1;
        hipError_t e;
#define SYLT_RLAUNCH(KER)                                                                       \
    do {                                                                                        \
        e = allow_lds(KER, lds);                                                                \
        if (e != hipSuccess) return e;                                                          \
        hipLaunchKernelGGL(KER, dim3((unsigned)tiles), dim3(kThreads), lds, s, B, X, R64,       \
                           last ? R32 : nullptr, p.dA, pa, sing, first, last, part_b, part_r);  \
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
            hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(kThreads), 0, s, part_b, tiles,
                               norms2_dev + 1);
        if (last && norms2_dev)
            hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(kThreads), 0, s, part_r, tiles,
                               norms2_dev + 0);
    }
    return hipGetLastError();
}

}  // namespace sylt
