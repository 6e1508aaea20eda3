// Small kernels of libsylt: eigenvalue-sum separation, elementwise
// conversions / updates and the grad-A contraction.
#include "sylt_internal.h"

#include <mutex>

// Fixed device memory for the entry point that allocates nothing
// (sylt_solve_backward_noalloc): the grad-A partial sums.  Every device the
// library runs on holds its own copy until the process ends.  In host code
// this name is only a stand-in for the symbol: the device address comes from
// hipGetSymbolAddress (noalloc_scratch below) and is the only form of it that
// reaches a kernel or a memory call.
static __device__ __align__(256) unsigned char scratch[sylt::kNoAllocScratchBytes];

namespace sylt {

hipError_t noalloc_scratch(void **ptr, size_t *bytes)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        // once per device, with that device current: its copy of the array
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = kNoAllocScratchBytes;
    return hipSuccess;
}

namespace {

constexpr int kThreads = 256;

// ------------------------------------------------------------ separation
// sep = min over multi-indices i of |shift + sum_j lambda_{j, i_j}| (the
// solvability condition of Section 2).  The compressed modes are split into a
// prefix [0, p) whose eigenvalue sums (at most 4096) are tabulated in LDS and
// the remaining modes, enumerated one index per lane; each lane scans the
// table.  Squared magnitudes are reduced; the square root is taken at the end.
struct SepDesc {
    int M, p;
    int d[kMaxModes];
    int64_t moff[kMaxModes];  // T_j offsets; lambda_{j,i} = T_j[i + d_j i]
    int nsing;
    int64_t singoff[kMaxModes];
    int64_t Pin, Pout;
};

__device__ inline double2 lambda_sum(const double2 *__restrict__ T, const SepDesc &sd, int j0,
                                     int j1, int64_t idx)
{
    double2 s = make_double2(0.0, 0.0);
    for (int j = j0; j < j1; ++j) {
        const int i = (int)(idx % sd.d[j]);
        idx /= sd.d[j];
        s = cadd(s, T[sd.moff[j] + (int64_t)i * (sd.d[j] + 1)]);
    }
    return s;
}

__global__ void __launch_bounds__(kThreads) separation_kernel(const double2 *__restrict__ T,
                                                              SepDesc sd, double *partial)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double2 *tab = reinterpret_cast<double2 *>(smem_raw);
    __shared__ double red[kThreads / 64];
    for (int64_t a = threadIdx.x; a < sd.Pin; a += blockDim.x)
        tab[a] = lambda_sum(T, sd, 0, sd.p, a);
    double2 shift = make_double2(0.0, 0.0);
    for (int i = 0; i < sd.nsing; ++i) shift = cadd(shift, T[sd.singoff[i]]);
    __syncthreads();
    double best = INFINITY;
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < sd.Pout;
         o += (int64_t)gridDim.x * blockDim.x) {
        const double2 b = cadd(shift, lambda_sum(T, sd, sd.p, sd.M, o));
        for (int64_t a = 0; a < sd.Pin; ++a) {
            const double2 v = cadd(tab[a], b);
            best = fmin(best, v.x * v.x + v.y * v.y);
        }
    }
    for (int off = 32; off > 0; off >>= 1) best = fmin(best, __shfl_down(best, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmin(m, red[w]);
        partial[blockIdx.x] = m;
    }
}

__global__ void min_sqrt_kernel(const double *__restrict__ partial, int n, double *out)
{
    __shared__ double red[kThreads / 64];
    double m = INFINITY;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmin(m, partial[i]);
    for (int off = 32; off > 0; off >>= 1) m = fmin(m, __shfl_down(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) t = fmin(t, red[w]);
        *out = sqrt(t);
    }
}

// ------------------------------------------------------------ elementwise
// out = complex64(scale * in); scale is a power of two, so only the cast rounds
__global__ void convert_kernel(float2 *__restrict__ out, const double2 *__restrict__ in, int64_t n,
                               double scale)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 v = in[i];
        out[i] = make_float2((float)(v.x * scale), (float)(v.y * scale));
    }
}

// X += unscale D (assign == 0) or X = unscale D (assign != 0), D complex64,
// X complex128; unscale is a power of two (exact)
__global__ void axpy_kernel(double2 *__restrict__ X, const float2 *__restrict__ D, int64_t n,
                            int assign, double unscale)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float2 d = D[i];
        const double dx = (double)d.x * unscale, dy = (double)d.y * unscale;
        if (assign) {
            X[i] = make_double2(dx, dy);
        } else {
            const double2 x = X[i];
            X[i] = make_double2(x.x + dx, x.y + dy);
        }
    }
}

// per-block maxima of max(|re|, |im|) (a NaN anywhere makes its block's NaN)
__global__ void max_abs_kernel(const double2 *__restrict__ in, int64_t n, double *partial)
{
    __shared__ double red[kThreads / 64];
    double m = 0.0;
    bool nan = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 v = in[i];
        nan |= v.x != v.x || v.y != v.y;
        m = fmax(m, fmax(fabs(v.x), fabs(v.y)));
    }
    if (nan) m = NAN;
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_down(m, off, 64);
        m = (m != m || o != o) ? NAN : fmax(m, o);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) t = (t != t || red[w] != red[w]) ? NAN : fmax(t, red[w]);
        partial[blockIdx.x] = t;
    }
}

__global__ void max_reduce_kernel(const double *__restrict__ partial, int n, double *out)
{
    __shared__ double red[kThreads / 64];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) m = (m != m || partial[i] != partial[i]) ? NAN : fmax(m, partial[i]);
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_down(m, off, 64);
        m = (m != m || o != o) ? NAN : fmax(m, o);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) t = (t != t || red[w] != red[w]) ? NAN : fmax(t, red[w]);
        *out = t;
    }
}

__global__ void copy_kernel(double2 *__restrict__ out, const double2 *__restrict__ in, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

unsigned grid_for(int64_t n)
{
    const int64_t blocks = (n + kThreads - 1) / kThreads;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks, 256 * 64));
}

// ------------------------------------------------------------ grad A
// grad_{A_k}(a, m) = -sum over fibres (l, r) of G[l, a, r] conj(X[l, m, r])
// with the tensor viewed as (L, n, R).  Stage 1: the fibres are cut into
// chunks of FB; a workgroup stages one chunk of G and X at a time in LDS and
// adds its n x n contribution into its own partial sum (chunks b, b + grid,
// ...); stage 2 adds the partials in a fixed order (deterministic) and negates.
__global__ void __launch_bounds__(kThreads) grad_partial_kernel(const double2 *__restrict__ G,
                                                                const double2 *__restrict__ X,
                                                                int64_t L, int n, int64_t R,
                                                                int FB, double2 *partial)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double2 *gt = reinterpret_cast<double2 *>(smem_raw);
    double2 *xt = gt + (int64_t)FB * n;
    const int64_t nfib = L * R;
    const int64_t nchunks = (nfib + FB - 1) / FB;
    double2 *mine = partial + (int64_t)blockIdx.x * n * n;
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t f0 = c * FB;
        const int nf = (int)std::min<int64_t>(FB, nfib - f0);
        for (int e = threadIdx.x; e < nf * n; e += blockDim.x) {
            const int fl = e % nf, m = e / nf;
            const int64_t f = f0 + fl;
            const int64_t l = f % L, r = f / L;
            const int64_t gi = l + L * (m + (int64_t)n * r);
            gt[fl + nf * m] = G[gi];
            xt[fl + nf * m] = X[gi];
        }
        __syncthreads();
        const bool first = c == blockIdx.x;
        for (int pair = threadIdx.x; pair < n * n; pair += blockDim.x) {
            const int a = pair % n, m = pair / n;
            double2 acc = first ? make_double2(0.0, 0.0) : mine[pair];
            for (int fl = 0; fl < nf; ++fl) {
                const double2 g = gt[fl + nf * a], x = xt[fl + nf * m];
                acc.x = fma(g.x, x.x, acc.x);
                acc.x = fma(g.y, x.y, acc.x);
                acc.y = fma(g.y, x.x, acc.y);
                acc.y = fma(-g.x, x.y, acc.y);
            }
            mine[pair] = acc;
        }
        __syncthreads();
    }
}

__global__ void grad_final_kernel(const double2 *__restrict__ partial, int nblocks, int n,
                                  double2 *__restrict__ out)
{
    const int pair = blockIdx.x * blockDim.x + threadIdx.x;
    if (pair >= n * n) return;
    double2 s = make_double2(0.0, 0.0);
    for (int b = 0; b < nblocks; ++b) s = cadd(s, partial[(int64_t)b * n * n + pair]);
    out[pair] = make_double2(-s.x, -s.y);
}

int grad_fibres_per_block(int n) { return std::max(1, 2048 / n); }

// workgroups of stage 1: one per chunk, at most kGradMaxBlocks (which bounds
// the partial sums at kGradMaxBlocks n^2 entries)
constexpr int64_t kGradMaxBlocks = 512;
int64_t grad_blocks(int64_t nfib, int n)
{
    const int FB = grad_fibres_per_block(n);
    return std::max<int64_t>(1, std::min<int64_t>((nfib + FB - 1) / FB, kGradMaxBlocks));
}

}  // namespace

hipError_t launch_separation(const sylt_plan_s &p, double *d_out, hipStream_t s)
{
    SepDesc sd{};
    sd.M = p.M;
    for (int j = 0; j < p.M; ++j) {
        sd.d[j] = p.cdim[j];
        sd.moff[j] = p.moff[p.cmode[j]];
    }
    for (int k = 0; k < p.N; ++k)
        if (p.n[k] == 1) sd.singoff[sd.nsing++] = p.moff[k];
    int64_t Pin = 1;
    int pfx = 0;
    while (pfx < p.M && Pin * p.cdim[pfx] <= 4096) Pin *= p.cdim[pfx++];
    sd.p = pfx;
    sd.Pin = Pin;
    sd.Pout = p.ntot / Pin;
    double *partial = p.dScratch;  // first 4096 doubles of the plan scratch
    const int64_t want = (sd.Pout + kThreads - 1) / kThreads;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, 4096));
    const size_t lds = (size_t)Pin * sizeof(double2);
    hipLaunchKernelGGL(separation_kernel, dim3(blocks), dim3(kThreads), lds, s, p.dT, sd, partial);
    hipLaunchKernelGGL(min_sqrt_kernel, dim3(1), dim3(kThreads), 0, s, partial, blocks, d_out);
    return hipGetLastError();
}

hipError_t launch_convert_c128_c64(float2 *out, const double2 *in, int64_t n, double scale,
                                   hipStream_t s)
{
    hipLaunchKernelGGL(convert_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, out, in, n, scale);
    return hipGetLastError();
}

hipError_t launch_axpy_c64(double2 *X, const float2 *D, int64_t n, int assign, double unscale,
                           hipStream_t s)
{
    hipLaunchKernelGGL(axpy_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, X, D, n, assign,
                       unscale);
    return hipGetLastError();
}

hipError_t launch_max_abs_c128(const double2 *in, int64_t n, double *partial, double *d_out,
                               hipStream_t s)
{
    const int blocks = (int)std::max<int64_t>(
        1, std::min<int64_t>((n + kThreads - 1) / kThreads, kMaxAbsBlocks));
    hipLaunchKernelGGL(max_abs_kernel, dim3(blocks), dim3(kThreads), 0, s, in, n, partial);
    hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(kThreads), 0, s, partial, blocks, d_out);
    return hipGetLastError();
}

hipError_t launch_copy_c128(double2 *out, const double2 *in, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, out, in, n);
    return hipGetLastError();
}

size_t grad_A_workspace(const sylt_plan_s &p)
{
    size_t need = 0;
    for (int k = 0; k < p.N; ++k) {
        const int n = (int)p.n[k];
        const int64_t blocks = grad_blocks(p.ntot / n, n);
        need = std::max(need, (size_t)blocks * n * n * sizeof(double2));
    }
    return need;
}

// The partial sums take blocks * n^2 entries; with a buffer smaller than
// grad_A_workspace the stage-1 grid shrinks to what fits (each workgroup then
// walks more chunks).  A buffer below one n x n matrix is rejected.
hipError_t launch_grad_A(const sylt_plan_s &p, const double2 *G, const double2 *X, double2 *const *GA,
                         void *ws, size_t ws_bytes, hipStream_t s)
{
    double2 *partial = static_cast<double2 *>(ws);
    for (int k = 0; k < p.N; ++k) {
        if (!GA[k]) continue;
        const int n = (int)p.n[k];
        if (ws_bytes < (size_t)n * n * sizeof(double2)) return hipErrorInvalidValue;
    }
    for (int k = 0; k < p.N; ++k) {
        if (!GA[k]) continue;
        const int n = (int)p.n[k];
        int64_t L = 1, R = 1;
        for (int j = 0; j < k; ++j) L *= p.n[j];
        for (int j = k + 1; j < p.N; ++j) R *= p.n[j];
        const int FB = grad_fibres_per_block(n);
        const int64_t fit = (int64_t)(ws_bytes / ((size_t)n * n * sizeof(double2)));
        const int64_t blocks = std::min(grad_blocks(L * R, n), fit);
        const size_t lds = (size_t)2 * FB * n * sizeof(double2);
        hipLaunchKernelGGL(grad_partial_kernel, dim3((unsigned)blocks), dim3(kThreads), lds, s, G, X,
                           L, n, R, FB, partial);
        hipLaunchKernelGGL(grad_final_kernel, dim3((n * n + kThreads - 1) / kThreads),
                           dim3(kThreads), 0, s, partial, (int)blocks, n, GA[k]);
    }
    return hipGetLastError();
}

}  // namespace sylt
