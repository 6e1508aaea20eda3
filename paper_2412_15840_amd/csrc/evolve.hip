// Device pieces of the time evolution (Theorem 1 in Schur form, eqs.
// e:sylvesterNDG and e:G): the matrix exponentials exp(t T_k) of the
// triangular Schur factors (eq. e:exptAj), the scalars contributed by the
// singleton modes, and an elementwise linear combination.
//
// exp(t T) for an upper triangular T (n <= 256) by scaling and squaring of a
// truncated Taylor series: with s the smallest integer such that
// ||t T||_1 / 2^s <= 1/2, exp(X) for X = t T / 2^s is summed to degree 18 by
// Horner's rule, P <- I + X P / k for k = 18, ..., 1 (the remainder is below
// (1/2)^19 / 19! < 1e-22 in norm), then squared s times.  Products of upper
// triangular matrices stay upper triangular, so only j >= i is formed.
#include "sylt_internal.h"

#include <algorithm>

namespace sylt {
namespace {

constexpr int kExpThreads = 256;
constexpr int kTaylorDegree = 18;

struct ExpJobs {
    int count;
    int n[kMaxModes];
    int64_t off[kMaxModes];
};

// C = A B for upper triangular n x n column-major matrices (C distinct from A, B)
__device__ void triu_product(double2 *C, const double2 *A, const double2 *B, int n)
{
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        const int i = idx % n, j = idx / n;
        double2 acc = make_double2(0.0, 0.0);
        for (int k = i; k <= j; ++k) acc = cmac(acc, A[i + n * k], B[k + n * j]);
        C[idx] = acc;
    }
}

// the three work matrices of a mode live in global memory (n up to 256); the
// block barrier orders their writes and reads within the workgroup
__global__ void __launch_bounds__(kExpThreads) expm_triu_kernel(ExpJobs jobs,
                                                                const double2 *__restrict__ T,
                                                                double2 *E, double2 *W, int64_t mtotal,
                                                                double t)
{
    const int job = blockIdx.x;
    const int n = jobs.n[job];
    const int64_t off = jobs.off[job];
    const double2 *Tj = T + off;
    double2 *X = W + off, *P = W + mtotal + off, *Q = W + 2 * mtotal + off;
    __shared__ int s_sq;
    if (threadIdx.x == 0) {
        double nrm = 0.0;  // 1-norm of t T (largest column sum)
        for (int j = 0; j < n; ++j) {
            double c = 0.0;
            for (int i = 0; i <= j; ++i) c += cabs2(Tj[i + n * j]);
            nrm = fmax(nrm, c);
        }
        nrm *= fabs(t);
        int sq = 0;
        while (nrm > 0.5 && sq < 1000) {
            nrm *= 0.5;
            ++sq;
        }
        s_sq = sq;
    }
    __syncthreads();
    const int sq = s_sq;
    const double scale = ldexp(t, -sq);
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        const int i = idx % n, j = idx / n;
        X[idx] = i <= j ? cscale(Tj[idx], scale) : make_double2(0.0, 0.0);
        P[idx] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    for (int k = kTaylorDegree; k >= 1; --k) {
        triu_product(Q, X, P, n);
        __syncthreads();
        const double inv = 1.0 / k;
        for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
            const int i = idx % n, j = idx / n;
            const double2 q = cscale(Q[idx], inv);
            P[idx] = i == j ? make_double2(1.0 + q.x, q.y) : q;
        }
        __syncthreads();
    }
    for (int r = 0; r < sq; ++r) {
        triu_product(Q, P, P, n);
        __syncthreads();
        for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) P[idx] = Q[idx];
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) E[off + idx] = P[idx];
}

// the coefficient pairs of the two linear combinations of an evolution:
// out = {prod exp(t a_k), -1, 1, sum a_k} over the singleton modes
__global__ void singleton_scalars_kernel(ExpJobs sing, const double2 *__restrict__ E,
                                         const double2 *__restrict__ T, double2 *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double2 prod = make_double2(1.0, 0.0), sum = make_double2(0.0, 0.0);
    for (int i = 0; i < sing.count; ++i) {
        prod = cmul(prod, E[sing.off[i]]);
        sum = cadd(sum, T[sing.off[i]]);
    }
    out[0] = prod;
    out[1] = make_double2(-1.0, 0.0);
    out[2] = make_double2(1.0, 0.0);
    out[3] = sum;
}

__global__ void lincomb_kernel(double2 *out, const double2 *x, const double2 *y,
                               const double2 *__restrict__ c, int64_t n)
{
    const double2 a = c[0], b = c[1];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 u = x[i], v = y[i];
        double2 r = make_double2(0.0, 0.0);
        r = cmac(r, a, u);
        r = cmac(r, b, v);
        out[i] = r;
    }
}

}  // namespace

hipError_t launch_expm(const sylt_plan_s &p, double t, hipStream_t s)
{
    ExpJobs jobs{}, sing{};
    for (int k = 0; k < p.N; ++k) {
        jobs.n[jobs.count] = (int)p.n[k];
        jobs.off[jobs.count] = p.moff[k];
        ++jobs.count;
        if (p.n[k] == 1) sing.off[sing.count++] = p.moff[k];
    }
    hipLaunchKernelGGL(expm_triu_kernel, dim3(jobs.count), dim3(kExpThreads), 0, s, jobs, p.dT, p.dE,
                       p.dEw, p.mtotal, t);
    hipLaunchKernelGGL(singleton_scalars_kernel, dim3(1), dim3(64), 0, s, sing, p.dE, p.dT, p.dEvo);
    return hipGetLastError();
}

hipError_t launch_lincomb(double2 *out, const double2 *x, const double2 *y, const double2 *c,
                          int64_t n, hipStream_t s)
{
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 256 * 64));
    hipLaunchKernelGGL(lincomb_kernel, dim3((unsigned)blocks), dim3(256), 0, s, out, x, y, c, n);
    return hipGetLastError();
}

}  // namespace sylt
