// Complex Schur factorisation A = U T U^* on the device (Section 2 of the
// paper: every A_j is reduced to upper-triangular T_j by a unitary U_j).
//
// One workgroup per matrix.  For n <= 64 one 64-lane wave holds H and U in
// LDS; larger matrices (up to 256) keep H and U in a global work buffer (L2
// resident) and use 256 lanes, the block barriers ordering their accesses
// within the workgroup.  Steps:
//  1. Householder reduction to upper Hessenberg form, accumulating U.
//  2. Single-shift complex QR iteration on the active unreduced window with a
//     Wilkinson shift (exceptional shifts every 10 iterations without
//     deflation), as in Golub & Van Loan, Matrix Computations, Sections
//     7.4-7.5.  Each step factors H_w - mu I with Givens rotations, multiplies
//     back and restores the shift; rotations are also applied to the parts of
//     H outside the window (so the full triangular T results) and to U.
//  3. T = H with its strictly lower part set to exactly zero.
// Rows / columns of every rotation and reflection are spread over the lanes.
#include "sylt_internal.h"

namespace sylt {
namespace {

struct SchurJobs {
    int count;
    int n[kMaxModes];
    int mode[kMaxModes];  // status slot of the job
    int64_t off[kMaxModes];
};

// 1/sqrt(x) for a normal positive x: the hardware estimate refined by two
// Newton steps y <- y + y (1 - x y^2) / 2 (quadratic convergence: each step
// doubles the correct bits of the estimate)
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double e = fma(-(x * y), y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

// FAST selects the reciprocal-square-root form for moduli in range (the
// large-extent kernel, where the rotation sits on the critical path of every
// QR step); the LDS kernel for n <= 64 keeps the hypot form, whose c and s are
// each within about one rounding of a unitary rotation.
template <bool FAST>
__device__ __forceinline__ void givens(double2 a, double2 b, double &c, double2 &s)
{
    // [c s; -conj(s) c] [a; b] = [r; 0] with real c and c^2 + |s|^2 = 1
    const double aa = a.x * a.x + a.y * a.y, bb = b.x * b.x + b.y * b.y;
    // fast form, for |a|^2 and |a|^2 + |b|^2 in [2^-500, 2^500] (which
    // excludes a = 0): w = 1 / (|a| rho) from one reciprocal square root of
    // their product, c = |a|^2 w and s = a conj(b) w; this sits on the
    // critical path of every QR step
    if (FAST && aa > 0x1p-500 && aa < 0x1p500 && bb < 0x1p500) {
        const double w = rsqrt_nr(aa * (aa + bb));
        c = aa * w;
        s = cscale(cmul(a, cconj(b)), w);
        // one first-order step towards c^2 + |s|^2 = 1: the products above
        // carry a few roundings each, and a rotation that is not unitary to
        // rounding lets U drift from unitarity over many QR sweeps
        const double g = fma(-0.5, fma(c, c, fma(s.x, s.x, s.y * s.y)), 1.5);
        c *= g;
        s = cscale(s, g);
        return;
    }
    if (b.x == 0.0 && b.y == 0.0) {
        c = 1.0;
        s = cd(0.0, 0.0);
        return;
    }
    if (a.x == 0.0 && a.y == 0.0) {
        const double absb = cabs2(b);
        c = 0.0;
        s = cd(b.x / absb, -b.y / absb);
        return;
    }
    const double absa = cabs2(a), absb = cabs2(b);
    const double rho = hypot(absa, absb);
    c = absa / rho;
    const double2 ph = cd(a.x / absa, a.y / absa);
    s = cscale(cmul(ph, cconj(b)), 1.0 / rho);
}

// ---- shifted QR of an upper Hessenberg H (global memory) by a 256-lane
// workgroup, for the large-extent form.  The same rotations as the LDS version
// below, ordered so that steps do not wait on memory round trips:
//  * deflation: every lane tests one subdiagonal entry; an LDS maximum gives
//    the largest negligible one (the bottom of the active window);
//  * left rotations (H_w - mu I = Q R): lane c owns column c and carries its
//    entry of the running row k+1; the two entries that define rotation k pass
//    through LDS (two alternating slots, one barrier a step), every lane
//    computes the rotation and lane 0 records it in LDS;
//  * right rotations (R Q, then U <- U Q): lane r owns row r and carries its
//    entry of the running column k+1; no barrier.
// Rows (columns) are loaded in groups of kQrGroup, one group ahead: with
// stores in flight, a wait on a load waits for every memory operation before
// it, so the groups leave one wait per kQrGroup steps.  Loads are unconditional
// from clamped addresses and used as loaded: a value outside the window is
// never used (the step's own lane test excludes it), while masking it (or
// subtracting the shift) right after the load would overwrite the load's
// register and so wait for the load at once, every step.
constexpr int kQrGroup = 8;

__device__ __forceinline__ int qr_block(double2 *H, double2 *Q, int n, int tid, int maxit,
                                        double2 *gs, double *gc, double2 *bc, int *red)
{
    constexpr int G = kQrGroup;
    const double eps = 2.220446049250313e-16;
#define HH(i, j) H[(i) + n * (j)]
    int hi = n - 1, iter = 0, total = 0;
    while (hi > 0) {
        if (tid == 0) *red = 0;
        __syncthreads();
        if (tid >= 1 && tid <= hi) {
            double tst = cabs1(HH(tid - 1, tid - 1)) + cabs1(HH(tid, tid));
            if (tst == 0.0) tst = 1.0;
            if (cabs1(HH(tid, tid - 1)) <= eps * tst) atomicMax(red, tid);
        }
        __syncthreads();
        const int lo = *red;
        if (lo > 0 && tid == 0) HH(lo, lo - 1) = cd(0.0, 0.0);
        if (lo == hi) {
            __syncthreads();
            --hi;
            iter = 0;
            continue;
        }
        if (++total > maxit) return 1;
        ++iter;
        double2 mu;
        const double2 hd = HH(hi, hi);
        if (iter % 10 == 0) {
            mu = cadd(hd, cd(0.75 * cabs1(HH(hi, hi - 1)), 0.0));
        } else {
            const double2 a = HH(hi - 1, hi - 1), b = HH(hi - 1, hi), c = HH(hi, hi - 1);
            const double2 p = cscale(csub(a, hd), 0.5);
            const double2 bc2 = cmul(b, c);
            const double2 disc = csqrt_(cadd(cmul(p, p), bc2));
            const double2 s1 = cadd(p, disc), s2 = csub(p, disc);
            const double2 den = cabs2(s1) >= cabs2(s2) ? s1 : s2;
            mu = (den.x == 0.0 && den.y == 0.0) ? hd : csub(hd, cdiv(bc2, den));
        }
        // left rotations: this lane's entry of row r of H_w - mu I
        const int col = tid;
        // loads from clamped addresses, used as loaded: every lane whose
        // value lies outside the window is masked where it is used, and
        // masking or shifting a value right after its load would make the
        // load wait at once (an overwrite of a load's register waits for it)
        auto ld_row = [&](int r) __attribute__((always_inline)) {
            return HH(min(r, n - 1), min(col, n - 1));
        };
        double2 cur = ld_row(lo), ra[G], rb[G];
        if (col == lo) cur = csub(cur, mu);
#pragma unroll
        for (int i = 0; i < G; ++i) ra[i] = ld_row(lo + 1 + i);
        auto lstep = [&](int k, double2 R) __attribute__((always_inline)) {
            if (k >= hi) return;
            if (col == k + 1) R = csub(R, mu);  // row k+1 of H_w - mu I
            double2 *slot = bc + 2 * (k & 1);
            if (col == k) {
                slot[0] = cur;
                slot[1] = R;
            }
            __syncthreads();
            double c;
            double2 s;
            givens<true>(slot[0], slot[1], c, s);
            if (tid == 0) {
                gc[k] = c;
                gs[k] = s;
            }
            if (col >= k && col < n) {
                HH(k, col) = cadd(cscale(cur, c), cmul(s, R));
                cur = csub(cscale(R, c), cmul(cconj(s), cur));
                if (col == k) HH(k + 1, k) = cd(0.0, 0.0);
            }
        };
        for (int k = lo; k < hi; k += 2 * G) {
#pragma unroll
            for (int i = 0; i < G; ++i) rb[i] = ld_row(k + 1 + G + i);
#pragma unroll
            for (int i = 0; i < G; ++i) lstep(k + i, ra[i]);
            if (k + G >= hi) break;
#pragma unroll
            for (int i = 0; i < G; ++i) ra[i] = ld_row(k + 1 + 2 * G + i);
#pragma unroll
            for (int i = 0; i < G; ++i) lstep(k + G + i, rb[i]);
        }
        if (col >= hi && col < n) HH(hi, col) = cur;
        __syncthreads();
        // right rotations on rows 0..k+1 of H (the shift returns to each
        // diagonal entry when its column is final), then on every row of U
        const int r = tid;
        auto right = [&](double2 *M, bool isH) __attribute__((always_inline)) {
            auto ld_col = [&](int j) __attribute__((always_inline)) {
                return M[min(r, n - 1) + n * min(j, n - 1)];
            };
            const double2 c0 = M[min(r, n - 1) + n * lo];
            double2 cc = (r < n && (!isH || r <= lo + 1)) ? c0 : cd(0.0, 0.0);
            double2 ya[G], yb[G];
#pragma unroll
            for (int i = 0; i < G; ++i) ya[i] = ld_col(lo + 1 + i);
            // the rotations of a group come from LDS in one batch (clamped
            // indices, no branch), so a step waits on no load
            double cg[G];
            double2 sg[G];
            auto ld_rot = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
                for (int i = 0; i < G; ++i) {
                    const int k = min(k0 + i, n - 1);
                    cg[i] = gc[k];
                    sg[i] = gs[k];
                }
            };
            auto rstep = [&](int k, double2 Y, double c, double2 s) __attribute__((always_inline)) {
                if (k >= hi) return;
                if (r < n && (!isH || r <= k + 1)) {
                    const double2 nk = cadd(cscale(cc, c), cmul(cconj(s), Y));
                    M[r + n * k] = (isH && r == k) ? cadd(nk, mu) : nk;
                    cc = csub(cscale(Y, c), cmul(s, cc));
                }
            };
            for (int k = lo; k < hi; k += 2 * G) {
#pragma unroll
                for (int i = 0; i < G; ++i) yb[i] = ld_col(k + 1 + G + i);
                ld_rot(k);
#pragma unroll
                for (int i = 0; i < G; ++i) rstep(k + i, ya[i], cg[i], sg[i]);
                if (k + G >= hi) break;
#pragma unroll
                for (int i = 0; i < G; ++i) ya[i] = ld_col(k + 1 + 2 * G + i);
                ld_rot(k + G);
#pragma unroll
                for (int i = 0; i < G; ++i) rstep(k + G + i, yb[i], cg[i], sg[i]);
            }
            if (r < n && (!isH || r <= hi)) M[r + n * hi] = (isH && r == hi) ? cadd(cc, mu) : cc;
        };
        right(H, true);
        right(Q, false);
        __syncthreads();
    }
    return 0;
#undef HH
}

template <int NT, bool GLOBAL>
__global__ void __launch_bounds__(NT) schur_kernel(SchurJobs jobs, const double2 *__restrict__ A,
                                                   double2 *__restrict__ Uout,
                                                   double2 *__restrict__ Tout, int *status,
                                                   int max_iter_per_n, double2 *work,
                                                   int64_t mtotal)
{
    extern __shared__ double2 smem[];
    const int job = blockIdx.x;
    const int n = jobs.n[job];
    const int64_t off = jobs.off[job];
    const int tid = threadIdx.x;
    // H and Q are n x n, column-major: H[i + n*j]
    double2 *H = GLOBAL ? work + off : smem;
    double2 *Q = GLOBAL ? work + mtotal + off : smem + n * n;
    double2 *v = GLOBAL ? smem : Q + n * n;  // Householder vector (n)
    double2 *gs = v + n;                // rotation sines (n)
    double *gc = reinterpret_cast<double *>(gs + n);  // rotation cosines (n)
#define HH(i, j) H[(i) + n * (j)]
#define QQ(i, j) Q[(i) + n * (j)]

    for (int idx = tid; idx < n * n; idx += NT) {
        H[idx] = A[off + idx];
        Q[idx] = cd((idx % n) == (idx / n) ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();

    // ---- 1. Hessenberg reduction
    for (int k = 0; k + 2 < n; ++k) {
        double sig = 0.0;
        if constexpr (GLOBAL) {
            // one entry per lane, summed over the wave and then over the waves
            // in a fixed order (partials in the sine array, alternating halves
            // by the parity of k so that the next column cannot overwrite them)
            double part = 0.0;
            for (int r = k + 2 + tid; r < n; r += NT) {
                const double2 h = HH(r, k);
                part += h.x * h.x + h.y * h.y;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
            double *red = reinterpret_cast<double *>(gs) + (k & 1) * (NT / 64);
            if ((tid & 63) == 0) red[tid >> 6] = part;
            __syncthreads();
            for (int w = 0; w < NT / 64; ++w) sig += red[w];
        } else {
            for (int r = k + 2; r < n; ++r) {
                const double2 h = HH(r, k);
                sig += h.x * h.x + h.y * h.y;
            }
        }
        if (sig == 0.0) continue;  // uniform: every lane read the same values
        const double2 x0 = HH(k + 1, k);
        const double ax0 = cabs2(x0);
        const double alpha = sqrt(ax0 * ax0 + sig);
        const double2 ph = ax0 > 0.0 ? cd(x0.x / ax0, x0.y / ax0) : cd(1.0, 0.0);
        const double2 v0 = cadd(x0, cscale(ph, alpha));
        const double tau = 2.0 / (v0.x * v0.x + v0.y * v0.y + sig);
        const double2 beta = cscale(ph, -alpha);
        __syncthreads();
        for (int r = k + 1 + tid; r < n; r += NT) v[r] = (r == k + 1) ? v0 : HH(r, k);
        __syncthreads();
        // left: rows k+1.., columns k..n-1:  H <- (I - tau v v^*) H
        for (int c = k + tid; c < n; c += NT) {
            double2 w = cd(0.0, 0.0);
#pragma unroll 8
            for (int r = k + 1; r < n; ++r) w = cmac_conj(w, v[r], HH(r, c));
            w = cscale(w, tau);
#pragma unroll 8
            for (int r = k + 1; r < n; ++r) HH(r, c) = csub(HH(r, c), cmul(v[r], w));
        }
        __syncthreads();
        // right: all rows, columns k+1..:  H <- H (I - tau v v^*),  U <- U (I - tau v v^*)
        for (int r = tid; r < n; r += NT) {
            double2 w = cd(0.0, 0.0);
            double2 wq = cd(0.0, 0.0);
#pragma unroll 8
            for (int c = k + 1; c < n; ++c) {
                w = cmac(w, HH(r, c), v[c]);
                wq = cmac(wq, QQ(r, c), v[c]);
            }
            w = cscale(w, tau);
            wq = cscale(wq, tau);
#pragma unroll 8
            for (int c = k + 1; c < n; ++c) {
                HH(r, c) = csub(HH(r, c), cmul(w, cconj(v[c])));
                QQ(r, c) = csub(QQ(r, c), cmul(wq, cconj(v[c])));
            }
        }
        __syncthreads();
        if (tid == 0) {
            HH(k + 1, k) = beta;
            for (int r = k + 2; r < n; ++r) HH(r, k) = cd(0.0, 0.0);
        }
        __syncthreads();
    }

    // ---- 2. shifted QR on the Hessenberg matrix
    const double eps = 2.220446049250313e-16;
    int hi = n - 1, iter = 0, total = 0, failed = 0;
    const int maxit = max_iter_per_n * n;
    if (GLOBAL) {
        // two pairs of broadcast slots after the cosines (16-byte aligned),
        // then the deflation maximum
        double2 *bc = reinterpret_cast<double2 *>(gc + n + (n & 1));
        failed = qr_block(H, Q, n, tid, maxit, gs, gc, bc, reinterpret_cast<int *>(bc + 4));
        __syncthreads();
        hi = 0;
    }
    while (hi > 0) {
        // deflation scan (every lane computes the same, reading the same LDS)
        int lo = hi;
        while (lo > 0) {
            const double2 h = HH(lo, lo - 1);
            double tst = cabs1(HH(lo - 1, lo - 1)) + cabs1(HH(lo, lo));
            if (tst == 0.0) tst = 1.0;
            if (cabs1(h) <= eps * tst) break;
            --lo;
        }
        __syncthreads();
        if (lo > 0 && tid == 0) HH(lo, lo - 1) = cd(0.0, 0.0);
        __syncthreads();
        if (lo == hi) {
            --hi;
            iter = 0;
            continue;
        }
        if (++total > maxit) {
            failed = 1;
            break;
        }
        ++iter;
        double2 mu;
        const double2 hd = HH(hi, hi);
        if (iter % 10 == 0) {
            // exceptional shift: perturb away from a possibly stagnating shift
            mu = cadd(hd, cd(0.75 * cabs1(HH(hi, hi - 1)), 0.0));
        } else {
            const double2 a = HH(hi - 1, hi - 1), b = HH(hi - 1, hi), c = HH(hi, hi - 1);
            const double2 p = cscale(csub(a, hd), 0.5);
            const double2 bc = cmul(b, c);
            const double2 disc = csqrt_(cadd(cmul(p, p), bc));
            const double2 s1 = cadd(p, disc), s2 = csub(p, disc);
            const double2 den = cabs2(s1) >= cabs2(s2) ? s1 : s2;
            mu = (den.x == 0.0 && den.y == 0.0) ? hd : csub(hd, cdiv(bc, den));
        }
        __syncthreads();
        for (int t = lo + tid; t <= hi; t += NT) HH(t, t) = csub(HH(t, t), mu);
        __syncthreads();
        // H_w - mu I = Q R : rotations from the left, applied across to column n-1
        for (int k = lo; k < hi; ++k) {
            double c;
            double2 s;
            givens<GLOBAL>(HH(k, k), HH(k + 1, k), c, s);
            if (tid == 0) {
                gc[k] = c;
                gs[k] = s;
            }
            __syncthreads();
            for (int col = k + tid; col < n; col += NT) {
                const double2 x = HH(k, col), y = HH(k + 1, col);
                HH(k, col) = cadd(cscale(x, c), cmul(s, y));
                HH(k + 1, col) = csub(cscale(y, c), cmul(cconj(s), x));
            }
            __syncthreads();
            if (tid == 0) HH(k + 1, k) = cd(0.0, 0.0);
            __syncthreads();
        }
        // R Q : rotations from the right on rows 0..k+1, and on U
        for (int k = lo; k < hi; ++k) {
            const double c = gc[k];
            const double2 s = gs[k];
            for (int r = tid; r <= k + 1; r += NT) {
                const double2 x = HH(r, k), y = HH(r, k + 1);
                HH(r, k) = cadd(cscale(x, c), cmul(cconj(s), y));
                HH(r, k + 1) = csub(cscale(y, c), cmul(s, x));
            }
            for (int r = tid; r < n; r += NT) {
                const double2 x = QQ(r, k), y = QQ(r, k + 1);
                QQ(r, k) = cadd(cscale(x, c), cmul(cconj(s), y));
                QQ(r, k + 1) = csub(cscale(y, c), cmul(s, x));
            }
            __syncthreads();
        }
        for (int t = lo + tid; t <= hi; t += NT) HH(t, t) = cadd(HH(t, t), mu);
        __syncthreads();
    }

    // ---- 3. write U and T (strictly lower part of T exactly zero)
    for (int idx = tid; idx < n * n; idx += NT) {
        const int i = idx % n, j = idx / n;
        Uout[off + idx] = Q[idx];
        Tout[off + idx] = (i > j) ? cd(0.0, 0.0) : H[idx];
    }
    if (tid == 0) status[jobs.mode[job]] = failed;
#undef HH
#undef QQ
}

// U^* (conjugate transpose) and complex64 copies of U and U^*; singleton modes
// get U = 1, T = A.
struct PrepJobs {
    int count;
    int n[kMaxModes];
    int64_t off[kMaxModes];
};

__global__ void prepare_factors_kernel(PrepJobs jobs, const double2 *__restrict__ U,
                                       double2 *__restrict__ Uh, float2 *__restrict__ U32,
                                       float2 *__restrict__ Uh32, const double2 *__restrict__ T,
                                       double2 *__restrict__ Tt, double2 *__restrict__ Tneg)
{
    const int job = blockIdx.x;
    const int n = jobs.n[job];
    const int64_t off = jobs.off[job];
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        const int i = idx % n, j = idx / n;
        const double2 u = U[off + idx];
        const double2 ut = U[off + j + (int64_t)n * i];
        Uh[off + idx] = cconj(ut);
        U32[off + idx] = make_float2((float)u.x, (float)u.y);
        Uh32[off + idx] = make_float2((float)ut.x, (float)-ut.y);
        Tt[off + idx] = T[off + j + (int64_t)n * i];
        const double2 tv = T[off + idx];
        Tneg[off + idx] = make_double2(-tv.x, -tv.y);
    }
}

}  // namespace

hipError_t launch_schur(const sylt_plan_s &p, int max_iter_per_n, hipStream_t s)
{
    // two launches: extents up to kSchurLdsMax in LDS, larger ones in the
    // plan's work buffer (3 mtotal entries; H and U take two of them)
    SchurJobs small{}, big{};
    int nsmall = 1, nbig = 1;
    for (int k = 0; k < p.N; ++k) {  // singleton modes give U = 1, T = A
        const int n = (int)p.n[k];
        const bool lds = n <= kSchurLdsMax;
        SchurJobs &j = lds ? small : big;
        j.n[j.count] = n;
        j.mode[j.count] = k;
        j.off[j.count] = p.moff[k];
        ++j.count;
        int &nmax = lds ? nsmall : nbig;
        nmax = std::max(nmax, n);
    }
    if (small.count > 0) {
        const size_t lds =
            (size_t)(2 * nsmall * nsmall + 2 * nsmall) * sizeof(double2) + nsmall * sizeof(double);
        hipError_t e = hipFuncSetAttribute((const void *)schur_kernel<64, false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((schur_kernel<64, false>), dim3(small.count), dim3(64), lds, s, small,
                           p.dA, p.dU, p.dT, p.dStatus, max_iter_per_n, p.dEw, p.mtotal);
    }
    if (big.count > 0) {
        // v, the rotation sines and cosines, four broadcast slots (aligned)
        // and the deflation maximum
        const size_t lds = (size_t)(2 * nbig + 7) * sizeof(double2) + nbig * sizeof(double);
        hipLaunchKernelGGL((schur_kernel<256, true>), dim3(big.count), dim3(256), lds, s, big, p.dA,
                           p.dU, p.dT, p.dStatus, max_iter_per_n, p.dEw, p.mtotal);
    }
    return hipGetLastError();
}

hipError_t launch_prepare_factors(const sylt_plan_s &p, hipStream_t s)
{
    PrepJobs jobs{};
    for (int k = 0; k < p.N; ++k) {
        jobs.n[jobs.count] = (int)p.n[k];
        jobs.off[jobs.count] = p.moff[k];
        ++jobs.count;
    }
    hipLaunchKernelGGL(prepare_factors_kernel, dim3(jobs.count), dim3(256), 0, s, jobs, p.dU,
                       p.dUh, p.dU32, p.dUh32, p.dT, p.dTt, p.dTneg);
    return hipGetLastError();
}

}  // namespace sylt
