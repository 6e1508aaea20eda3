// Internal declarations of libsylt (gfx950): complex arithmetic helpers, the
// plan object and the launch helpers each kernel file exports to the API layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sylt.h"

namespace sylt {

constexpr int kMaxModes = 32;     // N limit of the ABI
constexpr int kMaxExtent = 256;   // n_k limit of the ABI
constexpr int kSchurLdsMax = 64;  // Schur factors with H and U in LDS up to this extent
constexpr int kMaxGroup = 24;     // modes fused in one transform pass (n >= 2 each)
constexpr int kSweepTileCap = 9728;   // sweep tile entries (with diagonal blocks <= 160 KB LDS)
constexpr int kSweepThreads = 1024;   // lanes of a sweep workgroup
constexpr int kSweepMaxRounds = 32;   // local-solve rounds held per lane in registers
constexpr int kSweepPencilMax = 20;   // longest mode-0 pencil held in one lane's registers
constexpr int kSweepPencilModes = 8;  // most tiled modes of the pencil form
constexpr int kResidualMfmaCap = 4096;  // tile entries of the matrix-core residual pass
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;  // fixed device scratch per device
constexpr int kMaxAbsBlocks = 4096;  // partial maxima of the max-abs reduction

// ----------------------------------------------------------------- complex
// double2 / float2 hold (re, im).  All products are written as explicit fused
// multiply-adds so the rounding is the same in every kernel.
__host__ __device__ inline double2 cd(double re, double im) { return make_double2(re, im); }

template <typename V> struct CTraits;
template <> struct CTraits<double2> { using R = double; };
template <> struct CTraits<float2> { using R = float; };

// acc + a * b
template <typename V>
__device__ __forceinline__ V cmac(V acc, V a, V b)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
// acc + conj(a) * b
template <typename V>
__device__ __forceinline__ V cmac_conj(V acc, V a, V b)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
// acc - a * b and acc - conj(a) * b as four fused multiply-adds
__device__ __forceinline__ double2 cmsub(double2 acc, double2 a, double2 b)
{
    acc.x = fma(-a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(-a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
__device__ __forceinline__ double2 cmsub_conj(double2 acc, double2 a, double2 b)
{
    acc.x = fma(-a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(-a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double cabs1(double2 a) { return fabs(a.x) + fabs(a.y); }
__host__ __device__ inline double cabs2(double2 a) { return hypot(a.x, a.y); }
__host__ __device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// a / b by Smith's algorithm (R. L. Smith, CACM 5(8), 1962): scale by the
// larger component of b to avoid overflow in |b|^2.
__host__ __device__ inline double2 cdiv(double2 a, double2 b)
{
    if (fabs(b.x) >= fabs(b.y)) {
        const double r = b.y / b.x;
        const double den = b.x + b.y * r;
        return make_double2((a.x + a.y * r) / den, (a.y - a.x * r) / den);
    }
    const double r = b.x / b.y;
    const double den = b.x * r + b.y;
    return make_double2((a.x * r + a.y) / den, (a.y * r - a.x) / den);
}

// a / b with one division: b is scaled by an exact power of two 2^-e that
// brings its larger component into [1/2, 1), then a / b = (a conj(b') / |b'|^2) 2^-e.
__device__ inline double2 cdiv_scaled(double2 a, double2 b)
{
    int e;
    frexp(fmax(fabs(b.x), fabs(b.y)), &e);
    const double bx = ldexp(b.x, -e), by = ldexp(b.y, -e);
    const double inv = 1.0 / fma(bx, bx, by * by);
    const double px = fma(a.x, bx, a.y * by), py = fma(a.y, bx, -(a.x * by));
    return make_double2(ldexp(px * inv, -e), ldexp(py * inv, -e));
}

// principal square root: for z = x + iy with t = sqrt((|z| + |x|)/2),
// sqrt(z) = (t, y/(2t)) when x >= 0 and (|y|/(2t), sign(y) t) otherwise.
__host__ __device__ inline double2 csqrt_(double2 z)
{
    if (z.x == 0.0 && z.y == 0.0) return make_double2(0.0, 0.0);
    const double t = sqrt(0.5 * (hypot(z.x, z.y) + fabs(z.x)));
    if (z.x >= 0.0) return make_double2(t, z.y / (2.0 * t));
    return make_double2(fabs(z.y) / (2.0 * t), copysign(t, z.y));
}

template <typename V> __device__ __forceinline__ double2 to_d2(V v);
template <> __device__ __forceinline__ double2 to_d2<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ double2 to_d2<float2>(float2 v) { return make_double2(v.x, v.y); }
template <typename V> __device__ __forceinline__ V from_d2(double2 v);
template <> __device__ __forceinline__ double2 from_d2<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 from_d2<float2>(double2 v)
{
    return make_float2((float)v.x, (float)v.y);
}

// ------------------------------------------------------ transform passes
// A pass applies the mode products of a run of consecutive (non-singleton)
// modes [a, b) to the tensor viewed as (Lin, G, Rout): Lin = product of the
// extents below a, G = product of the group's extents, Rout = the rest.  One
// workgroup owns a tile of lb x G x rb entries held in LDS.
struct PassDesc {
    int64_t Lin, G, Rout;
    int lb, lbshift, rb;
    int64_t ntl, ntr;       // tile counts along l and r
    int ng;                 // modes in the group
    int gd[kMaxGroup];      // extents
    int gs[kMaxGroup];      // in-group strides
    int64_t moff[kMaxGroup];  // offset of each member's matrix in the plan buffers
    int uniform_n;          // common extent if all equal (else 0)
    int maxn;               // largest extent in the group
    size_t lds_bytes(size_t elem) const { return (size_t)lb * (size_t)G * (size_t)rb * elem; }
};

// ------------------------------------------------------------------ sweep
struct SweepDesc {
    int M;                       // compressed modes
    int d[kMaxModes];
    int64_t s[kMaxModes];        // global strides
    int b[kMaxModes], nb[kMaxModes];
    int ls[kMaxModes];           // local strides in the full tile
    int bitoff[kMaxModes], bitw[kMaxModes];
    int tdoff[kMaxModes];        // offsets of diagonal blocks in LDS (entries)
    int64_t moff[kMaxModes];     // offsets of T_j in the plan's matrix buffer
    int S;                       // entries of a full tile
    int nll;                     // local levels
    int tdiag;                   // total entries of the diagonal blocks
    int packed;                  // local-solve work in the per-lane packed table
    int penc;                    // local solve by mode-0 pencils, one per lane (the
                                 // table then holds one pencil per lane)
    int pen_long;                // some other mode has a block longer than 3
    int zero_slot;               // LDS entry (after the diagonal blocks) that holds 0
    int rounds;                  // rounds of that table (levels wider than the
                                 // workgroup take several rounds)
    int round_level[kSweepMaxRounds];  // local level of each round, ascending
    int nsing;                   // singleton modes: their scalars join every eigenvalue sum
    int64_t singoff[kMaxModes];  // offsets of those 1x1 T_k in the matrix buffer
    int csoff[kMaxModes];        // offset of mode j's cross-section table (entries)
};

struct SweepPlan {
    SweepDesc desc{};
    SweepDesc *d_desc = nullptr;     // device copy of desc
    std::vector<int64_t> level_off;  // tile-level offsets into tiles (size nlev + 1)
    int *d_tiles = nullptr;          // tile ids sorted by tile level
    int64_t *d_goff = nullptr;       // global offset of each local entry
    uint64_t *d_code = nullptr;      // packed local coordinates
    int *d_llist = nullptr;          // local entries sorted by local level
    int *d_lloff = nullptr;          // local level offsets
    int *d_lanetab = nullptr;        // [round][lane] packed local-solve work items
    int *d_cst = nullptr;            // per mode: cross-section position -> local entry at loc_j = 0
    void *arena = nullptr;           // the one device allocation holding the tables above
    size_t lds_bytes = 0;
};

}  // namespace sylt

// ------------------------------------------------------------------- plan
struct sylt_plan_s {
    int device = 0;
    int N = 0;
    std::vector<int64_t> n;          // extents as given
    int64_t ntot = 0;
    // compressed view: the modes with n_k > 1
    int M = 0;
    std::vector<int> cmode;          // compressed -> original mode
    std::vector<int> cdim;
    std::vector<int64_t> cstride;
    // per original mode: offset (in complex entries) of its n_k x n_k matrix
    std::vector<int64_t> moff;
    int64_t mtotal = 0;
    bool has_A = false;
    // device buffers (complex128 unless noted)
    double2 *dA = nullptr;           // A_k
    double2 *dU = nullptr;           // U_k
    double2 *dUh = nullptr;          // U_k^* (conjugate transpose), column-major
    double2 *dT = nullptr;           // T_k
    double2 *dTt = nullptr;          // T_k^T (rows of T_k contiguous)
    double2 *dTneg = nullptr;        // -T_k
    double2 *dE = nullptr;           // exp(t T_k) of the last evolution
    double2 *dEw = nullptr;          // three work matrices per mode for exp(t T_k)
    double2 *dEvo = nullptr;         // four device scalars of the last evolution
    float2 *dU32 = nullptr;          // complex64 copies
    float2 *dUh32 = nullptr;
    int *dStatus = nullptr;          // per-mode Schur status
    double *dScratch = nullptr;      // small reduction scratch (plan-owned)
    void *arena = nullptr;           // the one device allocation holding the buffers above
    size_t scratch_bytes = 0;
    double sep = 0.0;
    std::vector<sylt::PassDesc> passes;   // transform passes (one LDS tile)
    std::vector<sylt::PassDesc> rpasses;  // residual passes (two LDS tiles)
    std::vector<sylt::PassDesc> mrpasses; // residual passes of the matrix-core kernel
    bool residual_mfma = false;           // every residual pass runs on the matrix cores
    sylt::SweepPlan sweep;
    // every T_k diagonal (all A_k normal, Remark 1): the sweep is the Hadamard
    // product Y = Lambda o C, with the eigenvalue sum of entry p read from two
    // tables of partial sums, dslo[p % dlo] (the low modes and the singleton
    // scalars) + dshi[p / dlo] (the other modes)
    bool diagT = false;
    int dsplit = 0;                  // compressed modes of the low table
    int64_t dlo = 1, dhi = 1;        // entries of the two tables
    double2 *dslo = nullptr, *dshi = nullptr;
};

namespace sylt {

// launch helpers implemented in the kernel files -----------------------------
hipError_t launch_schur(const sylt_plan_s &p, int max_iter_per_n, hipStream_t s);
hipError_t launch_prepare_factors(const sylt_plan_s &p, hipStream_t s);
hipError_t launch_separation(const sylt_plan_s &p, double *d_out, hipStream_t s);
hipError_t launch_transform(const sylt_plan_s &p, int dir, int precision, void *X, hipStream_t s);
// FP64 chain whose first pass reads src and writes X (out of place; later
// passes in place): the copy of src into X is folded into the first pass
hipError_t launch_transform_from(const sylt_plan_s &p, int dir, const double2 *src, double2 *X,
                                 hipStream_t s);
hipError_t launch_sweep(const sylt_plan_s &p, int op, int precision, void *X, hipStream_t s);
// the two partial-sum tables of the diagonal sweep (p.dslo, p.dshi)
hipError_t launch_diag_tables(const sylt_plan_s &p, hipStream_t s);
// R64 (complex128, may alias B) = B - sum_k A_k x_k X; if R32 != nullptr the
// final pass also stores r32_scale R (a power of two) as complex64.  Partial
// sums of |R|^2 and |B|^2 (unscaled) are reduced into norms2_dev[0..1] (device).
hipError_t launch_residual(const sylt_plan_s &p, const double2 *B, const double2 *X, double2 *R64,
                           float2 *R32, double *norms2_dev, hipStream_t s, double r32_scale = 1.0);
// the same with the matrices M_k of Mbuf (offsets p.moff) in place of A_k
// passes of the residual as launched (matrix-core or VALU list)
inline size_t residual_pass_count(const sylt_plan_s &p)
{
    return p.residual_mfma ? p.mrpasses.size() : p.rpasses.size();
}
// LDS bytes of the matrix-core residual pass (two tiles and the A fragments)
size_t residual_mfma_lds(const PassDesc &pa);
hipError_t launch_residual_with(const sylt_plan_s &p, const double2 *Mbuf, const double2 *B,
                                const double2 *X, double2 *R64, float2 *R32, double *norms2_dev,
                                hipStream_t s, double r32_scale = 1.0);
// chain of mode products with the matrices of M (offsets p.moff; singleton modes skipped)
hipError_t launch_transform_with(const sylt_plan_s &p, const double2 *M, double2 *X, hipStream_t s);
// E_k = exp(t T_k) for every mode into p.dE, and p.dEvo = {prod of the
// singleton modes' exp(t a_k), -1, 1, sum of the singleton modes' a_k}
hipError_t launch_expm(const sylt_plan_s &p, double t, hipStream_t s);
// out = c[0] x + c[1] y with device scalars c (out may alias x or y)
hipError_t launch_lincomb(double2 *out, const double2 *x, const double2 *y, const double2 *c,
                          int64_t n, hipStream_t s);
// X (+)= unscale D and out = complex64(scale in), unscale and scale powers of two
hipError_t launch_axpy_c64(double2 *X, const float2 *D, int64_t n, int assign, double unscale,
                           hipStream_t s);
hipError_t launch_convert_c128_c64(float2 *out, const double2 *in, int64_t n, double scale,
                                   hipStream_t s);
// *d_out = max over entries of max(|re|, |im|) (NaN if any entry is NaN);
// partial holds kMaxAbsBlocks doubles
hipError_t launch_max_abs_c128(const double2 *in, int64_t n, double *partial, double *d_out,
                               hipStream_t s);
hipError_t launch_copy_c128(double2 *out, const double2 *in, int64_t n, hipStream_t s);
hipError_t launch_grad_A(const sylt_plan_s &p, const double2 *G, const double2 *X, double2 *const *GA,
                         void *ws, size_t ws_bytes, hipStream_t s);
// device address and size of the library's fixed scratch on the current
// device (looked up once per device)
hipError_t noalloc_scratch(void **ptr, size_t *bytes);
size_t grad_A_workspace(const sylt_plan_s &p);

// planning (api.cpp)
void plan_passes(sylt_plan_s &p);
// block sizes of the sweep tiles: chosen by the cost model when force_b is
// null, else force_b[j] for every compressed mode j (validated)
int plan_sweep(sylt_plan_s &p, const int *force_b = nullptr);
void free_sweep_tables(SweepPlan &sp);
size_t max_lds_bytes();

}  // namespace sylt
