/*
 * sylt_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU reference for the Schur
 * (Bartels-Stewart) solver of the N-dimensional Sylvester tensor equation
 *
 *     sum_j A_j []_j X = B          (Section 1, eq. e:sylvesterND)
 *
 * of Cuesta & de la Hoz, "A Non-Recursive, Dimension-Independent
 * Schur-Decomposition Algorithm for N-Dimensional Sylvester Tensor Equations"
 * (arXiv 2412.15840).  Only tests/, the smoke check and the benchmark's
 * cpu_baseline leg may load this library; the product path never does.
 * It shares no code with the HIP library.
 *
 * Conventions.  Tensors are flat arrays in column-major order: element
 * (i_1..i_N), 0-based, sits at sum_j i_j * prod_{l<j} n_l  (Section 2.2,
 * eq. e:index, shifted to 0-based).  Complex numbers are C99 double complex
 * (the same bytes as interleaved (re, im) doubles).  Matrices are n x n
 * column-major: M(i, m) = M[i + n*m].
 *
 * Nothing here is blocked, fused or reordered beyond what the paper states:
 * the mode products are the definition of []_j written as loops, the sweep is
 * Algorithm 3's single loop with the mixed-radix counter of Algorithm 2.
 */
#include <complex.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define MAT(M, n, i, m) ((M)[(int64_t)(i) + (int64_t)(n) * (int64_t)(m)])

static int64_t prod_range(const int64_t *n, int lo, int hi)
{
    int64_t p = 1;
    for (int j = lo; j < hi; ++j) p *= n[j];
    return p;
}

int64_t ora_numel(int N, const int64_t *n) { return prod_range(n, 0, N); }

/* OpenMP threads the parallel loops of this library use. */
int ora_num_threads(void) { return omp_get_max_threads(); }

/*
 * Mode product along mode k (0-based), in place:
 *     X <- M []_k X,   [M []_k X]_{..i_k..} = sum_m M(i_k, m) x_{..m..}
 * (definition of []_j, Section 1).  With adjoint != 0 the matrix used is M^*,
 * i.e. entry (i, m) is conj(M(m, i)); this is the U_j^* []_j of eq.
 * e:CUNU2U1B.  The tensor is viewed as (L, n_k, R) with L = prod_{j<k} n_j and
 * R = prod_{j>k} n_j; every fibre (l, r) is gathered, multiplied and scattered.
 * Only fibres f = l + L*r with f in [f_begin, f_end) are processed (the whole
 * tensor for [0, L*R)); this lets the benchmark time a bounded sample.
 */
void ora_mode_product_range(int N, const int64_t *n, int k, const cplx *M,
                            int adjoint, cplx *X, int64_t f_begin, int64_t f_end)
{
    const int64_t L = prod_range(n, 0, k);
    const int64_t nk = n[k];
    const int64_t R = prod_range(n, k + 1, N);
    if (f_end > L * R) f_end = L * R;
#pragma omp parallel
    {
        cplx *in = (cplx *)malloc(sizeof(cplx) * (size_t)nk);
        cplx *out = (cplx *)malloc(sizeof(cplx) * (size_t)nk);
#pragma omp for schedule(static)
        for (int64_t f = f_begin; f < f_end; ++f) {
            const int64_t l = f % L, r = f / L;
            cplx *base = X + l + L * nk * r;
            for (int64_t m = 0; m < nk; ++m) in[m] = base[L * m];
            for (int64_t i = 0; i < nk; ++i) {
                cplx acc = 0;
                for (int64_t m = 0; m < nk; ++m) {
                    cplx a = adjoint ? conj(MAT(M, nk, m, i)) : MAT(M, nk, i, m);
                    acc += a * in[m];
                }
                out[i] = acc;
            }
            for (int64_t i = 0; i < nk; ++i) base[L * i] = out[i];
        }
        free(in);
        free(out);
    }
}

void ora_mode_product(int N, const int64_t *n, int k, const cplx *M, int adjoint, cplx *X)
{
    ora_mode_product_range(N, n, k, M, adjoint, X, 0,
                           prod_range(n, 0, k) * prod_range(n, k + 1, N));
}

/*
 * Forward chain C = U_N^* []_N ( ... (U_1^* []_1 B)) (eq. e:CUNU2U1B) when
 * adjoint != 0, and the backward chain X = U_N []_N ( ... (U_1 []_1 Y))
 * (eq. e:XUNU2U1Y) when adjoint == 0.  In place.
 */
void ora_transform(int N, const int64_t *n, const cplx *const *U, int adjoint, cplx *X)
{
    for (int j = 0; j < N; ++j) ora_mode_product(N, n, j, U[j], adjoint, X);
}

/*
 * The sweep of Algorithm 3: solves sum_j T_j []_j Y = C (eq. e:TjYC) in
 * place, entry by entry with eq. e:yi1i2iN,
 *   y_i = (c_i - sum_j sum_{k > i_j} t_{j, i_j k} y_{i | i_j -> k}) / sum_j t_{j, i_j i_j},
 * visiting the linear index from n_1...n_N - 1 down to 0 while the tuple
 * (i_1..i_N) follows the mixed-radix counter of Algorithm 2: the first
 * component that is > 0 is decremented and every component before it is reset
 * to n - 1.  The neighbour y_{i | i_j -> i_j + q} sits at index + q*stride_j
 * (Section 4).  Only the first `max_entries` entries of that order are solved
 * when max_entries >= 0 (a bounded sample for timing); -1 means all.
 * Returns the number of inner-loop multiply-subtract steps performed.
 */
int64_t ora_sweep_upper(int N, const int64_t *n, const cplx *const *T, cplx *CY,
                        int64_t max_entries)
{
    int64_t stride[64], ii[64];
    if (N > 64) return -1;
    stride[0] = 1;
    for (int j = 1; j < N; ++j) stride[j] = stride[j - 1] * n[j - 1];
    for (int j = 0; j < N; ++j) ii[j] = n[j] - 1;
    const int64_t ntot = prod_range(n, 0, N);
    int64_t steps = 0, done = 0;
    for (int64_t index = ntot - 1; index >= 0; --index) {
        if (max_entries >= 0 && done >= max_entries) break;
        cplx num = CY[index];
        cplx den = 0;
        for (int j = 0; j < N; ++j) {
            const cplx *Tj = T[j];
            den += MAT(Tj, n[j], ii[j], ii[j]);
            for (int64_t q = 1; q <= n[j] - 1 - ii[j]; ++q) {
                num -= CY[index + q * stride[j]] * MAT(Tj, n[j], ii[j], ii[j] + q);
                ++steps;
            }
        }
        CY[index] = num / den;
        ++done;
        for (int k = 0; k < N; ++k) {
            if (ii[k] > 0) { ii[k] -= 1; break; }
            ii[k] = n[k] - 1;
        }
    }
    return steps;
}

/*
 * Adjoint sweep: solves sum_j T_j^* []_j Y = C in place.  T_j^* is lower
 * triangular with (T_j^*)(i, k) = conj(t_{j, k i}), so eq. e:yi1i2iN becomes
 *   y_i = (c_i - sum_j sum_{k < i_j} conj(t_{j, k i_j}) y_{i | i_j -> k}) / sum_j conj(t_{j, i_j i_j})
 * and the dependencies point to smaller indices: the single loop runs the
 * linear index upward with the mixed-radix counter incremented instead of
 * decremented (the mirror image of Algorithm 2).  Returns the step count.
 */
int64_t ora_sweep_adjoint(int N, const int64_t *n, const cplx *const *T, cplx *CY)
{
    int64_t stride[64], ii[64];
    if (N > 64) return -1;
    stride[0] = 1;
    for (int j = 1; j < N; ++j) stride[j] = stride[j - 1] * n[j - 1];
    for (int j = 0; j < N; ++j) ii[j] = 0;
    const int64_t ntot = prod_range(n, 0, N);
    int64_t steps = 0;
    for (int64_t index = 0; index < ntot; ++index) {
        cplx num = CY[index];
        cplx den = 0;
        for (int j = 0; j < N; ++j) {
            const cplx *Tj = T[j];
            den += conj(MAT(Tj, n[j], ii[j], ii[j]));
            for (int64_t q = 1; q <= ii[j]; ++q) {
                num -= CY[index - q * stride[j]] * conj(MAT(Tj, n[j], ii[j] - q, ii[j]));
                ++steps;
            }
        }
        CY[index] = num / den;
        for (int k = 0; k < N; ++k) {
            if (ii[k] < n[k] - 1) { ii[k] += 1; break; }
            ii[k] = 0;
        }
    }
    return steps;
}

/*
 * Records the order in which Algorithm 2 generates the tuples: out_index[t]
 * is the 1-based linear index of eq. e:index and out_tuple[t*N + j] the
 * 1-based component i_j of the t-th tuple (t < count).  Used to check the
 * counter against the worked example printed in Section 2.2.
 */
void ora_counter_trace(int N, const int64_t *n, int64_t count, int64_t *out_index,
                       int64_t *out_tuple)
{
    int64_t ii[64];
    for (int j = 0; j < N; ++j) ii[j] = n[j];
    int64_t index = prod_range(n, 0, N);
    for (int64_t t = 0; t < count && index >= 1; ++t, --index) {
        out_index[t] = index;
        for (int j = 0; j < N; ++j) out_tuple[t * N + j] = ii[j];
        for (int k = 0; k < N; ++k) {
            if (ii[k] > 1) { ii[k] -= 1; break; }
            ii[k] = n[k];
        }
    }
}

/*
 * Kronecker-sum apply  Y = sum_j A_j []_j X  (the operator of eq.
 * e:sylvesterND / e:systvec), written straight from the definition of []_j:
 * for each entry, sum over the modes and over the fibre through it.
 */
void ora_apply(int N, const int64_t *n, const cplx *const *A, const cplx *X, cplx *Y)
{
    int64_t stride[64];
    stride[0] = 1;
    for (int j = 1; j < N; ++j) stride[j] = stride[j - 1] * n[j - 1];
    const int64_t ntot = prod_range(n, 0, N);
#pragma omp parallel for schedule(static)
    for (int64_t index = 0; index < ntot; ++index) {
        cplx acc = 0;
        int64_t rem = index;
        for (int j = 0; j < N; ++j) {
            const int64_t ij = rem % n[j];
            rem /= n[j];
            const int64_t base = index - ij * stride[j];
            for (int64_t m = 0; m < n[j]; ++m)
                acc += MAT(A[j], n[j], ij, m) * X[base + m * stride[j]];
        }
        Y[index] = acc;
    }
}

/*
 * Same operator with every A_j replaced by A_j^* (the adjoint operator
 * sum_j A_j^* []_j, whose inverse gives the gradient with respect to B).
 */
void ora_apply_adjoint(int N, const int64_t *n, const cplx *const *A, const cplx *X, cplx *Y)
{
    int64_t stride[64];
    stride[0] = 1;
    for (int j = 1; j < N; ++j) stride[j] = stride[j - 1] * n[j - 1];
    const int64_t ntot = prod_range(n, 0, N);
#pragma omp parallel for schedule(static)
    for (int64_t index = 0; index < ntot; ++index) {
        cplx acc = 0;
        int64_t rem = index;
        for (int j = 0; j < N; ++j) {
            const int64_t ij = rem % n[j];
            rem /= n[j];
            const int64_t base = index - ij * stride[j];
            for (int64_t m = 0; m < n[j]; ++m)
                acc += conj(MAT(A[j], n[j], m, ij)) * X[base + m * stride[j]];
        }
        Y[index] = acc;
    }
}

/*
 * Algorithm 3 given the Schur factors A_j = U_j T_j U_j^* (Section 2):
 * X <- B; X <- U_j^* []_j X for every j; sweep; X <- U_j []_j X for every j.
 * In place on X (which holds B on entry), as the paper stores B, C, Y and X
 * in one array.
 */
int64_t ora_solve_factored(int N, const int64_t *n, const cplx *const *U,
                           const cplx *const *T, cplx *X)
{
    ora_transform(N, n, U, 1, X);
    int64_t steps = ora_sweep_upper(N, n, T, X, -1);
    ora_transform(N, n, U, 0, X);
    return steps;
}

/*
 * Solution of the adjoint equation sum_j A_j^* []_j G = W with the same
 * factors: A_j^* = U_j T_j^* U_j^*, so G = U-chain(adjoint sweep(U^*-chain(W))).
 */
int64_t ora_solve_adjoint_factored(int N, const int64_t *n, const cplx *const *U,
                                   const cplx *const *T, cplx *G)
{
    ora_transform(N, n, U, 1, G);
    int64_t steps = ora_sweep_adjoint(N, n, T, G);
    ora_transform(N, n, U, 0, G);
    return steps;
}

/*
 * Gradient of L with respect to A_k (0-based k), given G = dL/dB (the adjoint
 * solution) and the solution X:  out(a, m) = - sum over all entries with
 * i_k = a of G_i * conj(X_{i | i_k -> m}).  Derivation: dX = -A^{-1}(dA_k []_k X),
 * so dL = -Re<G, dA_k []_k X>.  out is n_k x n_k column-major.
 */
void ora_grad_A(int N, const int64_t *n, int k, const cplx *G, const cplx *X, cplx *out)
{
    const int64_t L = prod_range(n, 0, k);
    const int64_t nk = n[k];
    const int64_t R = prod_range(n, k + 1, N);
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t a = 0; a < nk; ++a) {
        for (int64_t m = 0; m < nk; ++m) {
            cplx acc = 0;
            for (int64_t r = 0; r < R; ++r)
                for (int64_t l = 0; l < L; ++l)
                    acc += G[l + L * (a + nk * r)] * conj(X[l + L * (m + nk * r)]);
            MAT(out, nk, a, m) = -acc;
        }
    }
}

/*
 * Eigenvalue-sum separation min_i |sum_j lambda_{j, i_j}| by brute force over
 * every multi-index (the solvability condition of Section 2: a solution exists
 * and is unique iff every such sum is nonzero).  lam[j] holds n[j] values.
 */
double ora_separation(int N, const int64_t *n, const cplx *const *lam)
{
    const int64_t ntot = prod_range(n, 0, N);
    double best = 1e308;
#pragma omp parallel for reduction(min : best) schedule(static)
    for (int64_t index = 0; index < ntot; ++index) {
        int64_t rem = index;
        cplx s = 0;
        for (int j = 0; j < N; ++j) {
            s += lam[j][rem % n[j]];
            rem /= n[j];
        }
        double a = cabs(s);
        if (a < best) best = a;
    }
    return best;
}
