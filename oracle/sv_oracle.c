/*
 * FP64 reference state-vector simulator ("the oracle").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The HIP product
 * library never links, loads or calls it, and the two share no code.
 *
 * Everything here is the plain definition, written for a reader to check by
 * eye: no blocking, no fusion, no reordering of the arithmetic the definition
 * states.  Build with contraction off (-ffp-contract=off) so every product and
 * sum is a separately rounded IEEE double operation.
 *
 * Conventions: an n-qubit state is 2^n complex doubles stored as (re, im)
 * pairs (the layout of numpy complex128).  Qubit q is bit q of the index
 * (little-endian).  A k-target gate matrix U is 2^k x 2^k row-major; bit b of
 * its row/column index belongs to targets[b].  Controls act on |1>.
 */
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    double re, im;
} cplx;

static cplx c_mul(cplx a, cplx b)
{
    cplx r;
    r.re = a.re * b.re - a.im * b.im;
    r.im = a.re * b.im + a.im * b.re;
    return r;
}

static cplx c_add(cplx a, cplx b)
{
    cplx r;
    r.re = a.re + b.re;
    r.im = a.im + b.im;
    return r;
}

static cplx c_conj(cplx a)
{
    a.im = -a.im;
    return a;
}

/*
 * |psi> <- |0...0>.  The state vector holds 2^n amplitudes (paper Sec. 2.1,
 * "State-Vector Simulation").
 */
void orc_zero_state(cplx *a, int n)
{
    uint64_t N = (uint64_t)1 << n;
    for (uint64_t i = 0; i < N; ++i) {
        a[i].re = 0.0;
        a[i].im = 0.0;
    }
    a[0].re = 1.0;
}

/*
 * Apply a (possibly controlled) k-qubit unitary to the state.
 *
 * Paper Sec. 2.1, "State-Vector Simulation": a gate acts on the state through
 * the tensor product of its unitary with identities on the other qubits; a
 * one-qubit gate multiplies pairs of amplitudes by its 2x2 matrix.  Written
 * out: for every index `base` whose target bits are all 0 and whose control
 * bits are all 1, gather the 2^k amplitudes
 *     v[j] = a[base | sum_b bit_b(j) * 2^targets[b]],
 * and write back a[idx[r]] = sum_col U[r][col] * v[col] (ascending col).
 * Indices whose control bits are not all 1 are left untouched (controlled-U
 * = |1..1><1..1| (x) U + (I - |1..1><1..1|) (x) I).
 *
 * Returns 0, or -1 on an argument error (k outside 1..6, c outside 0..8, a
 * qubit out of range or repeated).
 */
int orc_apply(cplx *a, int n, const cplx *U, const int *targets, int k, const int *controls, int c)
{
    if (n < 1 || n > 40 || k < 1 || k > 6 || c < 0 || c > 8 || k + c > n)
        return -1;
    uint64_t used = 0, mt = 0, mc = 0;
    for (int b = 0; b < k; ++b) {
        if (targets[b] < 0 || targets[b] >= n || (used >> targets[b]) & 1)
            return -1;
        used |= (uint64_t)1 << targets[b];
        mt |= (uint64_t)1 << targets[b];
    }
    for (int j = 0; j < c; ++j) {
        if (controls[j] < 0 || controls[j] >= n || (used >> controls[j]) & 1)
            return -1;
        used |= (uint64_t)1 << controls[j];
        mc |= (uint64_t)1 << controls[j];
    }
    const uint64_t N = (uint64_t)1 << n;
    const int d = 1 << k;

#pragma omp parallel for schedule(static)
    for (int64_t sbase = 0; sbase < (int64_t)N; ++sbase) {
        uint64_t base = (uint64_t)sbase;
        if ((base & mt) != 0)
            continue;
        if ((base & mc) != mc)
            continue;
        uint64_t idx[64];
        cplx v[64];
        for (int j = 0; j < d; ++j) {
            uint64_t off = 0;
            for (int b = 0; b < k; ++b)
                if ((j >> b) & 1)
                    off |= (uint64_t)1 << targets[b];
            idx[j] = base | off;
            v[j] = a[idx[j]];
        }
        for (int r = 0; r < d; ++r) {
            cplx acc = {0.0, 0.0};
            for (int col = 0; col < d; ++col)
                acc = c_add(acc, c_mul(U[r * d + col], v[col]));
            a[idx[r]] = acc;
        }
    }
    return 0;
}

/*
 * Marginal probabilities over the qubits Q[0..m): out[x] = sum of |a_i|^2
 * over all i whose bit Q[b] equals bit b of x (paper Sec. 2.1, "Measurement
 * and Sampling": the distribution is fixed by the amplitudes).  m = n with
 * Q = (0..n-1) gives the full distribution; m = 0 gives the squared norm.
 * Sequential FP64 sums in ascending index order.
 */
int orc_probabilities(const cplx *a, int n, const int *Q, int m, double *out)
{
    if (m < 0 || m > n || m > 30)
        return -1;
    for (int b = 0; b < m; ++b)
        if (Q[b] < 0 || Q[b] >= n)
            return -1;
    const uint64_t N = (uint64_t)1 << n;
    for (uint64_t x = 0; x < ((uint64_t)1 << m); ++x)
        out[x] = 0.0;
    for (uint64_t i = 0; i < N; ++i) {
        double p = a[i].re * a[i].re + a[i].im * a[i].im;
        uint64_t x = 0;
        for (int b = 0; b < m; ++b)
            x |= ((i >> Q[b]) & 1) << b;
        out[x] += p;
    }
    return 0;
}

/* <a|b> = sum_i conj(a_i) * b_i, sequential FP64 sum in ascending index order. */
void orc_inner(const cplx *a, const cplx *b, int n, double *out_re_im)
{
    const uint64_t N = (uint64_t)1 << n;
    cplx acc = {0.0, 0.0};
    for (uint64_t i = 0; i < N; ++i)
        acc = c_add(acc, c_mul(c_conj(a[i]), b[i]));
    out_re_im[0] = acc.re;
    out_re_im[1] = acc.im;
}

typedef struct {
    double t;
    int s;
} shot_key;

static int shot_cmp(const void *pa, const void *pb)
{
    const shot_key *x = (const shot_key *)pa, *y = (const shot_key *)pb;
    if (x->t < y->t)
        return -1;
    if (x->t > y->t)
        return 1;
    return x->s - y->s;
}

/*
 * Sampling (paper Sec. 2.1, "Measurement and Sampling"; shots of Sec. 2.2):
 * for each uniform u_s in [0, 1), the outcome is the smallest index i with
 * CDF(i) > u_s * norm, where CDF(i) = sum_{j<=i} |a_j|^2 accumulated
 * sequentially from j = 0 and norm = CDF(2^n - 1).  If rounding leaves no
 * such i, the outcome is the largest index of nonzero probability.
 * Shots are answered in one ascending walk over the CDF (queries sorted by
 * target); each answer is the same as a separate walk would give.
 */
int orc_sample(const cplx *a, int n, const double *u, int shots, int64_t *out)
{
    const uint64_t N = (uint64_t)1 << n;
    double norm = 0.0;
    uint64_t last_nz = 0;
    for (uint64_t i = 0; i < N; ++i) {
        double p = a[i].re * a[i].re + a[i].im * a[i].im;
        norm += p;
        if (p > 0.0)
            last_nz = i;
    }
    shot_key *keys = (shot_key *)malloc(sizeof(shot_key) * (size_t)(shots > 0 ? shots : 1));
    if (!keys)
        return -1;
    for (int s = 0; s < shots; ++s) {
        keys[s].t = u[s] * norm;
        keys[s].s = s;
    }
    qsort(keys, (size_t)shots, sizeof(shot_key), shot_cmp);
    int next = 0;
    double cdf = 0.0;
    for (uint64_t i = 0; i < N && next < shots; ++i) {
        cdf += a[i].re * a[i].re + a[i].im * a[i].im;
        while (next < shots && cdf > keys[next].t) {
            out[keys[next].s] = (int64_t)i;
            ++next;
        }
    }
    for (; next < shots; ++next)
        out[keys[next].s] = (int64_t)last_nz;
    free(keys);
    return 0;
}

/*
 * Qubit bit-field exchange: b[sigma(i)] = a[i], where sigma swaps index bits
 * [lo, lo+w) with [hi, hi+w) (the two fields must not overlap).  This is the
 * relayout a distributed simulator performs when it exchanges w global
 * (rank) bits with w local ones (paper Sec. 2.1 "State-Vector Simulation",
 * Sec. 2.5), done inside one memory domain.
 */
int orc_bitswap(const cplx *a, cplx *b, int n, int lo, int hi, int w)
{
    if (w < 1 || lo < 0 || hi < lo + w || hi + w > n)
        return -1;
    const uint64_t N = (uint64_t)1 << n;
    const uint64_t fmask = ((uint64_t)1 << w) - 1;
    for (uint64_t i = 0; i < N; ++i) {
        uint64_t flo = (i >> lo) & fmask;
        uint64_t fhi = (i >> hi) & fmask;
        uint64_t j = i & ~((fmask << lo) | (fmask << hi));
        j |= (flo << hi) | (fhi << lo);
        b[j] = a[i];
    }
    return 0;
}

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads the parallel loop of orc_apply uses (1 without OpenMP). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
