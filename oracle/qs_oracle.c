/*
 * qs_oracle.c -- plain, slow, obviously correct FP64 reference for state-vector gate application.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path links, loads or calls this file; only the tests,
 * the smoke check and the benchmark's CPU-baseline leg do. It shares no code, header or constant with the
 * GPU library.
 *
 * Every function applies one operation, unfused, exactly as the paper defines it (mpiQulacs, Sec. II-A):
 *   - the state is 2^n complex amplitudes, interleaved (re, im) doubles (Eq. 2; 2^(n+4) bytes);
 *   - qubit q is bit q of the amplitude index (Sec. II-A, Eq. 4; Sec. III-B: local qubits are the low
 *     index bits, global qubits the high ones);
 *   - a 1-qubit gate multiplies every amplitude pair whose indices differ only in bit q by U (Eq. 4); a
 *     k-qubit gate is the same rule on the 2^k amplitudes whose indices differ only in the target bits,
 *     with targets[j] <-> bit j of the matrix row/column index, row-major, psi' = U psi;
 *   - a diagonal gate multiplies amplitude i by d[a(i)], a(i) = the target bits of i;
 *   - a controlled gate is the dense rule restricted to indices whose control bits are all 1;
 *   - the fused-swap (Sec. III-D, Listing 1) is s successive swaps swap(p+j, q+j), j < s, with the two
 *     ranges [p, p+s) and [q, q+s) not overlapping; swap(a, b) exchanges the amplitudes of the two qubits;
 *   - probabilities are |a_i|^2 (Sec. II-A), the norm their sum with compensated (Kahan) summation.
 *
 * Products follow exact arithmetic in one respect: a matrix entry whose real or imaginary part is exactly
 * zero contributes nothing for that part (0*x = 0 exactly), and a sum starts from its first term rather than
 * from +0. Products by 0, +-1 and +-i are therefore exact moves, signed zeros included.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no FMA contraction, no hand SIMD).
 * Return codes: 0 ok, -1 invalid argument.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double re, im;
} cplx;

/* u * x with exact-zero parts of u skipped; *any is set when a term was produced. */
static cplx cmul_skip0(cplx u, cplx x, int *any)
{
    cplx r = {0.0, 0.0};
    int have = 0;
    if (u.re != 0.0) {
        r.re = u.re * x.re;
        r.im = u.re * x.im;
        have = 1;
    }
    if (u.im != 0.0) {
        double t_re = u.im * x.im;
        double t_im = u.im * x.re;
        if (have) {
            r.re = r.re - t_re;
            r.im = r.im + t_im;
        } else {
            r.re = -t_re;
            r.im = t_im;
            have = 1;
        }
    }
    *any = have;
    return r;
}

/* Index of the group member with target-bit pattern a, for a base index whose target bits are 0. */
static uint64_t with_pattern(uint64_t base, const int *t, int k, uint64_t a)
{
    uint64_t idx = base;
    for (int j = 0; j < k; j++)
        if ((a >> j) & 1u)
            idx |= (uint64_t)1 << t[j];
    return idx;
}

static int check_qubits(int n, const int *q, int cnt, uint64_t *mask)
{
    uint64_t m = 0;
    for (int j = 0; j < cnt; j++) {
        if (q[j] < 0 || q[j] >= n)
            return -1;
        uint64_t b = (uint64_t)1 << q[j];
        if (m & b)
            return -1;
        m |= b;
    }
    *mask = m;
    return 0;
}

void or_init_zero(double *psi, int n)
{
    uint64_t dim = (uint64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)(2 * dim); i++)
        psi[i] = 0.0;
    psi[0] = 1.0;
}

/* Dense k-qubit gate restricted to indices with (i & cmask) == cmask (cmask = 0: unrestricted). */
static int apply_matrix(double *psi, int n, const int *t, int k, uint64_t tmask, uint64_t cmask, const double *U)
{
    uint64_t dim = (uint64_t)1 << n;
    uint64_t K = (uint64_t)1 << k;
    const cplx *u = (const cplx *)U;
    cplx *st = (cplx *)psi;
    int err = 0;
#pragma omp parallel
    {
        cplx *in = (cplx *)malloc(K * sizeof(cplx));
        cplx *out = (cplx *)malloc(K * sizeof(cplx));
        uint64_t *idx = (uint64_t *)malloc(K * sizeof(uint64_t));
        if (!in || !out || !idx) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(static)
        for (int64_t i = 0; i < (int64_t)dim; i++) {
            if (!in || !out || !idx)
                continue;
            if ((uint64_t)i & tmask)
                continue; /* not a group base: some target bit is set */
            if (((uint64_t)i & cmask) != cmask)
                continue; /* a control bit is 0: amplitudes untouched */
            for (uint64_t a = 0; a < K; a++) {
                idx[a] = with_pattern((uint64_t)i, t, k, a);
                in[a] = st[idx[a]];
            }
            for (uint64_t a = 0; a < K; a++) {
                cplx acc = {0.0, 0.0};
                int started = 0;
                for (uint64_t b = 0; b < K; b++) {
                    int any;
                    cplx term = cmul_skip0(u[a * K + b], in[b], &any);
                    if (!any)
                        continue;
                    if (!started) {
                        acc = term;
                        started = 1;
                    } else {
                        acc.re = acc.re + term.re;
                        acc.im = acc.im + term.im;
                    }
                }
                out[a] = acc;
            }
            for (uint64_t a = 0; a < K; a++)
                st[idx[a]] = out[a];
        }
        free(in);
        free(out);
        free(idx);
    }
    return err;
}

int or_apply_dense(double *psi, int n, const int *targets, int k, const double *U)
{
    uint64_t tmask;
    if (!psi || !targets || !U || k < 1 || k > n || k > 12 || check_qubits(n, targets, k, &tmask))
        return -1;
    return apply_matrix(psi, n, targets, k, tmask, 0, U);
}

int or_apply_controlled(double *psi, int n, const int *controls, int c, const int *targets, int k, const double *U)
{
    uint64_t tmask, cmask;
    if (!psi || !targets || !controls || !U || k < 1 || c < 1 || c + k > n || k > 12)
        return -1;
    if (check_qubits(n, targets, k, &tmask) || check_qubits(n, controls, c, &cmask) || (tmask & cmask))
        return -1;
    return apply_matrix(psi, n, targets, k, tmask, cmask, U);
}

int or_apply_diag(double *psi, int n, const int *targets, int k, const double *d)
{
    uint64_t tmask;
    if (!psi || !targets || !d || k < 1 || k > n || k > 20 || check_qubits(n, targets, k, &tmask))
        return -1;
    uint64_t dim = (uint64_t)1 << n;
    const cplx *dd = (const cplx *)d;
    cplx *st = (cplx *)psi;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)dim; i++) {
        uint64_t a = 0;
        for (int j = 0; j < k; j++)
            a |= (((uint64_t)i >> targets[j]) & 1u) << j;
        int any;
        cplx r = cmul_skip0(dd[a], st[i], &any);
        if (!any)
            r.re = r.im = 0.0;
        st[i] = r;
    }
    return 0;
}

/* swap(a, b): exchange the amplitudes of qubits a and b, i.e. psi'[i] = psi[i with bits a and b exchanged]. */
int or_swap(double *psi, int n, int a, int b)
{
    if (!psi || a < 0 || b < 0 || a >= n || b >= n)
        return -1;
    if (a == b)
        return 0;
    uint64_t dim = (uint64_t)1 << n;
    uint64_t ba = (uint64_t)1 << a, bb = (uint64_t)1 << b;
    cplx *st = (cplx *)psi;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)dim; i++) {
        /* visit each exchanged pair once: from the member with bit a = 1 and bit b = 0 */
        if (((uint64_t)i & ba) && !((uint64_t)i & bb)) {
            uint64_t j = ((uint64_t)i ^ ba) | bb;
            cplx tmp = st[i];
            st[i] = st[j];
            st[j] = tmp;
        }
    }
    return 0;
}

/* fused_swap(p, q, s) as s successive swaps (Sec. III-D, Listing 1); the ranges may not overlap. */
int or_fused_swap(double *psi, int n, int p, int q, int s)
{
    if (!psi || s < 0 || p < 0 || q < 0)
        return -1;
    if (s == 0)
        return 0;
    if (p + s > n || q + s > n)
        return -1;
    int lo = p < q ? p : q, hi = p < q ? q : p;
    if (lo + s > hi)
        return -1; /* [p, p+s) and [q, q+s) overlap */
    for (int j = 0; j < s; j++)
        or_swap(psi, n, p + j, q + j);
    return 0;
}

/* out[i] = |psi_i|^2; *norm = sum_i out[i] (Kahan, index order). */
int or_probs(const double *psi, int n, double *out, double *norm)
{
    if (!psi || !out)
        return -1;
    uint64_t dim = (uint64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)dim; i++)
        out[i] = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
    if (norm) {
        double s = 0.0, c = 0.0;
        for (uint64_t i = 0; i < dim; i++) {
            double y = out[i] - c;
            double t = s + y;
            c = (t - s) - y;
            s = t;
        }
        *norm = s;
    }
    return 0;
}

/* psi *= f (f real). */
int or_scale(double *psi, int n, double f)
{
    if (!psi)
        return -1;
    uint64_t dim = (uint64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)(2 * dim); i++)
        psi[i] = psi[i] * f;
    return 0;
}
