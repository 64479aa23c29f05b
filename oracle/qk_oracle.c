/*
 * Plain FP64 state-vector oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  It shares no code with the GPU path.  It is deliberately
 * slow and obviously correct: every gate is applied by its definition, with
 * sequential index loops and index-order sums.
 *
 * What it computes (the paper's four commands: add qubits, gate operation,
 * measure, define gate as a matrix or a function; section "Q-Kit."):
 *   - a dense complex state psi of 2^n amplitudes, qubit q = bit q of the
 *     index; adding m qubits maps psi -> psi (x) |0..0>, the new qubits on the
 *     high bits, so old amplitudes keep their indices;
 *   - a gate with targets t_0..t_{k-1}, controls C and classical conditions
 *     (cbit, value): skipped unless every condition holds; otherwise for every
 *     index `base` with all target bits 0 and all control bits 1, the 2^k
 *     amplitudes psi[base | sum_j bit_j(m) 2^{t_j}] are multiplied by the
 *     2^k x 2^k matrix (row-major, row/column bit j <-> t_j), or moved by a
 *     permutation table f: the amplitude at m goes to f(m);
 *   - measurement of qubit q with a pre-drawn uniform u (the copy of the
 *     outcome into a classical bit is the paper's Copy command):
 *     p_b = sum of |psi_i|^2 over i with bit q = b, in index order;
 *     P0 = p0 / (p0 + p1); outcome o = (u < P0) ? 0 : 1; amplitudes with
 *     bit q = o are divided by sqrt(p_o), the others set to 0;
 *   - deferred measurement (shots drawn from the final state, which is left
 *     unchanged) and the marginal distribution of a list of qubits, from the
 *     running sum of |psi_i|^2 in index order.
 *
 * Build: gcc -O2 -shared -fPIC (single thread), or add -fopenmp to split the
 * gate loops over host threads (same code; measurement sums stay sequential).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

typedef struct orc {
    int n;              /* qubits */
    uint64_t dim;       /* 2^n */
    cplx* psi;
    int ncbits;
    unsigned char* cbits;
} orc;

enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_NOT_PERM = -3, ORC_E_OOM = -4, ORC_E_STATE = -6 };

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

orc* orc_new(void) {
    orc* o = (orc*)calloc(1, sizeof(orc));
    if (!o) return NULL;
    o->dim = 1;
    o->psi = (cplx*)malloc(sizeof(cplx));
    if (!o->psi) { free(o); return NULL; }
    o->psi[0] = 1.0;   /* zero qubits: the scalar 1 */
    return o;
}

void orc_free(orc* o) {
    if (!o) return;
    free(o->psi);
    free(o->cbits);
    free(o);
}

int orc_num_qubits(const orc* o) { return o->n; }

/* psi -> psi (x) |0^m>: new qubits take bits n..n+m-1. */
int orc_add_qubits(orc* o, int m) {
    if (m < 0 || o->n + m > 40) return ORC_E_ARG;
    uint64_t nd = o->dim << m;
    cplx* np = (cplx*)malloc(nd * sizeof(cplx));
    if (!np) return ORC_E_OOM;
    for (uint64_t i = 0; i < nd; ++i) np[i] = (i < o->dim) ? o->psi[i] : 0.0;
    free(o->psi);
    o->psi = np;
    o->dim = nd;
    o->n += m;
    return ORC_OK;
}

int orc_add_cbits(orc* o, int m) {
    if (m < 0) return ORC_E_ARG;
    unsigned char* nc = (unsigned char*)calloc((size_t)(o->ncbits + m) + 1, 1);
    if (!nc) return ORC_E_OOM;
    if (o->ncbits) memcpy(nc, o->cbits, (size_t)o->ncbits);
    free(o->cbits);
    o->cbits = nc;
    o->ncbits += m;
    return ORC_OK;
}

int orc_get_cbits(const orc* o, unsigned char* out, int n) {
    if (n > o->ncbits) return ORC_E_ARG;
    for (int i = 0; i < n; ++i) out[i] = o->cbits[i];
    return ORC_OK;
}

int orc_set_cbit(orc* o, int c, int v) {
    if (c < 0 || c >= o->ncbits) return ORC_E_ARG;
    o->cbits[c] = (unsigned char)(v != 0);
    return ORC_OK;
}

/* state as interleaved (re, im) doubles */
int orc_set_state(orc* o, const double* re_im, uint64_t dim) {
    if (dim != o->dim) return ORC_E_ARG;
    for (uint64_t i = 0; i < dim; ++i) o->psi[i] = re_im[2 * i] + I * re_im[2 * i + 1];
    return ORC_OK;
}

int orc_get_state(const orc* o, double* re_im, uint64_t dim) {
    if (dim != o->dim) return ORC_E_ARG;
    for (uint64_t i = 0; i < dim; ++i) {
        re_im[2 * i] = creal(o->psi[i]);
        re_im[2 * i + 1] = cimag(o->psi[i]);
    }
    return ORC_OK;
}

/* Shared argument check: indices in range, no qubit used twice. */
static int check_qubits(const orc* o, int k, const int* targets, int nc, const int* controls) {
    uint64_t seen = 0;
    for (int j = 0; j < k + nc; ++j) {
        int q = j < k ? targets[j] : controls[j - k];
        if (q < 0 || q >= o->n) return ORC_E_ARG;
        if (seen & (1ull << q)) return ORC_E_ARG;
        seen |= 1ull << q;
    }
    return ORC_OK;
}

/* Every condition (cbit, value) must hold for the gate to run. */
static int conditions_hold(const orc* o, int ncond, const int* cond_cbits, const int* cond_vals) {
    for (int i = 0; i < ncond; ++i)
        if ((int)o->cbits[cond_cbits[i]] != (cond_vals[i] != 0)) return 0;
    return 1;
}

static int check_conds(const orc* o, int ncond, const int* cond_cbits) {
    for (int i = 0; i < ncond; ++i)
        if (cond_cbits[i] < 0 || cond_cbits[i] >= o->ncbits) return ORC_E_ARG;
    return ORC_OK;
}

/* index of the amplitude in the group of `base` selected by gate index m */
static uint64_t group_index(uint64_t base, uint64_t m, int k, const int* targets) {
    uint64_t idx = base;
    for (int j = 0; j < k; ++j)
        if ((m >> j) & 1) idx |= 1ull << targets[j];
    return idx;
}

/* Matrix gate: m_re_im is 2^k x 2^k complex, row-major, interleaved. */
int orc_apply_matrix(orc* o, int k, const int* targets, const double* m_re_im,
                     int nc, const int* controls,
                     int ncond, const int* cond_cbits, const int* cond_vals) {
    if (k < 1 || k > 12) return ORC_E_ARG;
    int st = check_qubits(o, k, targets, nc, controls);
    if (st) return st;
    if ((st = check_conds(o, ncond, cond_cbits))) return st;
    if (!conditions_hold(o, ncond, cond_cbits, cond_vals)) return ORC_OK;
    const uint64_t K = 1ull << k;
    cplx* M = (cplx*)malloc(K * K * sizeof(cplx));
    if (!M) return ORC_E_OOM;
    for (uint64_t e = 0; e < K * K; ++e) M[e] = m_re_im[2 * e] + I * m_re_im[2 * e + 1];
    uint64_t tmask = 0, cmask = 0;
    for (int j = 0; j < k; ++j) tmask |= 1ull << targets[j];
    for (int j = 0; j < nc; ++j) cmask |= 1ull << controls[j];
    int oom = 0;
#pragma omp parallel
    {
        uint64_t* idx = (uint64_t*)malloc(K * sizeof(uint64_t));
        cplx* v = (cplx*)malloc(K * sizeof(cplx));
        if (!idx || !v) {
#pragma omp atomic write
            oom = 1;
        }
#pragma omp for schedule(static)
        for (uint64_t base = 0; base < o->dim; ++base) {
            if (!idx || !v) continue;
            if (base & tmask) continue;
            if ((base & cmask) != cmask) continue;
            for (uint64_t m = 0; m < K; ++m) {
                idx[m] = group_index(base, m, k, targets);
                v[m] = o->psi[idx[m]];
            }
            for (uint64_t r = 0; r < K; ++r) {
                cplx s = 0.0;
                for (uint64_t m = 0; m < K; ++m) s += M[r * K + m] * v[m];
                o->psi[idx[r]] = s;
            }
        }
        free(idx);
        free(v);
    }
    free(M);
    return oom ? ORC_E_OOM : ORC_OK;
}

/* Permutation gate: the amplitude at gate index m moves to gate index table[m]. */
int orc_apply_perm(orc* o, int k, const int* targets, const uint64_t* table,
                   int nc, const int* controls,
                   int ncond, const int* cond_cbits, const int* cond_vals) {
    if (k < 1 || k > 30) return ORC_E_ARG;
    int st = check_qubits(o, k, targets, nc, controls);
    if (st) return st;
    if ((st = check_conds(o, ncond, cond_cbits))) return st;
    const uint64_t K = 1ull << k;
    /* the table must be a bijection of [0, 2^k): every value in range, none twice */
    unsigned char* seen = (unsigned char*)calloc((size_t)((K + 7) / 8), 1);
    if (!seen) return ORC_E_OOM;
    for (uint64_t m = 0; m < K; ++m) {
        const uint64_t y = table[m];
        if (y >= K || (seen[y >> 3] >> (y & 7)) & 1) {
            free(seen);
            return ORC_E_NOT_PERM;
        }
        seen[y >> 3] |= (unsigned char)(1u << (y & 7));
    }
    free(seen);
    if (!conditions_hold(o, ncond, cond_cbits, cond_vals)) return ORC_OK;
    uint64_t tmask = 0, cmask = 0;
    for (int j = 0; j < k; ++j) tmask |= 1ull << targets[j];
    for (int j = 0; j < nc; ++j) cmask |= 1ull << controls[j];
    cplx* out = (cplx*)malloc(o->dim * sizeof(cplx));
    if (!out) return ORC_E_OOM;
    memcpy(out, o->psi, o->dim * sizeof(cplx));
#pragma omp parallel for schedule(static)
    for (uint64_t base = 0; base < o->dim; ++base) {
        if (base & tmask) continue;
        if ((base & cmask) != cmask) continue;
        for (uint64_t m = 0; m < K; ++m)
            out[group_index(base, table[m], k, targets)] = o->psi[group_index(base, m, k, targets)];
    }
    free(o->psi);
    o->psi = out;
    return ORC_OK;
}

/* p0, p1: index-order sums of |psi_i|^2 split by bit q. */
static void probabilities(const orc* o, int q, double* p0, double* p1) {
    double s0 = 0.0, s1 = 0.0;
    for (uint64_t i = 0; i < o->dim; ++i) {
        double a = creal(o->psi[i]) * creal(o->psi[i]) + cimag(o->psi[i]) * cimag(o->psi[i]);
        if ((i >> q) & 1) s1 += a; else s0 += a;
    }
    *p0 = s0;
    *p1 = s1;
}

static void collapse(orc* o, int q, int outcome, double p_o) {
    double s = 1.0 / sqrt(p_o);
    for (uint64_t i = 0; i < o->dim; ++i) {
        if ((int)((i >> q) & 1) == outcome) o->psi[i] *= s;
        else o->psi[i] = 0.0;
    }
}

/* Measure qubit q with uniform u; cbit < 0 means the outcome is not stored. */
int orc_measure(orc* o, int q, int cbit, double u, int* outcome, double* p0_out, double* p1_out) {
    if (q < 0 || q >= o->n || cbit >= o->ncbits) return ORC_E_ARG;
    double p0, p1;
    probabilities(o, q, &p0, &p1);
    double P0 = p0 / (p0 + p1);
    int oc = (u < P0) ? 0 : 1;
    double p_o = oc ? p1 : p0;
    if (!(p_o > 0.0)) return ORC_E_STATE;
    collapse(o, q, oc, p_o);
    if (cbit >= 0) o->cbits[cbit] = (unsigned char)oc;
    if (outcome) *outcome = oc;
    if (p0_out) *p0_out = p0;
    if (p1_out) *p1_out = p1;
    return ORC_OK;
}

/* Forced outcome (used to enumerate measurement branches exactly). */
int orc_postselect(orc* o, int q, int cbit, int outcome, double* prob_out) {
    if (q < 0 || q >= o->n || cbit >= o->ncbits || (outcome != 0 && outcome != 1)) return ORC_E_ARG;
    double p0, p1;
    probabilities(o, q, &p0, &p1);
    double p_o = outcome ? p1 : p0;
    if (prob_out) *prob_out = p_o / (p0 + p1);
    if (!(p_o > 0.0)) return ORC_E_STATE;
    collapse(o, q, outcome, p_o);
    if (cbit >= 0) o->cbits[cbit] = (unsigned char)outcome;
    return ORC_OK;
}

/* Deep copy, for branch enumeration. */
orc* orc_clone(const orc* o) {
    orc* c = (orc*)calloc(1, sizeof(orc));
    if (!c) return NULL;
    *c = *o;
    c->psi = (cplx*)malloc(o->dim * sizeof(cplx));
    c->cbits = (unsigned char*)calloc((size_t)o->ncbits + 1, 1);
    if (!c->psi || !c->cbits) { free(c->psi); free(c->cbits); free(c); return NULL; }
    memcpy(c->psi, o->psi, o->dim * sizeof(cplx));
    if (o->ncbits) memcpy(c->cbits, o->cbits, (size_t)o->ncbits);
    return c;
}

/* ---- deferred measurement: distribution and many-shot sampling ----------
 *
 * The paper's circuits end either in in-place measurement or in deferred
 * measurement of the qubits, and the state can be read out as a normalised
 * probability distribution (section "Q-Kit.").  Deferred measurement of a
 * list of qubits Q = (q_0..q_{m-1}) in one shot yields the bits of an index
 * i drawn with probability |psi_i|^2 / sum_j |psi_j|^2, read at Q; the state
 * is left as it is, so any number of shots can be drawn from it.
 */

/* Bits qubits[j] of i packed into bit j (nq = 0: i itself). */
static uint64_t project(uint64_t i, int nq, const int* qubits) {
    if (nq == 0) return i;
    uint64_t r = 0;
    for (int j = 0; j < nq; ++j) r |= ((i >> qubits[j]) & 1ull) << j;
    return r;
}

static int check_list(const orc* o, int nq, const int* qubits) {
    if (nq < 0 || nq > o->n || (nq > 0 && !qubits)) return ORC_E_ARG;
    for (int j = 0; j < nq; ++j) {
        if (qubits[j] < 0 || qubits[j] >= o->n) return ORC_E_ARG;
        for (int l = 0; l < j; ++l)
            if (qubits[l] == qubits[j]) return ORC_E_ARG;
    }
    return ORC_OK;
}

/* Marginal distribution of the listed qubits: out[m] = sum of |psi_i|^2 over
 * the i whose projection is m, summed in index order, divided by the total
 * (2^nq entries; not normalised when normalise == 0). */
int orc_marginal(const orc* o, int nq, const int* qubits, int normalise, double* out) {
    if (check_list(o, nq, qubits) || !out || o->n == 0) return ORC_E_ARG;
    uint64_t nout = 1ull << (nq ? nq : o->n);
    for (uint64_t m = 0; m < nout; ++m) out[m] = 0.0;
    double total = 0.0;
    for (uint64_t i = 0; i < o->dim; ++i) {
        double a = creal(o->psi[i]) * creal(o->psi[i]) + cimag(o->psi[i]) * cimag(o->psi[i]);
        out[project(i, nq, qubits)] += a;
        total += a;
    }
    if (normalise) {
        if (!(total > 0.0)) return ORC_E_STATE;
        for (uint64_t m = 0; m < nout; ++m) out[m] /= total;
    }
    return ORC_OK;
}

/* S shots: for each uniform u_s in [0,1), the smallest index i whose running
 * sum c_i = sum_{j<=i} |psi_j|^2 (index order) exceeds u_s * c_{dim-1};
 * out[s] = projection of i onto the listed qubits.  margin (optional) gets
 * min(u_s*T - c_{i-1}, c_i - u_s*T) / T with T = c_{dim-1} and c_{-1} = 0:
 * how far the draw lies from the nearer boundary of the interval it fell in. */
int orc_sample(const orc* o, int nq, const int* qubits, const double* u, int64_t S, uint64_t* out,
               double* margin) {
    if (check_list(o, nq, qubits) || S < 0 || (S > 0 && (!u || !out)) || o->n == 0) return ORC_E_ARG;
    double* c = (double*)malloc(o->dim * sizeof(double));
    if (!c) return ORC_E_OOM;
    double run = 0.0;
    for (uint64_t i = 0; i < o->dim; ++i) {
        run += creal(o->psi[i]) * creal(o->psi[i]) + cimag(o->psi[i]) * cimag(o->psi[i]);
        c[i] = run;
    }
    const double T = run;
    if (!(T > 0.0)) { free(c); return ORC_E_STATE; }
    for (int64_t s = 0; s < S; ++s) {
        if (!(u[s] >= 0.0 && u[s] < 1.0)) { free(c); return ORC_E_ARG; }
        const double target = u[s] * T;
        /* bisection for the first i with c[i] > target; c is nondecreasing and
           c[dim-1] = T > target unless the product rounded up to T */
        uint64_t lo = 0, hi = o->dim - 1;
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (c[mid] > target) hi = mid; else lo = mid + 1;
        }
        /* if the draw rounded onto T, step back to the last index of nonzero weight */
        while (lo > 0 && !(c[lo] > (lo ? c[lo - 1] : 0.0))) --lo;
        out[s] = project(lo, nq, qubits);
        if (margin) {
            double below = target - (lo ? c[lo - 1] : 0.0);
            double above = c[lo] - target;
            margin[s] = (below < above ? below : above) / T;
        }
    }
    free(c);
    return ORC_OK;
}
