/*
 * ORACLE — test infrastructure only.
 *
 * A plain, slow, complex128 gate-by-gate state-vector simulator used to check
 * the GPU path.  Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it; the product library never does.  It shares no
 * code, header or table with the GPU path: the only thing the two have in
 * common is the layout of the gate record they both read.
 *
 * What it computes (paper, Section 3.1 and Section 3.2):
 *   - a state of n qubits is a vector of 2^n complex amplitudes, qubit q being
 *     bit q of the index (the column-major stacking of Eq. 4 / Eq. 7);
 *   - a gate on one qubit is a 2x2 unitary, on two qubits a 4x4 unitary; its
 *     action on the full state is the Kronecker embedding of Eq. 5 / Eq. 6,
 *     carried out as the contraction of Eq. 9 (sum over the gate's input index
 *     for every value of the untouched indices);
 *   - the circuit is the gates applied one after the other in list order.
 * Every two-qubit gate, CX and CZ included, goes through the same generic 4x4
 * contraction on purpose.
 *
 * Expectation values and the adjoint gradient are not in the paper; they are
 * the textbook definitions (Pauli strings applied to a copy, inner product)
 * and the reverse-mode adjoint method of Jones & Gacon (arXiv:2009.02823).
 *
 * Gate matrices follow the OpenQASM 2 / textbook definitions (the paper names
 * H, CX and the phase gate; the others are standard):
 *   U3(t,p,l) = [[cos t/2, -e^{il} sin t/2], [e^{ip} sin t/2, e^{i(p+l)} cos t/2]]
 *   RX(t) = exp(-i t X/2), RY(t) = exp(-i t Y/2), RZ(t) = exp(-i t Z/2),
 *   RZZ(t) = exp(-i t Z(x)Z/2), P(l) = diag(1, e^{il}), CP(l) = diag(1,1,1,e^{il}).
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

/* Layout of the interchange record (a plain data format, not shared code). */
typedef struct {
    int32_t kind, q0, q1, param;
    double angle[3];
    double mat[32];
} og_gate;

typedef struct {
    double coeff;
    uint64_t x_mask; /* X or Y on the qubit */
    uint64_t z_mask; /* Z or Y on the qubit */
} og_pauli;

enum {
    OG_H = 1, OG_X = 2, OG_Y = 3, OG_Z = 4, OG_S = 5, OG_SDG = 6, OG_T = 7, OG_TDG = 8, OG_SX = 9,
    OG_RX = 10, OG_RY = 11, OG_RZ = 12, OG_P = 13, OG_U3 = 14,
    OG_CX = 20, OG_CY = 21, OG_CZ = 22, OG_CP = 23, OG_SWAP = 24, OG_RZZ = 25,
    OG_MAT1 = 30, OG_MAT2 = 31
};

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Number of qubits a gate kind acts on, 0 for an unknown kind. */
static int kind_arity(int kind)
{
    if ((kind >= OG_H && kind <= OG_U3) || kind == OG_MAT1) return 1;
    if ((kind >= OG_CX && kind <= OG_RZZ) || kind == OG_MAT2) return 2;
    return 0;
}

/*
 * Gate matrix in row-major order; for two-qubit gates the local index is
 * j = b(q0) + 2 b(q1) (q0 is the control of CX/CY/CZ/CP, q1 the target).
 * Returns the arity, or 0 for an unknown kind.
 */
static int gate_matrix(const og_gate *g, const double *theta, cplx m[16])
{
    int kind = g->kind;
    double a = g->angle[0];
    if (g->param >= 0) a = theta[g->param];
    double c = cos(a / 2.0), s = sin(a / 2.0);
    const double r2 = 1.0 / sqrt(2.0);
    memset(m, 0, 16 * sizeof(cplx));
    switch (kind) {
    case OG_H: m[0] = r2; m[1] = r2; m[2] = r2; m[3] = -r2; return 1;
    case OG_X: m[1] = 1; m[2] = 1; return 1;
    case OG_Y: m[1] = -I; m[2] = I; return 1;
    case OG_Z: m[0] = 1; m[3] = -1; return 1;
    case OG_S: m[0] = 1; m[3] = I; return 1;
    case OG_SDG: m[0] = 1; m[3] = -I; return 1;
    case OG_T: m[0] = 1; m[3] = cexp(I * M_PI / 4.0); return 1;
    case OG_TDG: m[0] = 1; m[3] = cexp(-I * M_PI / 4.0); return 1;
    case OG_SX: m[0] = 0.5 * (1 + I); m[1] = 0.5 * (1 - I); m[2] = 0.5 * (1 - I); m[3] = 0.5 * (1 + I); return 1;
    case OG_RX: m[0] = c; m[1] = -I * s; m[2] = -I * s; m[3] = c; return 1;
    case OG_RY: m[0] = c; m[1] = -s; m[2] = s; m[3] = c; return 1;
    case OG_RZ: m[0] = cexp(-I * a / 2.0); m[3] = cexp(I * a / 2.0); return 1;
    case OG_P: m[0] = 1; m[3] = cexp(I * a); return 1;
    case OG_U3: {
        double t = g->angle[0], p = g->angle[1], l = g->angle[2];
        double ct = cos(t / 2.0), st = sin(t / 2.0);
        m[0] = ct;
        m[1] = -cexp(I * l) * st;
        m[2] = cexp(I * p) * st;
        m[3] = cexp(I * (p + l)) * ct;
        return 1;
    }
    case OG_MAT1:
        for (int k = 0; k < 4; ++k) m[k] = g->mat[2 * k] + I * g->mat[2 * k + 1];
        return 1;
    /* two-qubit gates, local index j = b(q0) + 2 b(q1) */
    case OG_CX: /* b(q0)=1: flip b(q1): j=1 <-> j=3 */
        m[0 * 4 + 0] = 1; m[2 * 4 + 2] = 1; m[1 * 4 + 3] = 1; m[3 * 4 + 1] = 1; return 2;
    case OG_CY: /* b(q0)=1: Y on q1; j=1 is target 0, j=3 target 1 */
        m[0 * 4 + 0] = 1; m[2 * 4 + 2] = 1; m[1 * 4 + 3] = -I; m[3 * 4 + 1] = I; return 2;
    case OG_CZ: m[0] = 1; m[5] = 1; m[10] = 1; m[15] = -1; return 2;
    case OG_CP: m[0] = 1; m[5] = 1; m[10] = 1; m[15] = cexp(I * a); return 2;
    case OG_SWAP: m[0] = 1; m[1 * 4 + 2] = 1; m[2 * 4 + 1] = 1; m[15] = 1; return 2;
    case OG_RZZ: /* exp(-i a Z(x)Z / 2): phase e^{-ia/2} on even parity, e^{+ia/2} on odd */
        m[0] = cexp(-I * a / 2.0); m[5] = cexp(I * a / 2.0); m[10] = cexp(I * a / 2.0); m[15] = cexp(-I * a / 2.0);
        return 2;
    case OG_MAT2:
        for (int k = 0; k < 16; ++k) m[k] = g->mat[2 * k] + I * g->mat[2 * k + 1];
        return 2;
    default:
        return 0;
    }
}

/* Exported for the unitarity pins: writes the matrix as (re, im) pairs. */
int oracle_gate_matrix(const og_gate *g, const double *theta, double *out)
{
    cplx m[16];
    int k = gate_matrix(g, theta, m);
    int d = k == 1 ? 2 : 4;
    for (int i = 0; i < d * d; ++i) {
        out[2 * i] = creal(m[i]);
        out[2 * i + 1] = cimag(m[i]);
    }
    return k;
}

/* Eq. 9 for a one-qubit tensor: every pair of amplitudes that differ only in
 * bit q is multiplied by the 2x2 matrix. */
static void contract1(int n, int q, const cplx m[4], cplx *psi)
{
    int64_t half = (int64_t)1 << (n - 1), stride = (int64_t)1 << q;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < half; ++x) {
        int64_t i0 = ((x >> q) << (q + 1)) | (x & (stride - 1));
        int64_t i1 = i0 | stride;
        cplx a = psi[i0], b = psi[i1];
        psi[i0] = m[0] * a + m[1] * b;
        psi[i1] = m[2] * a + m[3] * b;
    }
}

/* Eq. 9 for a two-qubit tensor: every group of four amplitudes that differ
 * only in bits q0, q1 is multiplied by the 4x4 matrix (local j = b0 + 2 b1). */
static void contract2(int n, int q0, int q1, const cplx m[16], int dagger, cplx *psi)
{
    int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
    int64_t quarter = (int64_t)1 << (n - 2);
    int64_t s0 = (int64_t)1 << q0, s1 = (int64_t)1 << q1;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < quarter; ++x) {
        /* insert zero bits at positions lo then hi */
        int64_t y = ((x >> lo) << (lo + 1)) | (x & (((int64_t)1 << lo) - 1));
        y = ((y >> hi) << (hi + 1)) | (y & (((int64_t)1 << hi) - 1));
        int64_t idx[4] = {y, y | s0, y | s1, y | s0 | s1};
        cplx v[4], w[4];
        for (int j = 0; j < 4; ++j) v[j] = psi[idx[j]];
        for (int i = 0; i < 4; ++i) {
            cplx acc = 0;
            for (int j = 0; j < 4; ++j) acc += (dagger ? conj(m[j * 4 + i]) : m[i * 4 + j]) * v[j];
            w[i] = acc;
        }
        for (int j = 0; j < 4; ++j) psi[idx[j]] = w[j];
    }
}

static int check_gate(int n, const og_gate *g, int64_t n_params)
{
    int k = kind_arity(g->kind);
    if (k == 0) return -1;
    if (g->q0 < 0 || g->q0 >= n) return -2;
    if (k == 2 && (g->q1 < 0 || g->q1 >= n || g->q1 == g->q0)) return -2;
    if (g->param >= 0) {
        if (g->param >= n_params) return -3;
        if (g->kind != OG_RX && g->kind != OG_RY && g->kind != OG_RZ && g->kind != OG_RZZ) return -3;
    }
    return k;
}

static void apply_gate(int n, const og_gate *g, const double *theta, int dagger, cplx *psi)
{
    cplx m[16];
    int k = gate_matrix(g, theta, m);
    if (k == 1) {
        cplx u[4] = {m[0], m[1], m[2], m[3]};
        if (dagger) { u[0] = conj(m[0]); u[1] = conj(m[2]); u[2] = conj(m[1]); u[3] = conj(m[3]); }
        contract1(n, g->q0, u, psi);
    } else {
        contract2(n, g->q0, g->q1, m, dagger, psi);
    }
}

/*
 * psi <- U_G ... U_1 psi, in place, gates in list order.
 * Returns 0, or a negative value for an invalid gate (nothing applied).
 */
int oracle_apply(int n, const og_gate *gates, int64_t n_gates, const double *theta, int64_t n_params, cplx *psi)
{
    if (n < 1 || n > 40) return -4;
    for (int64_t i = 0; i < n_gates; ++i)
        if (check_gate(n, &gates[i], n_params) < 0) return check_gate(n, &gates[i], n_params);
    for (int64_t i = 0; i < n_gates; ++i) apply_gate(n, &gates[i], theta, 0, psi);
    return 0;
}

/* Same as oracle_apply but only the gate range [g0, g1) — for prefix timings. */
int oracle_apply_range(int n, const og_gate *gates, int64_t g0, int64_t g1, const double *theta, int64_t n_params, cplx *psi)
{
    return oracle_apply(n, gates + g0, g1 - g0, theta, n_params, psi);
}

/* out <- P psi for one Pauli string, by applying X, Y, Z qubit by qubit. */
static void apply_pauli(int n, const og_pauli *p, const cplx *psi, cplx *out)
{
    int64_t dim = (int64_t)1 << n;
    memcpy(out, psi, (size_t)dim * sizeof(cplx));
    const cplx X[4] = {0, 1, 1, 0}, Y[4] = {0, -I, I, 0}, Z[4] = {1, 0, 0, -1};
    for (int q = 0; q < n; ++q) {
        int x = (int)((p->x_mask >> q) & 1), z = (int)((p->z_mask >> q) & 1);
        if (x && z) contract1(n, q, Y, out);
        else if (x) contract1(n, q, X, out);
        else if (z) contract1(n, q, Z, out);
    }
}

static cplx inner(int64_t dim, const cplx *a, const cplx *b) /* <a|b> */
{
    cplx s = 0;
    for (int64_t x = 0; x < dim; ++x) s += conj(a[x]) * b[x];
    return s;
}

/* lam <- H psi = sum_t c_t P_t psi. */
static void apply_hamiltonian(int n, const og_pauli *H, int n_terms, const cplx *psi, cplx *lam, cplx *tmp)
{
    int64_t dim = (int64_t)1 << n;
    memset(lam, 0, (size_t)dim * sizeof(cplx));
    for (int t = 0; t < n_terms; ++t) {
        apply_pauli(n, &H[t], psi, tmp);
        for (int64_t x = 0; x < dim; ++x) lam[x] += H[t].coeff * tmp[x];
    }
}

/* E = sum_t c_t <psi|P_t|psi>; each term applied to a copy of psi.
 * Returns NAN when the work buffer cannot be allocated. */
double oracle_expect(int n, const og_pauli *H, int n_terms, const cplx *psi)
{
    int64_t dim = (int64_t)1 << n;
    cplx *tmp = (cplx *)malloc((size_t)dim * sizeof(cplx));
    if (!tmp) return NAN;
    double e = 0.0;
    for (int t = 0; t < n_terms; ++t) {
        apply_pauli(n, &H[t], psi, tmp);
        e += H[t].coeff * creal(inner(dim, psi, tmp));
    }
    free(tmp);
    return e;
}

/* Norm squared <psi|psi>. */
double oracle_norm2(int n, const cplx *psi)
{
    return creal(inner((int64_t)1 << n, psi, psi));
}

/*
 * Adjoint gradient (Jones & Gacon): psi = C|0..0>, lam = H psi; walking the
 * gates backwards, for a parameterised rotation exp(-i a P / 2) the
 * derivative is Im <lam|P|psi> with both states taken just after the gate,
 * then psi <- U^dag psi and lam <- U^dag lam.  A parameter used by several
 * gates receives the sum of their terms.  grad must hold n_params zeros.
 * Returns 0, or a negative value on invalid input / allocation failure.
 */
int oracle_adjoint(int n, const og_gate *gates, int64_t n_gates, const double *theta, int64_t n_params,
                   const og_pauli *H, int n_terms, double *energy, double *grad)
{
    if (n < 1 || n > 30) return -4;
    int64_t dim = (int64_t)1 << n;
    for (int64_t i = 0; i < n_gates; ++i)
        if (check_gate(n, &gates[i], n_params) < 0) return check_gate(n, &gates[i], n_params);
    cplx *psi = (cplx *)calloc((size_t)dim, sizeof(cplx));
    cplx *lam = (cplx *)malloc((size_t)dim * sizeof(cplx));
    cplx *tmp = (cplx *)malloc((size_t)dim * sizeof(cplx));
    if (!psi || !lam || !tmp) { free(psi); free(lam); free(tmp); return -5; }
    psi[0] = 1.0;
    for (int64_t i = 0; i < n_gates; ++i) apply_gate(n, &gates[i], theta, 0, psi);
    apply_hamiltonian(n, H, n_terms, psi, lam, tmp);
    *energy = creal(inner(dim, psi, lam));
    for (int64_t j = n_gates - 1; j >= 0; --j) {
        const og_gate *g = &gates[j];
        if (g->param >= 0) {
            og_pauli gen = {1.0, 0, 0};
            switch (g->kind) {
            case OG_RX: gen.x_mask = 1ull << g->q0; break;
            case OG_RY: gen.x_mask = 1ull << g->q0; gen.z_mask = 1ull << g->q0; break;
            case OG_RZ: gen.z_mask = 1ull << g->q0; break;
            case OG_RZZ: gen.z_mask = (1ull << g->q0) | (1ull << g->q1); break;
            default: break;
            }
            apply_pauli(n, &gen, psi, tmp);
            grad[g->param] += cimag(inner(dim, lam, tmp));
        }
        apply_gate(n, g, theta, 1, psi);
        apply_gate(n, g, theta, 1, lam);
    }
    free(psi); free(lam); free(tmp);
    return 0;
}
