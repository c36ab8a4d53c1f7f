/*
 * hubbard_oracle.c -- plain, slow, obviously-correct CPU reference for the
 * Hubbard Hamiltonian-variational state-vector path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the GPU library, and the GPU library never calls it.
 *
 * What it computes (the paper: Alvertis et al., "Classical Benchmarks for
 * Variational Quantum Eigensolver Simulations of the Hubbard Model"):
 *   - H of Eq. (1), generalised per bond/site as in Eq. (2), (15), (16):
 *       H = sum_bonds sum_sigma (-t_b)(a+_i a_j + a+_j a_i)
 *         + U sum_i n_i,up n_i,dn + sum_bonds V_b n_i n_j + sum_i eps_i n_i
 *     with n_i = n_i,up + n_i,dn, every unordered nearest-neighbour bond once.
 *   - the parameterised circuit of Eq. (3) built from the layer of Eq. (7):
 *     each layer is exp(-i th_0 D) followed by exp(-i th_g H_hop,g) for every
 *     hopping group g in application order (D = all diagonal terms of H).
 *   - the energy of Eq. (4), E = <psi|H|psi>.
 *   - the gradient of Sec. 2.1 (the inline adjoint formula): with
 *     U_k = exp(-i th_k G_k), dE/dth_k = 2 Im <lambda_k| G_k |psi_k>, where
 *     psi_k is the state after gate k and lambda_k = U_{k+1}^+ ... U_P^+ H psi.
 *
 * Encoding (Sec. 2.2.1, Jordan-Wigner): one qubit per spin-orbital, bit q of
 * the amplitude index b is the occupation of qubit q, and
 * a_q = (prod_{r<q} Z_r) sigma^-_q.  The qubit of (site, spin) is either
 * spin-blocked (q = site + nsites*spin) or interleaved (q = 2*site + spin);
 * energies and gradients do not depend on this choice.
 *
 * Everything is plain loops over all 2^n amplitudes in complex128; the only
 * concession to speed is an optional OpenMP split of the outermost amplitude
 * loops.  Sums use Neumaier compensation over fixed chunks so the result does
 * not depend on the thread count.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORC_MAX_SITES 32
#define ORC_MAX_BONDS 128

/* Model description filled by the Python side of the oracle (oracle/model.py).
 * bond_slot[b] is the parameter slot (1..ngroups) of the hopping group that
 * bond b belongs to; slot 0 of every layer is the diagonal D. */
typedef struct {
    int32_t nsites;
    int32_t nbonds;
    int32_t interleaved;
    int32_t ngroups;
    int32_t bond_i[ORC_MAX_BONDS];
    int32_t bond_j[ORC_MAX_BONDS];
    int32_t bond_slot[ORC_MAX_BONDS];
    double t[ORC_MAX_BONDS];
    double V[ORC_MAX_BONDS];
    double eps[ORC_MAX_SITES];
    double U;
} orc_model;

static int qubit_of(const orc_model *m, int site, int spin)
{
    if (m->interleaved)
        return 2 * site + spin;
    return site + m->nsites * spin;
}

static int nqubits(const orc_model *m) { return 2 * m->nsites; }

static int bit(uint64_t b, int q) { return (int)((b >> q) & 1u); }

/* ---------------------------------------------------------------- sums --- */

/* Neumaier-compensated running sum. */
typedef struct {
    double s, c;
} nsum;

static void nsum_add(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double nsum_value(const nsum *a) { return a->s + a->c; }

#define CHUNK_BITS 12

/* ---------------------------------------------------- diagonal part D --- */

/* D(b) = U sum_i n_up n_dn + sum_bonds V n_i n_j + sum_i eps_i n_i. */
static double diag_value(const orc_model *m, uint64_t b)
{
    double d = 0.0;
    for (int i = 0; i < m->nsites; i++) {
        int up = bit(b, qubit_of(m, i, 0));
        int dn = bit(b, qubit_of(m, i, 1));
        d += m->U * (double)(up * dn);
        d += m->eps[i] * (double)(up + dn);
    }
    for (int k = 0; k < m->nbonds; k++) {
        int i = m->bond_i[k], j = m->bond_j[k];
        int ni = bit(b, qubit_of(m, i, 0)) + bit(b, qubit_of(m, i, 1));
        int nj = bit(b, qubit_of(m, j, 0)) + bit(b, qubit_of(m, j, 1));
        d += m->V[k] * (double)(ni * nj);
    }
    return d;
}

/* -------------------------------------------- one hopping term a+a + h.c. */

/* Jordan-Wigner sign of a+_p a_q (or a+_q a_p) acting on b: (-1) to the
 * number of occupied qubits strictly between p and q. */
static double jw_sign(uint64_t b, int p, int q)
{
    int lo = p < q ? p : q, hi = p < q ? q : p;
    int count = 0;
    for (int r = lo + 1; r < hi; r++)
        count += bit(b, r);
    return (count & 1) ? -1.0 : 1.0;
}

/* psi <- exp(-i theta coef (a+_p a_q + a+_q a_p)) psi.
 * On each pair {x, y = x ^ (2^p + 2^q)} with exactly one of p, q occupied the
 * term acts as sg * [[0,1],[1,0]] (sg = jw_sign), so the exponential there is
 * cos(theta coef) 1 - i sin(theta coef) sg X; it is the identity elsewhere. */
static void apply_hop_term(int n, int p, int q, double coef, double theta, cplx *psi)
{
    const uint64_t dim = (uint64_t)1 << n;
    const uint64_t mask = ((uint64_t)1 << p) | ((uint64_t)1 << q);
    const double c = cos(theta * coef), s = sin(theta * coef);
#pragma omp parallel for schedule(static)
    for (int64_t xs = 0; xs < (int64_t)dim; xs++) {
        uint64_t x = (uint64_t)xs;
        if (bit(x, p) == 1 && bit(x, q) == 0) {
            uint64_t y = x ^ mask;
            double sg = jw_sign(x, p, q);
            cplx px = psi[x], py = psi[y];
            psi[x] = c * px - I * (sg * s) * py;
            psi[y] = -I * (sg * s) * px + c * py;
        }
    }
}

/* out += coef * (a+_p a_q + a+_q a_p) psi */
static void add_hop_term(int n, int p, int q, double coef, const cplx *psi, cplx *out)
{
    const uint64_t dim = (uint64_t)1 << n;
    const uint64_t mask = ((uint64_t)1 << p) | ((uint64_t)1 << q);
#pragma omp parallel for schedule(static)
    for (int64_t bs = 0; bs < (int64_t)dim; bs++) {
        uint64_t b = (uint64_t)bs;
        if (bit(b, p) != bit(b, q))
            out[b] += coef * jw_sign(b, p, q) * psi[b ^ mask];
    }
}

/* ----------------------------------------------------------- gates ------ */

void orc_init_basis(const orc_model *m, uint64_t b0, cplx *psi)
{
    const uint64_t dim = (uint64_t)1 << nqubits(m);
    memset(psi, 0, dim * sizeof(cplx));
    psi[b0] = 1.0;
}

/* psi <- exp(-i theta G_slot) psi.  Slot 0 is the diagonal D; slot g >= 1
 * is the hopping group g, whose terms act on disjoint qubit pairs and
 * therefore commute, so the group exponential is the product of the term
 * exponentials (each term for both spins). */
void orc_apply_slot(const orc_model *m, int slot, double theta, cplx *psi)
{
    const int n = nqubits(m);
    const uint64_t dim = (uint64_t)1 << n;
    if (slot == 0) {
#pragma omp parallel for schedule(static)
        for (int64_t bs = 0; bs < (int64_t)dim; bs++) {
            double ang = theta * diag_value(m, (uint64_t)bs);
            psi[bs] *= cos(ang) - I * sin(ang);
        }
        return;
    }
    for (int k = 0; k < m->nbonds; k++) {
        if (m->bond_slot[k] != slot)
            continue;
        for (int spin = 0; spin < 2; spin++) {
            int p = qubit_of(m, m->bond_i[k], spin);
            int q = qubit_of(m, m->bond_j[k], spin);
            apply_hop_term(n, p, q, -m->t[k], theta, psi);
        }
    }
}

/* out = G_slot psi (the generator itself, not its exponential). */
void orc_generator_apply(const orc_model *m, int slot, const cplx *psi, cplx *out)
{
    const int n = nqubits(m);
    const uint64_t dim = (uint64_t)1 << n;
    if (slot == 0) {
#pragma omp parallel for schedule(static)
        for (int64_t bs = 0; bs < (int64_t)dim; bs++)
            out[bs] = diag_value(m, (uint64_t)bs) * psi[bs];
        return;
    }
    memset(out, 0, dim * sizeof(cplx));
    for (int k = 0; k < m->nbonds; k++) {
        if (m->bond_slot[k] != slot)
            continue;
        for (int spin = 0; spin < 2; spin++) {
            int p = qubit_of(m, m->bond_i[k], spin);
            int q = qubit_of(m, m->bond_j[k], spin);
            add_hop_term(n, p, q, -m->t[k], psi, out);
        }
    }
}

/* out = H psi, matrix-free: D psi plus every hopping term of every bond. */
void orc_ham_apply(const orc_model *m, const cplx *psi, cplx *out)
{
    const int n = nqubits(m);
    const uint64_t dim = (uint64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t bs = 0; bs < (int64_t)dim; bs++)
        out[bs] = diag_value(m, (uint64_t)bs) * psi[bs];
    for (int k = 0; k < m->nbonds; k++) {
        for (int spin = 0; spin < 2; spin++) {
            int p = qubit_of(m, m->bond_i[k], spin);
            int q = qubit_of(m, m->bond_j[k], spin);
            add_hop_term(n, p, q, -m->t[k], psi, out);
        }
    }
}

/* Row b of H (Eq. (1) with the terms of Eq. (2), (15), (16)): H|b'> has
 * amplitude <b|H|b'> at b, so (H psi)_b = sum over the row of coef * psi[col].
 * The row holds the diagonal D(b) at col = b and, for every bond and spin
 * whose two qubits differ in occupation, -t_b times the Jordan-Wigner sign at
 * col = b ^ (2^p + 2^q).  cols/coefs need room for 1 + 2 * nbonds entries;
 * returns the number written. */
int orc_ham_row(const orc_model *m, uint64_t b, uint64_t *cols, double *coefs)
{
    int k = 0;
    cols[k] = b;
    coefs[k] = diag_value(m, b);
    k++;
    for (int e = 0; e < m->nbonds; e++) {
        for (int spin = 0; spin < 2; spin++) {
            int p = qubit_of(m, m->bond_i[e], spin);
            int q = qubit_of(m, m->bond_j[e], spin);
            if (bit(b, p) != bit(b, q)) {
                cols[k] = b ^ (((uint64_t)1 << p) | ((uint64_t)1 << q));
                coefs[k] = -m->t[e] * jw_sign(b, p, q);
                k++;
            }
        }
    }
    return k;
}

/* <a|b> = sum_b conj(a_b) b_b, compensated, chunk-deterministic. */
void orc_inner(int n, const cplx *a, const cplx *b, double *re, double *im)
{
    const uint64_t dim = (uint64_t)1 << n;
    const uint64_t chunk = dim < ((uint64_t)1 << CHUNK_BITS) ? dim : ((uint64_t)1 << CHUNK_BITS);
    const int64_t nchunks = (int64_t)(dim / chunk);
    double *pr = malloc((size_t)nchunks * sizeof(double));
    double *pi = malloc((size_t)nchunks * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nchunks; c++) {
        nsum sr = {0, 0}, si = {0, 0};
        for (uint64_t k = (uint64_t)c * chunk; k < (uint64_t)(c + 1) * chunk; k++) {
            cplx z = conj(a[k]) * b[k];
            nsum_add(&sr, creal(z));
            nsum_add(&si, cimag(z));
        }
        pr[c] = nsum_value(&sr);
        pi[c] = nsum_value(&si);
    }
    nsum tr = {0, 0}, ti = {0, 0};
    for (int64_t c = 0; c < nchunks; c++) {
        nsum_add(&tr, pr[c]);
        nsum_add(&ti, pi[c]);
    }
    *re = nsum_value(&tr);
    *im = nsum_value(&ti);
    free(pr);
    free(pi);
}

/* Eq. (3): psi = U_P ... U_1 |b0>, layer-major parameters theta[l*(1+G)+slot]. */
void orc_ansatz(const orc_model *m, const double *theta, int layers, uint64_t b0, cplx *psi)
{
    const int per = 1 + m->ngroups;
    orc_init_basis(m, b0, psi);
    for (int l = 0; l < layers; l++)
        for (int s = 0; s < per; s++)
            orc_apply_slot(m, s, theta[l * per + s], psi);
}

/* Eq. (4): E = <psi|H|psi> for a given state. scratch has 2^n entries. */
double orc_expectation(const orc_model *m, const cplx *psi, cplx *scratch)
{
    double re, im;
    orc_ham_apply(m, psi, scratch);
    orc_inner(nqubits(m), psi, scratch, &re, &im);
    return re;
}

/* Energy of the circuit state; returns 0 on success, -1 on allocation failure. */
int orc_energy(const orc_model *m, const double *theta, int layers, uint64_t b0, double *E)
{
    const uint64_t dim = (uint64_t)1 << nqubits(m);
    cplx *psi = malloc(dim * sizeof(cplx));
    cplx *phi = malloc(dim * sizeof(cplx));
    if (!psi || !phi) {
        free(psi);
        free(phi);
        return -1;
    }
    orc_ansatz(m, theta, layers, b0, psi);
    *E = orc_expectation(m, psi, phi);
    free(psi);
    free(phi);
    return 0;
}

/* Energy and gradient by the adjoint recursion of Sec. 2.1:
 *   psi <- psi_P, lambda <- H psi_P;
 *   for k = P .. 1:  g_k = 2 Im <lambda|G_k|psi>;  psi <- U_k^+ psi;
 *                    lambda <- U_k^+ lambda.
 * (G_k commutes with U_k, so evaluating the bracket before or after the
 * un-application gives the same number.)  Returns 0 or -1 (allocation). */
int orc_energy_grad(const orc_model *m, const double *theta, int layers, uint64_t b0,
                    double *E, double *grad)
{
    const int n = nqubits(m);
    const uint64_t dim = (uint64_t)1 << n;
    const int per = 1 + m->ngroups;
    cplx *psi = malloc(dim * sizeof(cplx));
    cplx *lam = malloc(dim * sizeof(cplx));
    cplx *tmp = malloc(dim * sizeof(cplx));
    if (!psi || !lam || !tmp) {
        free(psi);
        free(lam);
        free(tmp);
        return -1;
    }
    orc_ansatz(m, theta, layers, b0, psi);
    orc_ham_apply(m, psi, lam);
    double re, im;
    orc_inner(n, psi, lam, &re, &im);
    *E = re;
    for (int k = layers * per - 1; k >= 0; k--) {
        int slot = k % per;
        orc_generator_apply(m, slot, psi, tmp);
        orc_inner(n, lam, tmp, &re, &im);
        grad[k] = 2.0 * im;
        orc_apply_slot(m, slot, -theta[k], psi);
        orc_apply_slot(m, slot, -theta[k], lam);
    }
    free(psi);
    free(lam);
    free(tmp);
    return 0;
}

/* Number of OpenMP threads the oracle's loops use (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int t) { omp_set_num_threads(t); }
#else
int orc_threads(void) { return 1; }
void orc_set_threads(int t) { (void)t; }
#endif
