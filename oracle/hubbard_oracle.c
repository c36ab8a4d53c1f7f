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

/* ------------------------------------ fixed-(N_up, N_dn) sector form ----- */

/* Every hopping term moves one electron between two qubits of the same spin
 * and D is diagonal, so every gate of Eq. (7) and H itself conserve the
 * number of spin-up and of spin-down electrons.  A circuit started from the
 * basis state |b0> therefore stays in the sector of basis states with the
 * same counts, and every amplitude outside it stays exactly zero.  The
 * functions below keep only the sector's amplitudes (spin-blocked qubit order
 * only): at 4x4 half filling C(16,8)^2 = 1.66e8 of the 2^32 amplitudes.
 *
 * Sector position i = rd * n_up_patterns + ru, where ru (rd) is the rank of
 * the spin-up (spin-down) occupation pattern among all patterns with that
 * many electrons, in increasing numerical order; the full amplitude index is
 * up[ru] | (dn[rd] << nsites).  The gate and H arithmetic per amplitude pair
 * is the one of the full-space functions above, term for term. */

typedef struct {
    int ns;
    int64_t cu, cd;     /* number of spin-up / spin-down patterns */
    uint32_t *up, *dn;  /* patterns, increasing */
    int64_t *rank_up;   /* pattern -> rank, -1 if its popcount differs (2^ns) */
    int64_t *rank_dn;
} orc_sector;

static int popcount32(uint32_t x)
{
    int c = 0;
    for (; x; x &= x - 1u)
        c++;
    return c;
}

static void sector_free(orc_sector *S)
{
    free(S->up);
    free(S->dn);
    free(S->rank_up);
    free(S->rank_dn);
    memset(S, 0, sizeof(*S));
}

/* Patterns of nsites bits with exactly k set, and the inverse map. */
static int sector_patterns(int ns, int k, uint32_t **list, int64_t **rank, int64_t *count)
{
    const uint64_t np = (uint64_t)1 << ns;
    *rank = malloc(np * sizeof(int64_t));
    int64_t c = 0;
    if (!*rank)
        return -1;
    for (uint64_t u = 0; u < np; u++)
        (*rank)[u] = popcount32((uint32_t)u) == k ? c++ : -1;
    *list = malloc((size_t)(c ? c : 1) * sizeof(uint32_t));
    if (!*list)
        return -1;
    for (uint64_t u = 0; u < np; u++)
        if ((*rank)[u] >= 0)
            (*list)[(*rank)[u]] = (uint32_t)u;
    *count = c;
    return 0;
}

/* The sector of basis state b0 (its up and down electron counts). */
static int sector_make(const orc_model *m, uint64_t b0, orc_sector *S)
{
    memset(S, 0, sizeof(*S));
    if (m->interleaved)
        return -1;
    const int ns = m->nsites;
    const uint32_t smask = (uint32_t)(((uint64_t)1 << ns) - 1u);
    S->ns = ns;
    if (sector_patterns(ns, popcount32((uint32_t)b0 & smask), &S->up, &S->rank_up, &S->cu) ||
        sector_patterns(ns, popcount32((uint32_t)(b0 >> ns) & smask), &S->dn, &S->rank_dn,
                        &S->cd)) {
        sector_free(S);
        return -1;
    }
    return 0;
}

static uint64_t sector_full(const orc_sector *S, int64_t i)
{
    return (uint64_t)S->up[i % S->cu] | ((uint64_t)S->dn[i / S->cu] << S->ns);
}

static int64_t sector_pos(const orc_sector *S, uint64_t b)
{
    const uint64_t smask = ((uint64_t)1 << S->ns) - 1u;
    const int64_t ru = S->rank_up[b & smask], rd = S->rank_dn[(b >> S->ns) & smask];
    if (ru < 0 || rd < 0 || (b >> (2 * S->ns)) != 0)
        return -1;
    return rd * S->cu + ru;
}

static int64_t sector_dim(const orc_sector *S) { return S->cu * S->cd; }

/* psi <- exp(-i theta coef (a+_p a_q + a+_q a_p)) psi on the sector, p and q
 * of one spin: the pairs (x, y = x with the electron moved from p to q). */
static void sec_apply_hop(const orc_sector *S, int spin, int p, int q, double coef, double theta,
                          cplx *psi)
{
    const double c = cos(theta * coef), s = sin(theta * coef);
    const int ns = S->ns;
    const uint32_t pm = 1u << (p - ns * spin), qm = 1u << (q - ns * spin);
    if (spin == 0) {
        /* pairs inside one row of fixed down pattern */
#pragma omp parallel for schedule(static)
        for (int64_t rd = 0; rd < S->cd; rd++) {
            for (int64_t ru = 0; ru < S->cu; ru++) {
                const uint32_t u = S->up[ru];
                if (!(u & pm) || (u & qm))
                    continue;
                const int64_t x = rd * S->cu + ru, y = rd * S->cu + S->rank_up[u ^ pm ^ qm];
                const double sg = jw_sign(sector_full(S, x), p, q);
                cplx px = psi[x], py = psi[y];
                psi[x] = c * px - I * (sg * s) * py;
                psi[y] = -I * (sg * s) * px + c * py;
            }
        }
    } else {
#pragma omp parallel for schedule(static)
        for (int64_t rd = 0; rd < S->cd; rd++) {
            const uint32_t d = S->dn[rd];
            if (!(d & pm) || (d & qm))
                continue;
            const int64_t rd2 = S->rank_dn[d ^ pm ^ qm];
            for (int64_t ru = 0; ru < S->cu; ru++) {
                const int64_t x = rd * S->cu + ru, y = rd2 * S->cu + ru;
                const double sg = jw_sign(sector_full(S, x), p, q);
                cplx px = psi[x], py = psi[y];
                psi[x] = c * px - I * (sg * s) * py;
                psi[y] = -I * (sg * s) * px + c * py;
            }
        }
    }
}

/* out += coef * (a+_p a_q + a+_q a_p) psi on the sector. */
static void sec_add_hop(const orc_sector *S, int p, int q, double coef, const cplx *psi,
                        cplx *out)
{
    const uint64_t mask = ((uint64_t)1 << p) | ((uint64_t)1 << q);
    const int64_t dim = sector_dim(S);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; i++) {
        const uint64_t b = sector_full(S, i);
        if (bit(b, p) != bit(b, q))
            out[i] += coef * jw_sign(b, p, q) * psi[sector_pos(S, b ^ mask)];
    }
}

static void sec_apply_slot(const orc_model *m, const orc_sector *S, int slot, double theta,
                           cplx *psi)
{
    if (slot == 0) {
        const int64_t dim = sector_dim(S);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < dim; i++) {
            double ang = theta * diag_value(m, sector_full(S, i));
            psi[i] *= cos(ang) - I * sin(ang);
        }
        return;
    }
    for (int k = 0; k < m->nbonds; k++) {
        if (m->bond_slot[k] != slot)
            continue;
        for (int spin = 0; spin < 2; spin++)
            sec_apply_hop(S, spin, qubit_of(m, m->bond_i[k], spin),
                          qubit_of(m, m->bond_j[k], spin), -m->t[k], theta, psi);
    }
}

static void sec_generator_apply(const orc_model *m, const orc_sector *S, int slot,
                                const cplx *psi, cplx *out)
{
    const int64_t dim = sector_dim(S);
    if (slot == 0) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < dim; i++)
            out[i] = diag_value(m, sector_full(S, i)) * psi[i];
        return;
    }
    memset(out, 0, (size_t)dim * sizeof(cplx));
    for (int k = 0; k < m->nbonds; k++) {
        if (m->bond_slot[k] != slot)
            continue;
        for (int spin = 0; spin < 2; spin++)
            sec_add_hop(S, qubit_of(m, m->bond_i[k], spin), qubit_of(m, m->bond_j[k], spin),
                        -m->t[k], psi, out);
    }
}

static void sec_ham_apply(const orc_model *m, const orc_sector *S, const cplx *psi, cplx *out)
{
    const int64_t dim = sector_dim(S);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; i++)
        out[i] = diag_value(m, sector_full(S, i)) * psi[i];
    for (int k = 0; k < m->nbonds; k++)
        for (int spin = 0; spin < 2; spin++)
            sec_add_hop(S, qubit_of(m, m->bond_i[k], spin), qubit_of(m, m->bond_j[k], spin),
                        -m->t[k], psi, out);
}

/* <a|b> over n entries, compensated, chunk-deterministic. */
static void sec_inner(int64_t n, const cplx *a, const cplx *b, double *re, double *im)
{
    const int64_t chunk = (int64_t)1 << CHUNK_BITS;
    const int64_t nchunks = (n + chunk - 1) / chunk;
    double *pr = malloc((size_t)(nchunks ? nchunks : 1) * sizeof(double));
    double *pi = malloc((size_t)(nchunks ? nchunks : 1) * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nchunks; c++) {
        nsum sr = {0, 0}, si = {0, 0};
        const int64_t end = (c + 1) * chunk < n ? (c + 1) * chunk : n;
        for (int64_t k = c * chunk; k < end; k++) {
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

/* Number of amplitudes in the sector of b0 (0 for the interleaved order). */
int64_t orc_sector_dim(const orc_model *m, uint64_t b0)
{
    orc_sector S;
    if (sector_make(m, b0, &S))
        return 0;
    int64_t d = sector_dim(&S);
    sector_free(&S);
    return d;
}

/* Full amplitude index of every sector position (out holds dim entries). */
int orc_sector_indices(const orc_model *m, uint64_t b0, uint64_t *out)
{
    orc_sector S;
    if (sector_make(m, b0, &S))
        return -1;
    for (int64_t i = 0; i < sector_dim(&S); i++)
        out[i] = sector_full(&S, i);
    sector_free(&S);
    return 0;
}

/* Eq. (3) on the sector: psi (dim entries) = U_P ... U_1 |b0>. */
int orc_sector_ansatz(const orc_model *m, const double *theta, int layers, uint64_t b0, cplx *psi)
{
    orc_sector S;
    if (sector_make(m, b0, &S))
        return -1;
    const int per = 1 + m->ngroups;
    memset(psi, 0, (size_t)sector_dim(&S) * sizeof(cplx));
    psi[sector_pos(&S, b0)] = 1.0;
    for (int l = 0; l < layers; l++)
        for (int s = 0; s < per; s++)
            sec_apply_slot(m, &S, s, theta[l * per + s], psi);
    sector_free(&S);
    return 0;
}

/* out = H psi on the sector of b0 (H maps the sector into itself). */
int orc_sector_ham_apply(const orc_model *m, uint64_t b0, const cplx *psi, cplx *out)
{
    orc_sector S;
    if (sector_make(m, b0, &S))
        return -1;
    sec_ham_apply(m, &S, psi, out);
    sector_free(&S);
    return 0;
}

/* Energy and adjoint gradient on the sector: the recursion of
 * orc_energy_grad with every vector restricted to the sector.  Returns 0, or
 * -1 (allocation failure or interleaved order). */
int orc_sector_energy_grad(const orc_model *m, const double *theta, int layers, uint64_t b0,
                           double *E, double *grad)
{
    orc_sector S;
    if (sector_make(m, b0, &S))
        return -1;
    const int64_t dim = sector_dim(&S);
    const int per = 1 + m->ngroups;
    cplx *psi = malloc((size_t)dim * sizeof(cplx));
    cplx *lam = malloc((size_t)dim * sizeof(cplx));
    cplx *tmp = grad ? malloc((size_t)dim * sizeof(cplx)) : NULL;
    if (!psi || !lam || (grad && !tmp)) {
        free(psi);
        free(lam);
        free(tmp);
        sector_free(&S);
        return -1;
    }
    memset(psi, 0, (size_t)dim * sizeof(cplx));
    psi[sector_pos(&S, b0)] = 1.0;
    for (int l = 0; l < layers; l++)
        for (int s = 0; s < per; s++)
            sec_apply_slot(m, &S, s, theta[l * per + s], psi);
    sec_ham_apply(m, &S, psi, lam);
    double re, im;
    sec_inner(dim, psi, lam, &re, &im);
    *E = re;
    for (int k = grad ? layers * per - 1 : -1; k >= 0; k--) {
        int slot = k % per;
        sec_generator_apply(m, &S, slot, psi, tmp);
        sec_inner(dim, lam, tmp, &re, &im);
        grad[k] = 2.0 * im;
        sec_apply_slot(m, &S, slot, -theta[k], psi);
        sec_apply_slot(m, &S, slot, -theta[k], lam);
    }
    free(psi);
    free(lam);
    free(tmp);
    sector_free(&S);
    return 0;
}

/* ------------------------------------------- overlap loss, Eq. (5)/(6) --- */

/* f = log10(1 - F), F = |<ref|psi(theta)>|^2 (the logarithm of the
 * infidelity with a reference state), and df/dtheta_k.  F = <psi|P|psi> with
 * the projector P = |ref><ref|, so the adjoint recursion of the energy
 * applies with H replaced by P: lambda_P = P psi = <ref|psi> ref, and
 * dF/dtheta_k = 2 Im <lambda_k|G_k|psi_k>; then df = -dF / ((1 - F) ln 10).
 * out[0] = f, out[1] = F.  Returns 0 or -1 (allocation). */
int orc_overlap_grad(const orc_model *m, const double *theta, int layers, uint64_t b0,
                     const cplx *ref, double *out, double *grad)
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
    double re, im;
    orc_inner(n, ref, psi, &re, &im);   /* c = <ref|psi> */
    const cplx c = re + I * im;
    const double F = re * re + im * im;
    for (uint64_t b = 0; b < dim; b++)
        lam[b] = c * ref[b];
    out[0] = log10(1.0 - F);
    out[1] = F;
    for (int k = layers * per - 1; k >= 0; k--) {
        int slot = k % per;
        orc_generator_apply(m, slot, psi, tmp);
        orc_inner(n, lam, tmp, &re, &im);
        grad[k] = -2.0 * im / ((1.0 - F) * log(10.0));
        orc_apply_slot(m, slot, -theta[k], psi);
        orc_apply_slot(m, slot, -theta[k], lam);
    }
    free(psi);
    free(lam);
    free(tmp);
    return 0;
}

/* ------------------------------------- spin correlations, Eq. (17) ------ */

/* C[i*ns + j] = <S^z_i S^z_j> - <S^z_i><S^z_j> and Sz[i] = <S^z_i> of a
 * state, S^z_i = (n_i,up - n_i,dn) / 2, every expectation a sum over all
 * amplitudes of |psi_b|^2 times the operator's (diagonal) value at b. */
void orc_spin_correlation(const orc_model *m, const cplx *psi, double *C, double *Sz)
{
    const int ns = m->nsites;
    const uint64_t dim = (uint64_t)1 << nqubits(m);
    nsum *ss = calloc((size_t)ns * ns, sizeof(nsum));
    nsum *s1 = calloc((size_t)ns, sizeof(nsum));
    double *sz = malloc((size_t)ns * sizeof(double));
    for (uint64_t b = 0; b < dim; b++) {
        const double p = creal(psi[b]) * creal(psi[b]) + cimag(psi[b]) * cimag(psi[b]);
        if (p == 0.0)
            continue;
        for (int i = 0; i < ns; i++)
            sz[i] = 0.5 * (double)(bit(b, qubit_of(m, i, 0)) - bit(b, qubit_of(m, i, 1)));
        for (int i = 0; i < ns; i++) {
            nsum_add(&s1[i], p * sz[i]);
            for (int j = 0; j < ns; j++)
                nsum_add(&ss[i * ns + j], p * sz[i] * sz[j]);
        }
    }
    for (int i = 0; i < ns; i++)
        Sz[i] = nsum_value(&s1[i]);
    for (int i = 0; i < ns; i++)
        for (int j = 0; j < ns; j++)
            C[i * ns + j] = nsum_value(&ss[i * ns + j]) - Sz[i] * Sz[j];
    free(ss);
    free(s1);
    free(sz);
}

/* ------------------------------------------- NP ansatz, Eq. (8) -------- */

/* The number-preserving (NP) ansatz of Sec. 2.2.1: R_z(theta) on every qubit
 * before the first layer, then per layer one two-qubit gate U_NP(theta, phi)
 * (Eq. (8)) on every pair of qubits that a term of Eq. (1) couples: the two
 * spin qubits of every site (on-site terms), then every bond of every
 * hopping group, spin up then spin down.  In fermionic form, with the
 * Jordan-Wigner string that the paper's fermionic swaps supply,
 *   U_NP(theta, phi) = exp(i theta (a+_p a_q + a+_q a_p)) exp(i phi n_p n_q),
 * the rotation acting on the one-electron pair states and the phase on the
 * doubly occupied one; R_z(theta) = exp(-i theta Z / 2), Z = 1 - 2 n.
 * Parameters: [R_z of qubit 0..n-1], then per layer per term (theta, phi) in
 * the order above.  The term list (pairs of qubits) is passed in: np_p[k],
 * np_q[k] for k < n_terms (one layer). */

/* psi <- exp(-i theta coef [all bits of mask set]) psi */
static void apply_mask_phase(int n, uint64_t mask, double coef, double theta, cplx *psi)
{
    const uint64_t dim = (uint64_t)1 << n;
    const cplx ph = cos(theta * coef) - I * sin(theta * coef);
#pragma omp parallel for schedule(static)
    for (int64_t bs = 0; bs < (int64_t)dim; bs++)
        if (((uint64_t)bs & mask) == mask)
            psi[bs] *= ph;
}

/* psi <- R_z(theta) on qubit q: exp(-i theta/2) on |0>, exp(i theta/2) on |1> */
static void apply_rz(int n, int q, double theta, cplx *psi)
{
    const uint64_t dim = (uint64_t)1 << n;
    const cplx p0 = cos(0.5 * theta) - I * sin(0.5 * theta);
    const cplx p1 = cos(0.5 * theta) + I * sin(0.5 * theta);
#pragma omp parallel for schedule(static)
    for (int64_t bs = 0; bs < (int64_t)dim; bs++)
        psi[bs] *= bit((uint64_t)bs, q) ? p1 : p0;
}

/* Gate k of the NP circuit (k indexes theta): k < n is R_z of qubit k; then
 * per layer per term two gates, the rotation (even k - n) and the phase. */
static void np_apply(const orc_model *m, int nt, const int32_t *np_p, const int32_t *np_q, int k,
                     double theta, cplx *psi)
{
    const int n = nqubits(m);
    if (k < n) {
        apply_rz(n, k, theta, psi);
        return;
    }
    const int r = (k - n) % (2 * nt), term = r / 2;
    const int p = np_p[term], q = np_q[term];
    if (r % 2 == 0)
        apply_hop_term(n, p, q, -1.0, theta, psi);   /* exp(i theta K) */
    else
        apply_mask_phase(n, ((uint64_t)1 << p) | ((uint64_t)1 << q), -1.0, theta, psi);
}

/* out = G_k psi, the generator of gate k written as exp(-i theta G_k):
 * Z/2 for R_z, -K for the rotation, -n_p n_q for the phase. */
static void np_generator(const orc_model *m, int nt, const int32_t *np_p, const int32_t *np_q,
                         int k, const cplx *psi, cplx *out)
{
    const int n = nqubits(m);
    const uint64_t dim = (uint64_t)1 << n;
    if (k < n) {
#pragma omp parallel for schedule(static)
        for (int64_t bs = 0; bs < (int64_t)dim; bs++)
            out[bs] = (bit((uint64_t)bs, k) ? -0.5 : 0.5) * psi[bs];
        return;
    }
    const int r = (k - n) % (2 * nt), term = r / 2;
    const int p = np_p[term], q = np_q[term];
    if (r % 2 == 0) {
        memset(out, 0, dim * sizeof(cplx));
        add_hop_term(n, p, q, -1.0, psi, out);
    } else {
        const uint64_t mask = ((uint64_t)1 << p) | ((uint64_t)1 << q);
#pragma omp parallel for schedule(static)
        for (int64_t bs = 0; bs < (int64_t)dim; bs++)
            out[bs] = (((uint64_t)bs & mask) == mask) ? -psi[bs] : 0.0;
    }
}

void orc_np_ansatz(const orc_model *m, int nt, const int32_t *np_p, const int32_t *np_q,
                   const double *theta, int layers, uint64_t b0, cplx *psi)
{
    const int P = nqubits(m) + 2 * nt * layers;
    orc_init_basis(m, b0, psi);
    for (int k = 0; k < P; k++)
        np_apply(m, nt, np_p, np_q, k, theta[k], psi);
}

/* E and dE/dtheta of the NP circuit by the adjoint recursion (as
 * orc_energy_grad).  Returns 0 or -1 (allocation). */
int orc_np_energy_grad(const orc_model *m, int nt, const int32_t *np_p, const int32_t *np_q,
                       const double *theta, int layers, uint64_t b0, double *E, double *grad)
{
    const int n = nqubits(m);
    const uint64_t dim = (uint64_t)1 << n;
    const int P = n + 2 * nt * layers;
    cplx *psi = malloc(dim * sizeof(cplx));
    cplx *lam = malloc(dim * sizeof(cplx));
    cplx *tmp = malloc(dim * sizeof(cplx));
    if (!psi || !lam || !tmp) {
        free(psi);
        free(lam);
        free(tmp);
        return -1;
    }
    orc_np_ansatz(m, nt, np_p, np_q, theta, layers, b0, psi);
    orc_ham_apply(m, psi, lam);
    double re, im;
    orc_inner(n, psi, lam, &re, &im);
    *E = re;
    for (int k = P - 1; k >= 0 && grad; k--) {
        np_generator(m, nt, np_p, np_q, k, psi, tmp);
        orc_inner(n, lam, tmp, &re, &im);
        grad[k] = 2.0 * im;
        np_apply(m, nt, np_p, np_q, k, -theta[k], psi);
        np_apply(m, nt, np_p, np_q, k, -theta[k], lam);
    }
    free(psi);
    free(lam);
    free(tmp);
    return 0;
}
