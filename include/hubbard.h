/*
 * hubbard.h -- C ABI of the MI355X (gfx950) state-vector engine for the
 * Hubbard Hamiltonian-variational ansatz.
 *
 * The model is the single-band Hubbard Hamiltonian of Eq. (1) of Alvertis et
 * al., "Classical Benchmarks for Variational Quantum Eigensolver Simulations
 * of the Hubbard Model", generalised as in Eq. (2), (15) and (16) to a
 * hopping t_b and an off-site interaction V_b per nearest-neighbour bond and
 * an on-site energy eps_i per site:
 *
 *   H = sum_b sum_sigma (-t_b)(a+_{i sigma} a_{j sigma} + h.c.)
 *     + U sum_i n_{i up} n_{i dn} + sum_b V_b n_i n_j + sum_i eps_i n_i,
 *   n_i = n_{i up} + n_{i dn}, every unordered bond b = (i, j) counted once.
 *
 * The circuit is Eq. (3) with the Hamiltonian-variational layer of Eq. (7):
 * each layer applies exp(-i th_0 D) (D = every diagonal term of H: U, V, eps)
 * and then exp(-i th_g H_hop,g) for each hopping group g in order, where the
 * groups split the bonds into sets of mutually commuting terms.  Parameters
 * are layer-major: theta[l * params_per_layer + slot], slot 0 = D.
 *
 * hubbard_set_ansatz selects the number-preserving ansatz of Eq. (8)
 * instead (its parameter layout is described there).
 *
 * Encoding (Sec. 2.2.1): Jordan-Wigner with a_q = (prod_{r<q} Z_r) sigma^-_q;
 * sites are row-major s = x*ny + y; qubit q = s + nsites*spin (spin 0 = up),
 * i.e. all spin-up qubits below all spin-down qubits; bit q of an amplitude
 * index is the occupation of qubit q.  The start state is the checkerboard
 * product state of Sec. 2.1: site (x, y) holds spin up when x+y is even and
 * spin down otherwise, amplitude +1.
 *
 * State vectors are complex128 (two doubles, real then imaginary) of length
 * 2^n_qubits in device memory, at most 32 qubits.
 *
 * Conventions for every call:
 *   - Pointers whose name ends in _dev are device pointers (hipMalloc'd or
 *     from a torch CUDA/HIP tensor); all others are host pointers.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Device calls are asynchronous on that stream; the status they return
 *     reports argument and launch errors only, and a kernel fault surfaces at
 *     the caller's next synchronisation.
 *   - Vectors and scratch are caller-owned: the caller asks
 *     hubbard_workspace_size (or hubbard_batch_workspace_size) for the byte
 *     count and passes a buffer.  The only device memory the library
 *     allocates itself is small read-only tables (model constants and pass
 *     plans, KiB per handle, layer count and device; batch tables per
 *     distinct batch), uploaded on first use and kept until
 *     hubbard_destroy (batch tables: until the process ends).
 *   - Every call returns a hubbard_status; on failure hubbard_last_error()
 *     returns a message (thread-local, valid until the next call on the same
 *     thread).  No C++ exception crosses this boundary.
 *   - A handle may be used from one host thread at a time; calls that share
 *     a workspace on different streams race.
 *   - Once a call of energy (or of energy_grad) with a given handle, device
 *     and layer count has uploaded its plan, later such calls only launch
 *     kernels (no allocation, memset or synchronisation) and may be captured
 *     into a HIP graph and replayed with new theta values in place; the
 *     batch call states its own rule.
 */
#ifndef HUBBARD_H
#define HUBBARD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HUBBARD_OK = 0,
    HUBBARD_ERR_ARG = 1,     /* invalid argument (shape, range, aliasing, NULL) */
    HUBBARD_ERR_SIZE = 2,    /* workspace smaller than hubbard_workspace_size */
    HUBBARD_ERR_DEVICE = 3,  /* HIP runtime error (launch, copy, attribute) */
    HUBBARD_ERR_NOMEM = 4,   /* host or device allocation of internal tables failed */
    HUBBARD_ERR_STATE = 5    /* call not valid for this handle (e.g. destroyed) */
} hubbard_status;

typedef struct hubbard_model *hubbard_t;

/* Lattice model, Eq. (1)/(2)/(15)/(16).  All pointers are host pointers,
 * read during hubbard_create only.
 *   nx, ny          rows and columns (a chain is nx = 1); 1 <= nx*ny <= 16.
 *   periodic_x/_y   nonzero: wrap bond between the last and first row/column;
 *                   needs that length >= 3 (and even with default groups).
 *   t_bond          n_bonds hoppings in canonical bond order (NULL: all 1).
 *   U               on-site interaction.
 *   V_bond          n_bonds nearest-neighbour interactions (NULL: all 0).
 *   eps_site        nx*ny on-site energies (NULL: all 0).
 *   bond_group      n_bonds group ids >= 0 (NULL: default rule); groups are
 *                   applied in increasing id, empty ids skipped, and each
 *                   group must be a matching (no site in two of its bonds).
 *
 * Canonical bond order: every horizontal bond (x,y)-(x,y+1) by start site
 * row-major, the periodic wrap (x,ny-1)-(x,0) right after its row; then every
 * vertical bond (x,y)-(x+1,y) by start site row-major, wraps (nx-1,y)-(0,y)
 * last.  Default groups (the commuting split of Eq. (7) into h1, v1, h2, v2):
 * horizontal bonds by the parity of the start column, vertical bonds by the
 * parity of the start row; a direction of length 2 whose transverse length is
 * >= 3 splits by the transverse parity instead. */
typedef struct {
    int32_t nx, ny;
    int32_t periodic_x, periodic_y;
    const double *t_bond;
    double U;
    const double *V_bond;
    const double *eps_site;
    const int32_t *bond_group;
} hubbard_desc;

/* Build a model handle from a lattice description (host only; no GPU work).
 * Errors: HUBBARD_ERR_ARG for an invalid lattice, a non-matching group, more
 * than 32 qubits or a non-finite coefficient; HUBBARD_ERR_NOMEM. */
hubbard_status hubbard_create(const hubbard_desc *desc, hubbard_t *out);

/* The same model on an arbitrary graph of sites (Eq. (2)/(15)/(16) with any
 * set of bonds, e.g. other lattices or boundary conditions).  All pointers
 * are host pointers, read during hubbard_create_graph only.
 *   n_sites         1 <= n_sites <= 16 (qubit q = site + n_sites * spin)
 *   n_bonds         0 <= n_bonds <= 64
 *   bond_i, bond_j  the sites of each bond (distinct, in range; an unordered
 *                   pair may appear once); this is the bond order of t_bond,
 *                   V_bond and bond_group
 *   t_bond, V_bond, eps_site, U   as in hubbard_desc (NULL: t = 1, V = 0,
 *                   eps = 0)
 *   bond_group      group ids >= 0, each group a matching, applied in
 *                   increasing id (NULL: in bond order each bond joins the
 *                   lowest group that has neither of its sites yet)
 *   site_spin       start state: site s holds one electron of spin
 *                   site_spin[s] (0 up, 1 down); NULL: up on even sites,
 *                   down on odd ones
 * Errors: HUBBARD_ERR_ARG (a bad or repeated bond, a non-matching group, a
 * bad spin, a non-finite coefficient), HUBBARD_ERR_NOMEM. */
typedef struct {
    int32_t n_sites, n_bonds;
    const int32_t *bond_i, *bond_j;
    const double *t_bond;
    double U;
    const double *V_bond;
    const double *eps_site;
    const int32_t *bond_group;
    const int32_t *site_spin;
} hubbard_graph_desc;

hubbard_status hubbard_create_graph(const hubbard_graph_desc *desc, hubbard_t *out);

/* The ansatz of the circuit (every later call that applies it):
 *   HUBBARD_ANSATZ_HVA (default)  the Hamiltonian-variational layer of
 *       Eq. (7): params_per_layer = 1 + n_groups, no leading parameters.
 *   HUBBARD_ANSATZ_NP  the number-preserving ansatz of Eq. (8) (Sec. 2.2.1):
 *       before the first layer R_z on every qubit, applied as the phase gate
 *       exp(i th n_q) (R_z up to a global phase, which changes no energy,
 *       gradient or overlap magnitude); then per layer one
 *       U_NP(theta, phi) = exp(i theta (a+_p a_q + a+_q a_p)) exp(i phi n_p n_q)
 *       (the matrix of Eq. (8) in Jordan-Wigner form, the fermionic swaps
 *       of the paper's circuit supplied by the string sign) on every pair
 *       of qubits that a term of Eq. (1) couples: the up and down qubits of
 *       every site (in site order), then every bond of every hopping group
 *       in group and bond order, spin up then spin down.  Parameters:
 *       n_qubits R_z angles, then per layer (theta, phi) of each term in
 *       that order: params_per_layer = 2 (n_sites + 2 n_bonds).
 * The parameter count of n_layers is hubbard_param_count (energy,
 * energy_grad, the batch and the optimiser use it).  Drops the handle's
 * plans and every planned batch that includes it (like hubbard_set_tiles). */
enum { HUBBARD_ANSATZ_HVA = 0, HUBBARD_ANSATZ_NP = 1 };
hubbard_status hubbard_set_ansatz(hubbard_t h, int32_t ansatz);
hubbard_status hubbard_param_count(hubbard_t h, int32_t n_layers, int64_t *count);

/* Release the handle and its device tables (synchronises nothing; the caller
 * must not destroy a handle with work still queued on a stream). */
void hubbard_destroy(hubbard_t h);

/* Host-side description of the handle.  Any out pointer may be NULL. */
hubbard_status hubbard_query(hubbard_t h, int32_t *n_qubits, int32_t *n_bonds,
                             int32_t *n_groups, int32_t *params_per_layer,
                             uint64_t *neel_index);

/* Bond list in canonical order: sites bi[b], bj[b] and the 0-based group slot
 * (application order) of each bond; each array holds n_bonds entries. */
hubbard_status hubbard_bonds(hubbard_t h, int32_t *bi, int32_t *bj, int32_t *group);

const char *hubbard_last_error(void);

/* Operations for hubbard_workspace_size. */
enum {
    HUBBARD_OP_ENERGY = 0,       /* energy():      psi + reduction partials */
    HUBBARD_OP_ENERGY_GRAD = 1,  /* energy_grad(): psi + lambda + partials */
    HUBBARD_OP_OVERLAP = 2,      /* hubbard_overlap(): partial sums (hubbard_vector_workspace_size) */
    HUBBARD_OP_LANCZOS = 3,      /* hubbard_lanczos(): three vectors + partial sums (same) */
    HUBBARD_OP_OVERLAP_GRAD = 4, /* overlap_grad(): as energy_grad + overlap partials */
    HUBBARD_OP_SPIN_CORR = 5     /* hubbard_spin_correlation(): moment partials (vector size call) */
};

/* Bytes of device workspace needed by energy()/energy_grad() for n_layers. */
hubbard_status hubbard_workspace_size(hubbard_t h, int32_t n_layers, int32_t op,
                                      size_t *bytes);

/* psi_dev <- checkerboard start state |b0> (2^n complex128 written). */
hubbard_status hubbard_init_neel(hubbard_t h, void *psi_dev, void *stream);

/* Eq. (3)/(7): psi_dev <- U_P(theta_P) ... U_1(theta_1) psi_dev, in place on a
 * caller-owned vector of 2^n complex128.  theta_dev holds
 * n_layers * params_per_layer doubles in device memory.  n_layers >= 0. */
hubbard_status ansatz_apply(hubbard_t h, const double *theta_dev, int32_t n_layers,
                            void *psi_dev, void *stream);

/* Matrix-free H|psi> (Eq. (4)'s operator): out_dev <- H psi_dev.  Both are
 * 2^n complex128; out_dev must not overlap psi_dev (HUBBARD_ERR_ARG). */
hubbard_status hamiltonian_apply(hubbard_t h, const void *psi_dev, void *out_dev,
                                 void *stream);

/* Eq. (4): E_dev[0] <- <psi(theta)|H|psi(theta)> with psi(theta) prepared
 * from the start state |b0> in the workspace (the workspace's contents on
 * entry are not read).  ws_dev must hold
 * hubbard_workspace_size(..., HUBBARD_OP_ENERGY) bytes (HUBBARD_ERR_SIZE). */
hubbard_status energy(hubbard_t h, const double *theta_dev, int32_t n_layers,
                      double *E_dev, void *ws_dev, size_t ws_bytes, void *stream);

/* Energy and its gradient by the adjoint recursion of Sec. 2.1:
 * grad_dev[k] = dE/dtheta_k = 2 Im <lambda_k| G_k |psi_k> for all
 * P = n_layers * params_per_layer parameters, computed in one reverse sweep
 * that un-applies the gates to psi and lambda = H psi in the workspace.
 * ws_dev must hold hubbard_workspace_size(..., HUBBARD_OP_ENERGY_GRAD); its
 * contents on entry are not read, and on return they are scratch (psi and
 * lambda are kept there in a layout of the library's own). */
hubbard_status energy_grad(hubbard_t h, const double *theta_dev, int32_t n_layers,
                           double *E_dev, double *grad_dev, void *ws_dev,
                           size_t ws_bytes, void *stream);

/* Bytes of device workspace for hubbard_overlap (op HUBBARD_OP_OVERLAP: 16
 * KiB of partial sums) or hubbard_lanczos (HUBBARD_OP_LANCZOS: three state
 * vectors and the partial sums). */
hubbard_status hubbard_vector_workspace_size(hubbard_t h, int32_t op, size_t *bytes);

/* Overlap of two state vectors of the handle's size, as in the fidelity
 * F = |<Psi_VQE|Psi_ref>|^2 of Sec. 3.4: out_dev[0] + i out_dev[1] =
 * <a|b> = sum_x conj(a_x) b_x over all 2^n amplitudes (device doubles),
 * summed in a fixed order (reproducible).  Asynchronous on `stream`. */
hubbard_status hubbard_overlap(hubbard_t h, const void *a_dev, const void *b_dev, double *out_dev,
                               void *ws_dev, size_t ws_bytes, void *stream);

/* Lowest eigenvalue of H (Eq. (1)/(2)/(15)/(16)) in the Krylov space of a
 * start vector, by the Lanczos recurrence on hamiltonian_apply: the
 * reference ground state that the VQE error per site of Sec. 3.1 and the
 * fidelity of Sec. 3.4 are measured against (the paper uses DMRG).  H keeps
 * N_up and N_dn, so a start vector inside one particle-number sector (for
 * example the checkerboard state after any circuit of Eq. (7)) gives that
 * sector's ground state, and every amplitude outside it stays exactly zero.
 *   start_dev  2^n complex128, any nonzero norm; not modified
 *   max_iter   most Lanczos steps (each one H application, two vector
 *              passes and one host synchronisation)
 *   tol        stop when the Ritz residual ||H x - E0 x|| = beta_j |s_j|
 *              (s: lowest eigenvector of the projected tridiagonal matrix)
 *              is below tol * max(1, |E0|), or at an invariant subspace
 *   E0, iters, residual   host outputs (iters, residual may be NULL)
 *   gs_dev     NULL, or 2^n complex128 receiving the unit Ritz vector x (a
 *              second run of the recurrence with the stored coefficients)
 *   ws_dev     hubbard_vector_workspace_size(HUBBARD_OP_LANCZOS) bytes; the
 *              start and state vectors must not overlap it
 * Synchronises `stream` at every step (the projected problem is solved on
 * the host); not for graph capture.  No reorthogonalisation: the lowest
 * Ritz value converges before orthogonality loss matters. */
hubbard_status hubbard_lanczos(hubbard_t h, const void *start_dev, int32_t max_iter, double tol,
                               double *E0, int32_t *iters, double *residual, void *gs_dev,
                               void *ws_dev, size_t ws_bytes, void *stream);

/* The overlap loss of Eq. (5)/(6) and its gradient: with F(theta) =
 * |<ref|psi(theta)>|^2, out_dev[0] = f = log10(1 - F) and out_dev[1] = F,
 * grad_dev[k] = df/dtheta_k = -(dF/dtheta_k) / ((1 - F) ln 10).  F is the
 * expectation of the projector P = |ref><ref|, so dF/dtheta_k comes from
 * energy_grad's reverse sweep seeded with lambda = P psi = <ref|psi> ref
 * instead of H psi (the intermediate states of Sec. 2.1, one reduction per
 * parameter).  ref_dev: 2^n complex128 of unit norm (caller-owned, not
 * overlapping the workspace); ws_dev: hubbard_workspace_size(...,
 * HUBBARD_OP_OVERLAP_GRAD) bytes.  F = 1 gives f = -inf.  Asynchronous. */
hubbard_status overlap_grad(hubbard_t h, const double *theta_dev, int32_t n_layers,
                            const void *ref_dev, double *out_dev, double *grad_dev, void *ws_dev,
                            size_t ws_bytes, void *stream);

/* Spin correlations of Eq. (17) of a state vector: C_dev[i * n_sites + j] =
 * <S^z_i S^z_j> - <S^z_i><S^z_j> and Sz_dev[i] = <S^z_i>, S^z_i =
 * (n_i,up - n_i,dn) / 2 (device doubles), from one read of psi_dev: the
 * occupation second moments sum_x |psi_x|^2 n_a(x) n_b(x) over all qubit
 * pairs, in a fixed order.  ws_dev: hubbard_vector_workspace_size(...,
 * HUBBARD_OP_SPIN_CORR) bytes.  Asynchronous. */
hubbard_status hubbard_spin_correlation(hubbard_t h, const void *psi_dev, double *C_dev,
                                        double *Sz_dev, void *ws_dev, size_t ws_bytes,
                                        void *stream);

/* The VQE optimisation of Sec. 2.1: minimise E(theta) = <psi(theta)|H|psi(theta)>
 * by L-BFGS (limited-memory BFGS, strong-Wolfe line search) on energy_grad
 * evaluations, stopping when the energy changes by less than e_tol between
 * consecutive iterates, the gradient's Euclidean norm is below g_tol, or
 * after max_steps iterations (the paper: 1e-7, 1e-6, 1000).  The paper runs
 * ten optimisations from random starts and keeps the lowest energy; here
 * n_starts > 1 advances that many independent optimisations of the same
 * model in lockstep, every round one energy_grad_batch launch for all of
 * them (finished ones are evaluated at their final point).
 *   theta_dev   n_starts * n_layers * params_per_layer doubles (device):
 *               in: the start points, out: each optimisation's final iterate
 *   opts        NULL: the paper's settings (history 10)
 *   results     n_starts entries (host): final energy, gradient norm,
 *               iterations, evaluations, stopping reason
 *   ws_dev      hubbard_vqe_workspace_size bytes
 * Synchronises `stream` at every round (the optimiser runs on the host). */
typedef struct {
    int32_t max_steps;   /* iterations (1000) */
    int32_t history;     /* (s, y) pairs kept (10) */
    double e_tol;        /* |E_k - E_{k-1}| (1e-7) */
    double g_tol;        /* ||grad||_2 (1e-6) */
} hubbard_vqe_opts;

enum {
    HUBBARD_VQE_RUNNING = 0,
    HUBBARD_VQE_ENERGY_TOL = 1,
    HUBBARD_VQE_GRAD_TOL = 2,
    HUBBARD_VQE_MAX_STEPS = 3,
    HUBBARD_VQE_LINE_SEARCH = 4,   /* no acceptable step: a local minimum to rounding */
    HUBBARD_VQE_NOT_FINITE = 5
};

typedef struct {
    double E;            /* energy at the final iterate */
    double grad_norm;    /* its gradient's Euclidean norm */
    int32_t steps;       /* L-BFGS iterations */
    int32_t evals;       /* energy+gradient evaluations */
    int32_t reason;      /* HUBBARD_VQE_* */
    int32_t pad;
} hubbard_vqe_result;

hubbard_status hubbard_vqe_workspace_size(hubbard_t h, int32_t n_layers, int32_t n_starts,
                                          size_t *bytes);
hubbard_status hubbard_vqe(hubbard_t h, int32_t n_layers, int32_t n_starts, double *theta_dev,
                           const hubbard_vqe_opts *opts, hubbard_vqe_result *results,
                           void *ws_dev, size_t ws_bytes, void *stream);

/* energy_grad for callers that cannot allocate device memory or pass a
 * workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same kernels and results as energy_grad, with
 * psi, lambda and the reduction partials in a 48 MiB array that the library
 * holds in every device's memory from its load until the process ends.
 * It allocates nothing, creates no events and synchronises nothing.
 *   - At most 20 qubits and 128 reduction rows (the circuits of up to 20
 *     qubits used here have fewer than 70); larger: HUBBARD_ERR_SIZE.
 *   - The handle's plan for this device and layer count must already be
 *     uploaded by one earlier energy_grad call (HUBBARD_ERR_STATE
 *     otherwise).
 *   - Every call on a device shares that device's array and keeps the last
 *     call's contents; each call writes the parts it reads before reading
 *     them.  Calls that overlap on one device (other streams, other host
 *     threads) race. */
hubbard_status energy_grad_noalloc(hubbard_t h, const double *theta_dev, int32_t n_layers,
                                   double *E_dev, double *grad_dev, void *stream);

/* Batched energy and gradient of many independent instances (different
 * lattices, sizes, U, disorder, V and layer counts; each its own parameters)
 * with no host work per call: a fixed sequence of launches on `stream` --
 * for each position j of the forward, H and reverse schedules, launches that
 * run pass j of every instance that has one (two: passes whose tiles fill the
 * workgroup's registers exactly, and the others; a large instance's tiles
 * spread over many workgroups; the first forward passes build the start
 * states themselves), then one reduction of the partial sums into E and the
 * gradients, in a fixed order (results are reproducible run to run).  The
 * instances are split into lanes by schedule length (those that fit one
 * tile, and groups of shorter forward schedules); each lane's launches run
 * on a stream of the library's own, forked from `stream` by an event and
 * joined back before the reduction, so that a lane that has finished its
 * forward runs its H and reverse passes while longer ones still run
 * theirs; under graph capture every branch is recorded.  psi and lambda in
 * the workspace are scratch: an instance's last reverse pass does not
 * store them.
 *   hs[i]           instance handles (n >= 1)
 *   theta_dev       all parameters, instance i's n_layers[i]*params_per_layer
 *                   values starting at theta_dev + theta_off[i] (device)
 *   theta_off, n_layers  host arrays of n entries
 *   E_dev[i]        energy of instance i (device, n doubles)
 *   grad_dev        gradient of instance i at grad_dev + theta_off[i] (device)
 *   ws_dev          hubbard_batch_workspace_size bytes (device): each
 *                   instance's psi and lambda, then the partial sums
 * The first call with a given set of handles, layer counts, offsets, theta
 * and workspace pointers plans the batch and uploads its tables (it must not
 * be under graph capture); later calls only launch kernels, allocate
 * nothing, and may be captured into a graph and replayed with new theta
 * values in place.
 * Lifetime of a planned batch: it is keyed by each handle's identity (a
 * number never given to another handle, not its address) and tile
 * configuration, so a batch of new handles never reuses an old plan.  It
 * points into its members' device tables, so hubbard_destroy,
 * hubbard_set_tiles or hubbard_tune of any member discards it (after
 * waiting for the device to go idle), and at most 16 planned batches are
 * kept: planning a 17th discards the least recently called one.  A graph
 * captured from a discarded batch -- or an energy/energy_grad graph
 * captured before hubbard_set_tiles or hubbard_tune of its handle -- must
 * not be replayed; the next eager call plans again.
 * Errors: HUBBARD_ERR_ARG, HUBBARD_ERR_SIZE (workspace), HUBBARD_ERR_STATE
 * (first call under capture), HUBBARD_ERR_DEVICE. */
hubbard_status hubbard_batch_workspace_size(const hubbard_t *hs, int32_t n,
                                            const int32_t *n_layers, size_t *bytes);
hubbard_status energy_grad_batch(const hubbard_t *hs, int32_t n, const double *theta_dev,
                                 const int64_t *theta_off, const int32_t *n_layers,
                                 double *E_dev, double *grad_dev, void *ws_dev, size_t ws_bytes,
                                 void *stream);

/* ---- Particle-number sector form of the HVA circuit ----------------------
 * H (Eq. (1)/(2)/(15)/(16)) and every gate of the Eq. (7) layer keep N_up and
 * N_dn, so the circuit state prepared from the checkerboard start |b0> of
 * Sec. 2.1 has nonzero amplitudes only on the basis states with b0's
 * (N_up, N_dn).  These calls store only those amplitudes: a sector vector
 * holds C(Ns, N_dn) x C(Ns, N_up) complex128 values, element
 * r_dn * C(Ns, N_up) + r_up for the basis state whose spin-down site
 * pattern has rank r_dn and spin-up pattern rank r_up (rank: position among
 * the site patterns with that many electrons, in increasing numeric order;
 * site i is bit i, as qubit i / Ns + i of the full vector).  At 4x4 half
 * filling that is 12870^2 = 1.66e8 amplitudes (2.6 GB) instead of 2^32
 * (64 GiB).  The results equal those of the full-vector calls on the same
 * model and parameters (the amplitudes outside the sector are exactly zero
 * there).  HVA circuit only: a handle switched to the NP ansatz (whose
 * on-site gates change N_up and N_dn) gives HUBBARD_ERR_STATE.
 * Layout: each spin's gates act along the rows of the matrix whose columns
 * that spin indexes; between runs of gates of the two spins the state is
 * transposed through LDS tiles (a workspace copy).  All calls are
 * asynchronous on `stream`; the first call per handle, device and layer
 * count builds and uploads the sector's tables (pair slots and
 * Jordan-Wigner signs per gate and rank: 4 bytes x ranks x bonds x 2). */
enum {
    HUBBARD_SECTOR_ANSATZ = 0,        /* sector_ansatz_apply: one sector vector */
    HUBBARD_SECTOR_ENERGY_GRAD = 1,   /* sector_energy_grad: four vectors + partial sums */
    HUBBARD_SECTOR_HAMILTONIAN = 2,   /* sector_hamiltonian_apply: two vectors */
    HUBBARD_SECTOR_LANCZOS = 3        /* hubbard_sector_lanczos: five vectors + partial sums */
};

/* C(Ns, N_up) and C(Ns, N_dn) of the handle's start state (host outputs). */
hubbard_status hubbard_sector_dim(hubbard_t h, int64_t *n_up, int64_t *n_dn);

/* Device workspace bytes of a sector call (op HUBBARD_SECTOR_*). */
hubbard_status hubbard_sector_workspace_size(hubbard_t h, int32_t n_layers, int32_t op,
                                             size_t *bytes);

/* psi_dev (a sector vector) <- |b0>. */
hubbard_status hubbard_sector_init_neel(hubbard_t h, void *psi_dev, void *stream);

/* Eq. (3)/(7) on a sector vector, in place: psi_dev <- U(theta) psi_dev.
 * theta_dev: n_layers * params_per_layer doubles (device); ws_dev:
 * hubbard_sector_workspace_size(HUBBARD_SECTOR_ANSATZ) bytes, not
 * overlapping psi_dev. */
hubbard_status sector_ansatz_apply(hubbard_t h, const double *theta_dev, int32_t n_layers,
                                   void *psi_dev, void *ws_dev, size_t ws_bytes, void *stream);

/* out_dev <- H psi_dev on sector vectors (distinct, else HUBBARD_ERR_ARG);
 * ws_dev: HUBBARD_SECTOR_HAMILTONIAN bytes, overlapping neither. */
hubbard_status sector_hamiltonian_apply(hubbard_t h, const void *psi_dev, void *out_dev,
                                        void *ws_dev, size_t ws_bytes, void *stream);

/* energy_grad in the sector form: E_dev[0] = <psi(theta)|H|psi(theta)> and
 * grad_dev[k] = 2 Im <lambda_k|G_k|psi_k> (Sec. 2.1) for all
 * n_layers * params_per_layer parameters, psi(theta) prepared from |b0> and
 * the reverse sweep un-applying the gates to psi and lambda = H psi, one
 * reduction per gate into its parameter (fixed order: reproducible).  The
 * workspace (HUBBARD_SECTOR_ENERGY_GRAD bytes) is scratch. */
hubbard_status sector_energy_grad(hubbard_t h, const double *theta_dev, int32_t n_layers,
                                  double *E_dev, double *grad_dev, void *ws_dev, size_t ws_bytes,
                                  void *stream);

/* hubbard_lanczos on sector vectors: the lowest eigenvalue of H (Eq.
 * (1)/(2)/(15)/(16)) in the sector of the handle's start state, the
 * reference ground state of Sec. 2.1/3.1/3.4, by the same Lanczos recurrence
 * (same stopping rule, same arithmetic order) with sector_hamiltonian_apply
 * as H.  start_dev and gs_dev (NULL or the unit Ritz vector) are sector
 * vectors; ws_dev: HUBBARD_SECTOR_LANCZOS bytes (three Krylov vectors, H's
 * two layout-B vectors, partial sums), overlapping neither.  Synchronises
 * `stream` at every step. */
hubbard_status hubbard_sector_lanczos(hubbard_t h, const void *start_dev, int32_t max_iter,
                                      double tol, double *E0, int32_t *iters, double *residual,
                                      void *gs_dev, void *ws_dev, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HUBBARD_H */
