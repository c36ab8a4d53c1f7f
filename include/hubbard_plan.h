/*
 * hubbard_plan.h -- host-only introspection and tuning of the pass schedule
 * behind include/hubbard.h.  None of these calls touches a GPU.
 *
 * A pass loads tiles of 2^k amplitudes whose index bits are k chosen qubits
 * (always including the lowest c bits of the amplitude index, for contiguous
 * loads), applies an ordered list of operations of the Eq. (7) layer (or of
 * H for the Hamiltonian passes) whose qubits all lie in the tile, and stores
 * the tiles back.  Operations keep the circuit order of Eq. (3) except where
 * they commute (hopping terms on disjoint qubit pairs; diagonal terms).
 */
#ifndef HUBBARD_PLAN_H
#define HUBBARD_PLAN_H

#include "hubbard.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Flat dump of a schedule for n_layers.  which: 0 forward passes, 1 H passes
 * (energy_grad), 2 reverse passes (energy_grad), 3 expectation passes
 * (energy).  Layout (int32): n_passes, then per pass: k, k tile bit
 * positions, flags, n_ops, then per op: kind (0 diagonal, 1 hop), param
 * (-1 for H terms), p, q (hop qubits, -1 for diagonal), umask, emask, n_v,
 * n_v V-bond indices.  *len receives the length; buf may be NULL to size it;
 * HUBBARD_ERR_SIZE if cap is too small. */
hubbard_status hubbard_plan_dump(hubbard_t h, int32_t n_layers, int32_t which, int32_t *buf,
                                 int64_t cap, int64_t *len);

/* Tile bits of forward and reverse passes (2..13) and the minimum contiguous
 * low bits c of every tile; k - c >= 2 unless k covers every qubit
 * (HUBBARD_ERR_ARG otherwise).  Drops cached device programs of the handle and
 * every planned batch that includes it (graphs captured from them must not
 * be replayed afterwards); call it before queueing work, not while work is
 * in flight. */
hubbard_status hubbard_set_tiles(hubbard_t h, int32_t fwd_k, int32_t rev_k, int32_t c);

/* Current tile configuration: cfg[0] forward k, cfg[1] reverse k, cfg[2] c. */
hubbard_status hubbard_get_tiles(hubbard_t h, int32_t *cfg);

/* Autotuner: times energy_grad (n_layers, theta_dev) for each candidate tile
 * configuration (forward k in {11,12,13}, reverse/H k in {10,11,12}, c in
 * {4,5}, clipped to the qubit count; each fixes a different fusion schedule)
 * with HIP events on `stream`, best of `reps` runs, and leaves the fastest
 * configured on the handle.  Configurations whose workspace exceeds ws_bytes
 * are skipped.  If table is not NULL it receives up to table_cap rows of
 * (fwd_k, rev_k, c) and table_ms their times; *n_tried counts the timed
 * configurations.  Allocates two small output buffers for its own runs and
 * synchronises the stream; not for use under graph capture. */
hubbard_status hubbard_tune(hubbard_t h, int32_t n_layers, const double *theta_dev, void *ws_dev,
                            size_t ws_bytes, void *stream, int32_t reps, int32_t *table,
                            int32_t table_cap, int32_t *n_tried, float *table_ms);

/* Planning parameters of later batches (energy_grad_batch): work items per
 * instance pass (a power of two in [1, 4096]; an instance's tiles are split
 * over up to that many workgroups) and stream lanes in [1, 4] (1: every
 * launch on the caller's stream; else the single-tile instances on one lane
 * of their own and the others split over lanes-1 groups by forward length).
 * A batch is planned with the values current at its first call and keyed
 * by them, so batches planned under different values coexist.  Default
 * (32, 4).  Host only; process-wide. */
hubbard_status hubbard_batch_set_config(int32_t items, int32_t lanes);
hubbard_status hubbard_batch_get_config(int32_t *items, int32_t *lanes);

/* The projected problem of hubbard_lanczos on the host: lowest eigenvalue of
 * the symmetric tridiagonal matrix with diagonal a[0..m-1] and off-diagonal
 * b[0..m-2] (Sturm-sequence bisection) and, if vec is not NULL, its unit
 * eigenvector (inverse iteration; largest component positive). */
hubbard_status hubbard_tridiag_lowest(const double *a, const double *b, int32_t m, double *lam,
                                      double *vec);

/* hubbard_vqe's optimiser on the host, driven by the caller's evaluations
 * (reverse communication): create it at x0, evaluate f and its gradient at
 * the point it returns, tell it, and repeat while *state is 0; the final
 * iterate is returned once *state is a HUBBARD_VQE_* reason. */
typedef struct hubbard_lbfgs *hubbard_lbfgs_t;
hubbard_status hubbard_lbfgs_create(const double *x0, int32_t n, const hubbard_vqe_opts *opts,
                                    hubbard_lbfgs_t *out);
hubbard_status hubbard_lbfgs_tell(hubbard_lbfgs_t L, double f, const double *g, int32_t *state,
                                  double *x_next);
hubbard_status hubbard_lbfgs_result(hubbard_lbfgs_t L, hubbard_vqe_result *res);
void hubbard_lbfgs_destroy(hubbard_lbfgs_t L);

/* Number of planned batches (energy_grad_batch) the library currently
 * keeps (at most 16). */
hubbard_status hubbard_batch_cached(int32_t *count);

/* Phase timing.  When enabled, every later call records HIP events on its own
 * stream around its phases: the forward passes, the H (or expectation)
 * passes and the reverse passes.  hubbard_phase_ms waits for the last
 * recorded event and returns the phase durations of the most recent call in
 * milliseconds (-1 for a phase that call did not have).  Not for use under
 * graph capture. */
hubbard_status hubbard_set_timing(hubbard_t h, int32_t enable);
hubbard_status hubbard_phase_ms(hubbard_t h, float *fwd_ms, float *ham_ms, float *rev_ms);

/* Per-launch timing of the pass kernel.  With timing enabled, every launch of
 * the pass kernel is bracketed by its own pair of events; this call waits for
 * them and returns, for the most recent call, the summed duration in
 * milliseconds and the number of launches of one kernel mode:
 *   mode 0 forward (gate application), 1 reverse (adjoint sweep),
 *        2 H|psi>, 3 expectation value.
 * A mode the call did not launch gives 0 ms and 0 launches. */
hubbard_status hubbard_kernel_ms(hubbard_t h, int32_t mode, float *total_ms, int32_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* HUBBARD_PLAN_H */
