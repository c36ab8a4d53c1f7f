// hubvqe.hpp -- internal structures shared by the host runtime (model.cpp,
// plan.cpp, engine.hip) and the gfx950 kernels.  Not part of the public ABI
// (include/hubbard.h is).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#if !defined(__HIPCC__)
#define __host__
#define __device__
#endif

namespace hv {

constexpr int kMaxSites = 16;
constexpr int kMaxQubits = 32;
constexpr int kMaxBonds = 64;
constexpr int kMaxTileBits = 13;
constexpr int kMaxOpsPerPass = 96;
constexpr int kMaxDiagPerPass = 32;
constexpr int kMaxRedPerPass = 12;
constexpr int kDiagTab = kMaxSites + 1;   // U-count phase table entries

enum OpKind : int32_t {
    OP_DIAG = 0,   // diagonal sub-term: U and eps of a set of sites, V of a set of bonds
    OP_HOP = 1,    // one hopping term (a+_p a_q + h.c.) of one bond and spin
    OP_MASK = 2    // diagonal coef * [every qubit of a mask occupied] (NP phases, R_z)
};

// Op kinds a pass kernel decodes (a template argument of the pass kernels).
enum OpSet : int {
    OPS_HVA = 0,   // OP_HOP, OP_DIAG: the HVA circuit, H and expectations
    OPS_NP = 1,    // OP_HOP, OP_MASK: gate passes of the NP circuit
    OPS_ALL = 2    // all three: gate passes of a batch with NP instances
};

enum PassFlags : int32_t {
    PF_HAM_FIRST = 1,   // H pass: phi <- D psi + terms (else phi += terms)
    PF_HAM_LAST = 2,    // H pass: also reduce Re <psi|phi> into row 0
    // never planned; set on a launch's copy of a pass (single state) or in a
    // batch's own pass array:
    PF_FROM_START = 4,  // forward pass: the input is the start state |b0>, not read
    PF_NO_STORE = 8,    // reverse pass: the vectors are not needed afterwards
};

// One device operation inside a pass (64 bytes).  The fields a hopping term
// needs in the inner loop come first, so one 32-byte scalar load fetches them.
struct DevOp {
    int32_t kind;
    int32_t pair;       // HOP: register-bit pair (0..5: 01 02 03 12 13 23) in its phase
    uint32_t flip;      // HOP: bit j = parity of register j's global bits in `between`
    uint32_t between;   // HOP: global bits strictly between p and q (Jordan-Wigner string);
                        // MASK: the global bits that must all be set
    int32_t red;        // reduction row within the pass (-1: none)
    int32_t dtab;       // DIAG: index of its phase table within the pass
    double t;           // HOP: bond hopping t_b; MASK: coefficient
    int32_t param;      // theta index (-1 for Hamiltonian terms)
    uint32_t umask;     // DIAG: spin-up qubits of the sites whose U term it carries
    uint32_t emask;     // DIAG: qubits whose eps term it carries
    int32_t v_begin;    // DIAG: V bonds [v_begin, v_end) of the plan's V table
    int32_t v_end;
    int32_t pad[3];
};
static_assert(sizeof(DevOp) == 64, "DevOp layout");

// LDS slot of tile-local index l in the exchange buffer: the high bits are
// l's, the low four bits are A (l & 15) XOR a 4-bit mask per set bit 4..12
// of l, with A an invertible 4 x 4 matrix over GF(2) (its columns in bits
// 4..19 of s1) and the masks in nibble b - 4 of s0 (bits 4..11) and bits
// 0..3 of s1 (bit 12), chosen per pass so that the 16-byte slots a wave
// touches in one access spread over the banks.  Linear over GF(2), hence a
// bijection on [0, 2^k), and slot(a ^ b) = slot(a) ^ slot(b).
__host__ __device__ inline uint32_t slot(uint32_t l, uint32_t s0, uint32_t s1)
{
    uint32_t f = ((l >> 12) & 1u) ? (s1 & 15u) : 0u;
#pragma unroll
    for (int b = 0; b < 4; ++b)
        if ((l >> b) & 1u)
            f ^= (s1 >> (4 + 4 * b)) & 15u;
#pragma unroll
    for (int b = 4; b < 12; ++b)
        if ((l >> b) & 1u)
            f ^= (s0 >> (4 * (b - 4))) & 15u;
    return (l & ~15u) | f;
}

// Register layout of one phase of a pass (64 bytes).  Each thread holds 16
// amplitudes of the tile in registers: register j holds tile-local index
// tloc | pdep(j, register bits), where tloc deposits the lane id over lmask
// and the wave id over wmask.  Because the deposit and slot() are linear,
// register j's global-index bits are the OR of gb[i] over the set bits i of
// j, and its LDS byte offset is slot(tloc) * 16 XOR the XOR of sb[i].  Gates
// of the phase act on register bits only; between phases the tile is
// re-laid out through LDS.
constexpr int kRegs = 16;
constexpr int kRegBits = 4;
struct DevPhase {
    int32_t op_begin, op_end;   // ops of this phase (pass-relative indices)
    uint32_t gb[kRegBits];      // global index bit of register bit i (0: phantom bit)
    uint32_t sb[kRegBits];      // slot(tile-local bit of register bit i) * 16
    uint32_t lmask;             // tile-local bits that carry the lane id (ascending)
    uint32_t wmask;             // tile-local bits that carry the wave id (ascending)
    uint32_t valid;             // bit j: register j holds an amplitude (tiles < 16)
    uint32_t cross;             // 1: entering this phase moves data between waves
    int32_t pad[2];
};
static_assert(sizeof(DevPhase) == 64, "DevPhase layout");

// A class of V bonds of one diagonal op, as the device reads it: the bonds
// (i, i + delta) for every site i set in src, all with the same V.  With the
// site occupation bit sets U (spin up) and D (spin down), the class adds
// V * sum over its bonds of n_i n_j = V * (popc(U & U') + popc(U & D') +
// popc(D & U') + popc(D & D')), X' = X shifted down by delta, masked by src.
struct DevVBond {
    uint32_t src;
    int32_t delta;
    double V;
};
static_assert(sizeof(DevVBond) == 16, "DevVBond layout");

// Pass descriptor, passed by value as a kernel argument.
struct DevPass {
    int32_t k;          // tile bits
    int32_t c;          // tile bits 0..c-1 are global bits 0..c-1 (coalesced run)
    int32_t nfree;      // n - k
    int32_t op_begin;   // first op in the plan's op array
    int32_t n_ops;
    int32_t n_diag;     // DIAG ops (phase tables) in this pass
    int32_t red_base;   // first partial row of this pass
    int32_t n_red;      // partial rows written by this pass
    int32_t flags;
    int32_t phase_begin;   // first phase in the plan's phase array
    int32_t n_phases;      // phases (the first and last are the load/store layouts)
    int32_t tbits;         // thread-id bits: a workgroup has 2^tbits threads
    uint32_t hi_mask;      // global bits of tile bits c..k-1 (tile bits 0..c-1 = global 0..c-1)
    uint32_t free_mask;    // global bits not in the tile (the tile id is deposited here)
    uint32_t swz[2];       // slot() masks of the tile-local bits 0..12 (bank spreading)
};

// One instance of a batched energy+gradient evaluation: its model tables,
// parameters and state vectors (every pointer is a device pointer).
struct DevInstance {
    int32_t general;        // diagonal has eps or V terms
    int32_t pad;
    const struct DevPhase *phases;
    const struct DevOp *ops;
    const struct DevVBond *vb;
    const struct DevModel *model;
    const double *theta;
    void *psi, *lam;
};

// One work item of a batched pass launch: tiles [tile0, tile1) of pass
// `pass` of instance `inst`; its reduction row r goes to
// partial[part + r * stride].
struct DevWork {
    int32_t inst, pass;
    uint32_t tile0, tile1;
    int64_t part;
    int32_t stride, pad;
};
static_assert(sizeof(DevWork) == 32, "DevWork layout");

// Model constants in device memory.
struct DevModel {
    int32_t n, ns;
    int32_t general;        // 0: D = U * (#doubly occupied sites) only
    uint32_t b0;            // index of the start state (Neel configuration)
    double U;
    double eps_q[kMaxQubits];   // on-site energy of each qubit's site (0 beyond n)
};

// LDS carve-up shared by host (launch size) and device: one tile-sized
// exchange buffer, per-phase lane and wave tables (global bits and LDS byte
// offset of each lane's and each wave's part of the tile-local index),
// per-op rotation coefficients, diagonal phase tables and reduction rows.
constexpr int kMaxWaves = 8;   // 512 threads
struct SmemPlan {
    uint32_t xbuf, ltab, wtab, opc, dtab, etab, cis, red, rows, total;
};

// Reduction rows: a pass over many tiles keeps one accumulator per row and
// group of four lanes (the four are summed in registers first; one per
// thread below four threads); a single-tile pass reduces every op at once
// into one value per row.
__host__ __device__ inline uint32_t red_rows_per(int threads, bool single_tile)
{
    return single_tile ? 1u : (threads >= 4 ? (uint32_t)threads / 4u : (uint32_t)threads);
}

// General diagonal (eps or V terms): per diag op eight nibble tables of the
// eps sum over its qubits, and one table of 2^kCisBits unit phases shared by
// all ops of the pass.
constexpr int kCisBits = 8;

__host__ __device__ inline SmemPlan smem_plan(int k, int n_ops, int n_diag, int n_red,
                                              int n_phases, int threads, bool single_tile,
                                              bool general)
{
    SmemPlan s;
    uint32_t at = 0;
    s.xbuf = at;
    at += (1u << k) * 16u;
    s.ltab = at;
    at += (uint32_t)n_phases * 64u * 8u;
    s.wtab = at;
    at += (uint32_t)n_phases * kMaxWaves * 8u;
    s.opc = at;
    at += (uint32_t)n_ops * 16u;
    s.dtab = at;
    at += (uint32_t)n_diag * kDiagTab * 16u;
    s.etab = at;
    s.cis = at + (general ? (uint32_t)n_diag * 8u * 16u * 8u : 0u);
    if (general && n_diag > 0)
        at = s.cis + (1u << kCisBits) * 16u;
    s.red = at;
    s.rows = red_rows_per(threads, single_tile);
    at += (uint32_t)n_red * s.rows * 8u;
    at += 16u * 8u;   // per-wave partial sums
    s.total = at;
    return s;
}

// Vector kernels (k_vdot and friends): threads per block and the most blocks
// a launch uses (also the number of reduction partials).
constexpr int kVecThreads = 256;
constexpr int kVecBlocks = 1024;
// Occupation moments (k_bit_moments): a workgroup covers 2^(LO+MID)
// amplitudes, LO <= kMomLo bits from the thread id, MID <= kMomMid from a loop.
constexpr int kMomLo = 8;
constexpr int kMomMid = 10;

// ------------------------------------------------------------------ host --

struct Model {
    int nx = 0, ny = 0, px = 0, py = 0;
    int ns = 0, nq = 0, nb = 0, ngroups = 0;
    std::vector<int> bi, bj, slot;   // slot: 1..ngroups (application order)
    std::vector<double> t, V, eps;
    double U = 0.0;
    uint64_t neel = 0;
    bool general = false;            // any eps or V nonzero
    int ansatz = 0;                  // 0: HVA layer of Eq. (7); 1: NP ansatz of Eq. (8)
    int qubit(int site, int spin) const { return site + ns * spin; }
    // NP: one U_NP(theta, phi) per on-site pair and per bond and spin
    int np_terms() const { return ns + 2 * nb; }
    int params_per_layer() const { return ansatz == 1 ? 2 * np_terms() : 1 + ngroups; }
    // NP: R_z angles of every qubit before the first layer
    int lead_params() const { return ansatz == 1 ? nq : 0; }
    int n_params(int layers) const { return lead_params() + layers * params_per_layer(); }
};

// Lowest eigenvalue of the symmetric tridiagonal matrix with diagonal
// a[0..m-1] and off-diagonal b[0..m-2] (Sturm-sequence bisection); if vec is
// not NULL it receives the unit eigenvector (inverse iteration, largest
// component positive).  m >= 1.
double tridiag_lowest(const double *a, const double *b, int m, double *vec);

// L-BFGS with a strong-Wolfe line search as a reverse-communication state
// machine (lbfgs.cpp): construct with the start point, evaluate trial(),
// pass the value and gradient to tell(); repeat while it returns
// LBFGS_EVALUATE.  x() is the current iterate, trial() the point to
// evaluate next (the final iterate once finished).
enum LbfgsStatus {
    LBFGS_EVALUATE = 0,
    LBFGS_ENERGY_TOL = 1,   // |E_k - E_{k-1}| < e_tol
    LBFGS_GRAD_TOL = 2,     // ||g||_2 < g_tol
    LBFGS_MAX_STEPS = 3,
    LBFGS_LINE_SEARCH = 4,  // no acceptable step along the search direction
    LBFGS_NOT_FINITE = 5    // the start point's value or gradient is not finite
};
struct LbfgsOptions {
    int max_steps = 1000;
    int history = 10;
    double e_tol = 1e-7;
    double g_tol = 1e-6;
};
class Lbfgs {
  public:
    Lbfgs(const double *x0, int n, const LbfgsOptions &o);
    int tell(double f, const double *g);
    const std::vector<double> &trial_point() const { return trial; }
    const std::vector<double> &iterate() const { return x; }
    double value() const { return f; }
    double grad_norm() const { return gnorm; }
    int state() const { return status; }
    int n_steps() const { return steps; }
    int n_evals() const { return evals; }

  private:
    void direction();
    void start_line_search();
    void request(double a);
    int accept(double ft, const double *gt);
    int finish(int reason);
    LbfgsOptions opt;
    int n;
    std::vector<double> x, g, d, trial;
    std::vector<std::vector<double>> S, Y;
    std::vector<double> rho;
    double f = 0.0, gnorm = 0.0, dphi0 = 0.0, alpha = 0.0;
    double a_prev = 0.0, f_prev = 0.0, df_prev = 0.0;
    double a_lo = 0.0, f_lo = 0.0, df_lo = 0.0, a_hi = 0.0;
    bool first = true, zooming = false, give_up = false;
    int line_evals = 0, steps = 0, evals = 0, status = LBFGS_EVALUATE;
};

// Build and validate a model; returns an empty string or an error message.
std::string build_model(int nx, int ny, int px, int py, const double *t, double U,
                        const double *V, const double *eps, const int32_t *groups, Model &m);
std::string build_graph_model(int n_sites, int n_bonds, const int32_t *bi, const int32_t *bj,
                              const double *t, double U, const double *V, const double *eps,
                              const int32_t *groups, const int32_t *site_spin, Model &m);

// One elementary operation of the forward circuit or of H.
struct HostOp {
    int kind = OP_DIAG;
    int param = -1;
    uint32_t qmask = 0;     // qubits it touches (ordering constraints); MASK: its mask
    int p = -1, q = -1;     // HOP qubits, p < q
    double t = 0.0;         // HOP: t_b; MASK: coefficient
    uint32_t umask = 0, emask = 0;
    std::vector<int> vbonds;
};

// Ops [op_begin, op_end) of a pass whose hopping terms all act on the
// phase's register bits `regs` (tile-local bit indices, at most four).
struct HostPhase {
    std::vector<int> regs;
    std::vector<int> wave;   // tile-local bits that index the workgroup's waves
    int op_begin = 0, op_end = 0;
};

struct HostPass {
    std::vector<int> tile;          // sorted global bit positions
    std::vector<HostOp> ops;        // application order (grouped by phase)
    std::vector<HostPhase> phases;  // register layouts, in order
    int flags = 0;
};

struct TileConfig {
    int k = 12;          // tile bits
    int c = 4;           // minimum contiguous low bits in every tile
    int lookahead = 4;   // forward planner: candidates kept per lookahead level
    int depth = 3;       // forward planner: passes of lookahead
};

// Forward circuit (layers of Eq. (7)) as elementary ops, then fused passes.
std::vector<HostOp> circuit_ops(const Model &m, int layers);
std::vector<HostPass> plan_forward(const Model &m, int layers, const TileConfig &tc);
// Fused passes of an op list on n qubits (the forward planner's search).
std::vector<HostPass> plan_ops(const std::vector<HostOp> &ops, int n, const TileConfig &tc);
// Passes that together apply H (terms split over tiles, D in the first).
std::vector<HostPass> plan_hamiltonian(const Model &m, const TileConfig &tc);
// Split a pass's ops into register phases (reorders ops within the pass only
// where they commute) and add load/store layouts.
void plan_phases(HostPass &p);
// The same passes un-applied: pass order, phase order and op order reversed.
std::vector<HostPass> reversed_passes(std::vector<HostPass> p);

}  // namespace hv
