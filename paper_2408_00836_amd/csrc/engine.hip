// engine.hip -- host runtime behind include/hubbard.h: device programs built
// from the pass plans, kernel launches and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/hubbard.h"
#include "../../include/hubbard_plan.h"
#include "hubvqe.hpp"

namespace hv {
template <int MODE, bool GEN, bool FULL, int NT, bool START = false, int OPS = OPS_HVA>
__global__ void k_pass(DevPass, const DevPhase *, const DevOp *, const DevVBond *, const double *,
                       const DevModel *, double2 *, double2 *, double *, int, uint32_t);
__global__ void k_init_basis(double2 *, uint64_t, uint64_t, uint32_t);
template <int MODE, bool GEN, bool FULL, bool START, int OPS = OPS_HVA>
__global__ void k_batch_pass(const DevInstance *, const DevPass *, const DevWork *, double *);
__global__ void k_reduce_seg(const double *, const int32_t *, const int64_t *, const int32_t *,
                             const double *, const int64_t *, int, double *, double *);
__global__ void k_reduce(const double *, int, const int32_t *, const int32_t *, const int32_t *,
                         const double *, double *, double *, int);
__global__ void k_vdot(const double2 *, const double2 *, uint64_t, double2 *);
__global__ void k_krylov_update(double2 *, const double2 *, const double2 *, double, double,
                                uint64_t, double2 *);
__global__ void k_vscale(double2 *, const double2 *, double, uint64_t);
__global__ void k_vaxpy(double2 *, const double2 *, double, uint64_t);
__global__ void k_vsum(const double2 *, int, double2 *);
__global__ void k_vscale_dev(double2 *, const double2 *, const double2 *, uint64_t);
__global__ void k_overlap_finish(const double2 *, double *, int, double *);
__global__ void k_bit_moments(const double2 *, int, int, double *);
__global__ void k_moments_final(const double *, int, int, int, double *);
__global__ void k_spin_corr(const double *, int, double *, double *);

// H applied to a device vector (in -> out) on the caller's stream.
using ApplyH = std::function<hubbard_status(const double2 *, double2 *)>;
hubbard_status lanczos_run(const ApplyH &apply, uint64_t n, const double2 *start_dev,
                           int32_t max_iter, double tol, double *E0, int32_t *iters,
                           double *residual, double2 *gs_dev, double2 *const buf[3],
                           double2 *partial, hipStream_t s);
size_t lanczos_partial_bytes();
}  // namespace hv

using namespace hv;

namespace {

thread_local std::string g_err;

hubbard_status fail(hubbard_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

// Pass grids: one tile per workgroup while the workgroups fit the chip at
// once (256 CUs x two tile-sized workgroups), else at least two tiles (or
// tile pairs) per workgroup -- a workgroup's set-up (layout tables,
// rotation coefficients) is then amortised -- and at most kGridMax
// workgroups: many more than are resident, so that the last round of
// workgroups leaves little of the chip idle.  Measured at 32 qubits (2^20
// tiles): 16384 workgroups beat 2048 by 3.6 %; at 24 qubits (4096 tiles)
// two tiles per workgroup beat one by 7 %.
constexpr int kGridMax = 16384;
constexpr uint64_t kGridFill = 512;
uint64_t pass_grid(uint64_t units)
{
    return std::min<uint64_t>(std::max(std::min(units, kGridFill), units / 2), kGridMax);
}
enum { M_FWD = 0, M_REV = 1, M_HAM = 2, M_EXP = 3 };

// Bank-conflict cycles of a pass's LDS exchanges under the slot masks mask[b]
// (the low four slot bits that tile-local bit b moves).  In each
// phase's layout the lane id sits on the tile-local bits outside the register
// and wave bits (ascending), so a lane bit i moves the slot's low bits by
// v_i.  A wave's 16-byte LDS write is served 8 lanes at a time (slots equal
// modulo 8 conflict: lane bits 0-2 must move slot bits 0-2 independently), a
// 16-byte read 16 lanes at a time (modulo 16, lane bits 0-3).  A phase is
// written when left and read when entered (not the load and store layouts).
int gf2_rank(uint32_t *v, int n)
{
    int r = 0;
    for (int bit = 0; bit < 4 && r < n; ++bit) {
        int piv = -1;
        for (int i = r; i < n; ++i)
            if ((v[i] >> bit) & 1u) {
                piv = i;
                break;
            }
        if (piv < 0)
            continue;
        std::swap(v[r], v[piv]);
        for (int i = 0; i < n; ++i)
            if (i != r && ((v[i] >> bit) & 1u))
                v[i] ^= v[r];
        ++r;
    }
    return r;
}
int exchange_conflicts(const HostPass &p, int k, const uint32_t *mask)
{
    int cost = 0;
    const int np = (int)p.phases.size();
    for (int q = 0; q < np; ++q) {
        uint32_t other = 0;
        for (int b : p.phases[q].regs)
            other |= 1u << b;
        for (int b : p.phases[q].wave)
            other |= 1u << b;
        uint32_t v[4];
        int nl = 0;
        for (int b = 0; b < k && nl < 4; ++b)
            if (!((other >> b) & 1u))
                v[nl++] = mask[b];
        if (nl < 4)
            continue;
        if (q + 1 < np) {
            uint32_t w[3] = {v[0] & 7u, v[1] & 7u, v[2] & 7u};
            cost += ((1 << (3 - gf2_rank(w, 3))) - 1) * 8;
        }
        if (q > 0) {
            uint32_t w[4] = {v[0], v[1], v[2], v[3]};
            cost += ((1 << (4 - gf2_rank(w, 4))) - 1) * 4;
        }
    }
    return cost;
}
// The pass's slot masks (packed as slot() reads them): the identity on bits
// 0..3 with the fixed fold of bits 4..11 onto them, unless one of 256
// pseudo-random mask sets (a fixed sequence; bits 0..3 an invertible
// matrix) costs fewer conflict cycles.  On the 32-qubit torus every pass
// gets a conflict-free set.
void choose_slot_masks(const HostPass &p, int k, uint32_t swz[2])
{
    uint32_t best[13] = {0}, cand[13] = {0};
    for (int b = 0; b < 12; ++b)
        best[b] = 1u << (b % 4);
    int best_cost = exchange_conflicts(p, k, best);
    uint64_t x = 0x9E3779B97F4A7C15ull;
    auto next4 = [&x]() {
        x = x * 6364136223846793005ull + 1442695040888963407ull;
        return (uint32_t)(x >> 60);
    };
    for (int t = 0; t < 256 && best_cost > 0; ++t) {
        uint32_t low[4];
        do {
            for (int b = 0; b < 4; ++b)
                cand[b] = low[b] = next4();
        } while (gf2_rank(low, 4) < 4);
        for (int b = 4; b < 13; ++b)
            cand[b] = b < k ? next4() : 0u;
        const int c = exchange_conflicts(p, k, cand);
        if (c < best_cost) {
            best_cost = c;
            std::copy(cand, cand + 13, best);
        }
    }
    swz[0] = 0;
    for (int b = 4; b < 12; ++b)
        swz[0] |= (best[b] & 15u) << (4 * (b - 4));
    swz[1] = best[12] & 15u;
    for (int b = 0; b < 4; ++b)
        swz[1] |= (best[b] & 15u) << (4 + 4 * b);
}

enum ProgKind { PROG_ANSATZ = 0, PROG_HAM = 1, PROG_ENERGY = 2, PROG_GRAD = 3 };

// A flattened set of passes of one kind.
struct PassList {
    std::vector<DevPass> pass;
    std::vector<int> grid;
    std::vector<int> smem;
    std::vector<int> threads;
    std::vector<int> nt;   // tiles per loop iteration (2: one-vector full-tile passes)
};

// Everything one call needs on one device.
struct Program {
    int kind = 0;
    int layers = 0;
    bool general = false;   // diagonal has eps or V terms
    bool np = false;        // NP circuit: gate passes hold hopping terms and mask phases
    PassList fwd, ham, rev, exp;
    // device tables
    DevOp *d_ops = nullptr;
    DevPhase *d_phases = nullptr;
    DevVBond *d_vb = nullptr;
    int32_t *d_row_ptr = nullptr, *d_row_idx = nullptr, *d_row_nblk = nullptr;
    int32_t *d_row_param = nullptr;
    double *d_scale = nullptr;
    int n_rows = 0, n_out = 0;
    size_t partial_bytes = 0;
    // host copies (introspection, batch layout)
    std::vector<HostPass> h_fwd, h_ham, h_rev, h_exp;
    std::vector<int> row_param;   // per reduction row: parameter, or -1 for the energy
    ~Program()
    {
        (void)hipFree(d_ops);
        (void)hipFree(d_phases);
        (void)hipFree(d_vb);
        (void)hipFree(d_row_ptr);
        (void)hipFree(d_row_idx);
        (void)hipFree(d_row_nblk);
        (void)hipFree(d_row_param);
        (void)hipFree(d_scale);
    }
};

struct DeviceState {
    DevModel *d_model = nullptr;
    std::map<std::pair<int, int>, std::unique_ptr<Program>> progs;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct hubbard_model {
    Model m;
    // identity of the handle for caches that outlive a call: never reused by
    // a later handle (unlike its address); gen counts the changes of the
    // tile configuration, which replace the device programs
    uint64_t uid = 0;
    uint64_t gen = 0;
    TileConfig fwd_tc{12, 4};
    TileConfig rev_tc{12, 4};
    std::map<int, DeviceState> dev;
    std::mutex mu;
    // optional phase timing: events recorded on the call's stream
    bool timing = false;
    bool ev_ready = false;
    hipEvent_t ev[4];
    int ev_used = 0;
    // per-launch timing of the pass kernels: event pairs around each launch
    // of the last call, and the kernel mode of each
    std::vector<hipEvent_t> kev;
    std::vector<int> kmode;
    // forward schedules already planned, by (layers, k, c, lookahead, depth)
    std::mutex plan_mu;
    std::map<std::tuple<int, int, int, int, int>, std::vector<HostPass>> fwd_plans;
};

namespace {

// ----------------------------------------------------------- flattening --

struct Builder {
    const Model &m;
    std::vector<DevOp> ops;
    std::vector<DevPhase> phases;
    std::vector<DevVBond> vb;
    std::vector<int> row_param;   // param (or -1 for energy) of each partial row
    std::vector<int> row_nblk;
    explicit Builder(const Model &mm) : m(mm) {}

    // rows: 0 none, 1 one row per distinct param (reverse), 2 one energy row.
    // dual: forward passes of a U-only model over full tiles take two tiles
    // per loop iteration, on half the workgroups.
    PassList add(const std::vector<HostPass> &passes, int rows, bool last_only_energy,
                 bool dual = false)
    {
        PassList pl;
        for (size_t pi = 0; pi < passes.size(); ++pi) {
            const HostPass &hp = passes[pi];
            DevPass P;
            std::memset(&P, 0, sizeof(P));
            const int n = m.nq;
            P.k = (int)hp.tile.size();
            int c = 0;
            while (c < P.k && hp.tile[c] == c)
                ++c;
            P.c = c;
            uint32_t S = 0;
            for (int j = 0; j < P.k; ++j) {
                S |= 1u << hp.tile[j];
                if (j >= c)
                    P.hi_mask |= 1u << hp.tile[j];
            }
            int nf = 0;
            for (int b = 0; b < n; ++b)
                if (!(S & (1u << b))) {
                    P.free_mask |= 1u << b;
                    ++nf;
                }
            P.nfree = nf;
            P.flags = hp.flags;
            choose_slot_masks(hp, P.k, P.swz);
            P.op_begin = (int)ops.size();
            const uint64_t ntiles = (uint64_t)1 << nf;
            // (the HVA circuit only: NP passes carry many per-register phases)
            const bool two = dual && !m.general && m.ansatz == 0 && P.k >= kRegBits && nf >= 1;
            const int grid = (int)pass_grid(two ? ntiles / 2 : ntiles);
            std::map<int, int> red_of;
            P.red_base = (int)row_param.size();
            if (rows == 2 && (!last_only_energy || (hp.flags & PF_HAM_LAST))) {
                red_of[-2] = 0;
                row_param.push_back(-1);
                row_nblk.push_back(grid);
            }
            int n_diag = 0;
            std::vector<int> op_pl, op_ql;   // tile-local bits of each op's qubits
            for (const HostOp &h : hp.ops) {
                DevOp o;
                std::memset(&o, 0, sizeof(o));
                o.kind = h.kind;
                o.param = h.param;
                o.red = -1;
                o.dtab = -1;
                o.v_begin = o.v_end = 0;
                if (rows == 1 && h.param >= 0) {
                    auto it = red_of.find(h.param);
                    if (it == red_of.end()) {
                        int r = (int)red_of.size();
                        red_of[h.param] = r;
                        row_param.push_back(h.param);
                        row_nblk.push_back(grid);
                        o.red = r;
                    } else {
                        o.red = it->second;
                    }
                }
                if (h.kind == OP_HOP) {
                    int pl = -1, ql = -1;
                    for (int j = 0; j < P.k; ++j) {
                        if (hp.tile[j] == h.p)
                            pl = j;
                        if (hp.tile[j] == h.q)
                            ql = j;
                    }
                    op_pl.push_back(pl);
                    op_ql.push_back(ql);
                    const int lo = std::min(h.p, h.q), hi = std::max(h.p, h.q);
                    uint32_t bw = 0;
                    for (int b = lo + 1; b < hi; ++b)
                        bw |= 1u << b;
                    o.between = bw;
                    o.t = h.t;
                } else if (h.kind == OP_MASK) {
                    op_pl.push_back(-1);
                    op_ql.push_back(-1);
                    o.between = h.qmask;
                    o.t = h.t;
                } else {
                    op_pl.push_back(-1);
                    op_ql.push_back(-1);
                    o.dtab = n_diag++;
                    o.umask = h.umask;
                    o.emask = h.emask;
                    // V bonds in classes of equal site offset and equal V
                    o.v_begin = (int)vb.size();
                    for (int b : h.vbonds) {
                        const int delta = m.bj[b] - m.bi[b];
                        size_t c = (size_t)o.v_begin;
                        while (c < vb.size() && !(vb[c].delta == delta && vb[c].V == m.V[b]))
                            ++c;
                        if (c == vb.size()) {
                            DevVBond v;
                            std::memset(&v, 0, sizeof(v));
                            v.delta = delta;
                            v.V = m.V[b];
                            vb.push_back(v);
                        }
                        vb[c].src |= 1u << m.bi[b];
                    }
                    o.v_end = (int)vb.size();
                }
                ops.push_back(o);
            }
            P.n_ops = (int)hp.ops.size();
            P.n_diag = n_diag;
            P.n_red = (int)red_of.size();
            // register layouts
            const int rbits = std::min(P.k, kRegBits);
            P.tbits = P.k - rbits;
            P.phase_begin = (int)phases.size();
            P.n_phases = (int)hp.phases.size();
            for (const HostPhase &hph : hp.phases) {
                DevPhase D;
                std::memset(&D, 0, sizeof(D));
                D.op_begin = hph.op_begin;
                D.op_end = hph.op_end;
                uint32_t regmask = 0, wmask = 0;
                for (int b : hph.regs)
                    regmask |= 1u << b;
                for (int b : hph.wave)
                    wmask |= 1u << b;
                D.wmask = wmask;
                D.lmask = 0;
                for (int b = 0; b < P.k; ++b)
                    if (!((regmask >> b) & 1u) && !((wmask >> b) & 1u))
                        D.lmask |= 1u << b;
                if (__builtin_popcount(D.lmask) > 6 ||
                    (__builtin_popcount(wmask) > 0 && __builtin_popcount(D.lmask) != 6))
                    throw std::runtime_error("phase layout needs 6 lane bits before wave bits");
                D.cross = (!phases.empty() && (int)phases.size() > P.phase_begin &&
                           phases.back().wmask != wmask)
                              ? 1u
                              : 0u;
                D.valid = 0;
                for (int i = 0; i < kRegBits; ++i) {
                    if (i < (int)hph.regs.size()) {
                        D.gb[i] = 1u << hp.tile[hph.regs[i]];
                        D.sb[i] = slot(1u << hph.regs[i], P.swz[0], P.swz[1]) << 4;
                    } else {
                        D.gb[i] = D.sb[i] = 0;   // phantom register bit of a tile < 16
                    }
                }
                std::vector<uint32_t> goff(kRegs, 0);
                for (int j = 0; j < kRegs; ++j) {
                    bool ok = true;
                    for (int i = 0; i < kRegBits; ++i)
                        if ((j >> i) & 1) {
                            if (i >= (int)hph.regs.size())
                                ok = false;
                            goff[j] |= D.gb[i];
                        }
                    if (ok)
                        D.valid |= 1u << j;
                }
                // pair index of each hop of the phase
                for (int o = hph.op_begin; o < hph.op_end; ++o) {
                    DevOp &op = ops[P.op_begin + o];
                    if (op.kind != OP_HOP)
                        continue;
                    int ra = -1, rb = -1;
                    for (size_t i = 0; i < hph.regs.size(); ++i) {
                        if (hph.regs[i] == op_pl[o])
                            ra = (int)i;
                        if (hph.regs[i] == op_ql[o])
                            rb = (int)i;
                    }
                    if (ra < 0 || rb < 0)
                        throw std::runtime_error("hop outside its phase's register bits");
                    int a = std::min(ra, rb), b = std::max(ra, rb);
                    static const int pair_of[4][4] = {
                        {-1, 0, 1, 2}, {0, -1, 3, 4}, {1, 3, -1, 5}, {2, 4, 5, -1}};
                    op.pair = pair_of[a][b];
                    op.flip = 0;
                    for (int j = 0; j < kRegs; ++j)
                        if (__builtin_popcount(goff[j] & op.between) & 1)
                            op.flip |= 1u << j;
                }
                phases.push_back(D);
            }
            pl.pass.push_back(P);
            pl.nt.push_back(two ? 2 : 1);
            pl.grid.push_back(grid);
            pl.smem.push_back(0);
            pl.threads.push_back(1 << P.tbits);
        }
        return pl;
    }
};

int max_smem_per_block()
{
    // gfx950 gives a workgroup up to 160 KiB of LDS; ask the device when one
    // is present so that planning without a GPU gives the same plan.
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 160 * 1024;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 160 * 1024;
    return v;
}

void set_smem(PassList &pl, bool force_red1, bool general)
{
    for (size_t i = 0; i < pl.pass.size(); ++i) {
        const DevPass &P = pl.pass[i];
        int nred = force_red1 ? 1 : P.n_red;
        pl.smem[i] = (int)smem_plan(P.k, P.n_ops, P.n_diag, nred, P.n_phases, pl.threads[i],
                                    P.nfree == 0, general)
                         .total;
    }
}

int max_of(const PassList &pl)
{
    int m = 0;
    for (int s : pl.smem)
        m = std::max(m, s);
    return m;
}

// Forward schedule for a layer count and tile configuration, planned once per
// handle (the lookahead search makes planning cost a fraction of a second at
// 32 qubits, and workspace queries and uploads ask for the same plans).
std::vector<HostPass> cached_forward(hubbard_model *h, int layers, const TileConfig &tc)
{
    const auto key = std::make_tuple(layers, tc.k, tc.c, tc.lookahead, tc.depth);
    {
        std::lock_guard<std::mutex> lk(h->plan_mu);
        auto it = h->fwd_plans.find(key);
        if (it != h->fwd_plans.end())
            return it->second;
    }
    std::vector<HostPass> plan = plan_forward(h->m, layers, tc);
    std::lock_guard<std::mutex> lk(h->plan_mu);
    h->fwd_plans.emplace(key, plan);
    return plan;
}

// Builds host plans only (no device work): used by introspection and upload.
void plan_program(hubbard_model *h, int kind, int layers, int smem_limit, Program &pr)
{
    const Model &m = h->m;
    pr.kind = kind;
    pr.layers = layers;
    pr.general = m.general;
    pr.np = m.ansatz != 0;
    if (kind != PROG_HAM)
        pr.h_fwd = cached_forward(h, layers, h->fwd_tc);
    TileConfig tc2 = h->rev_tc;
    for (;;) {
        if (kind == PROG_HAM || kind == PROG_GRAD)
            pr.h_ham = plan_hamiltonian(m, tc2);
        if (kind == PROG_GRAD)
            pr.h_rev = reversed_passes(cached_forward(h, layers, tc2));
        // check LDS fit of the two-vector kernels; shrink the tile if needed
        Builder b(m);
        PassList ph = b.add(pr.h_ham, 2, true), pv = b.add(pr.h_rev, 1, false);
        set_smem(ph, false, m.general);
        set_smem(pv, false, m.general);
        if (std::max(max_of(ph), max_of(pv)) <= smem_limit || tc2.k <= 6)
            break;
        tc2.k -= 1;
    }
    if (kind == PROG_ENERGY)
        pr.h_exp = plan_hamiltonian(m, h->fwd_tc);
}

// Device-form pass lists of a planned program (no device work).
void build_lists(Builder &b, Program &pr)
{
    pr.fwd = b.add(pr.h_fwd, 0, false, true);
    pr.ham = b.add(pr.h_ham, pr.kind == PROG_GRAD ? 2 : 0, true);
    pr.rev = b.add(pr.h_rev, 1, false);
    pr.exp = b.add(pr.h_exp, 2, false);
    set_smem(pr.fwd, false, pr.general);
    set_smem(pr.ham, false, pr.general);
    set_smem(pr.rev, false, pr.general);
    set_smem(pr.exp, true, pr.general);
    pr.row_param.assign(b.row_param.begin(), b.row_param.end());
}

hubbard_status upload_program(hubbard_model *h, DeviceState &ds, Program &pr)
{
    const Model &m = h->m;
    Builder b(m);
    build_lists(b, pr);
    int lim = max_smem_per_block();
    for (const PassList *l : {&pr.fwd, &pr.ham, &pr.rev, &pr.exp})
        if (max_of(*l) > lim)
            return fail(HUBBARD_ERR_ARG, "a pass needs more LDS than a workgroup may use; "
                                         "choose smaller tiles");
    const int P = m.n_params(pr.layers);
    // reduction map: output 0 = E, outputs 1..P = gradient
    pr.n_out = (pr.kind == PROG_GRAD) ? 1 + P : 1;
    std::vector<std::vector<int>> rows_of(pr.n_out);
    for (size_t r = 0; r < b.row_param.size(); ++r) {
        int p = b.row_param[r];
        if (p < 0)
            rows_of[0].push_back((int)r);
        else if (pr.kind == PROG_GRAD)
            rows_of[1 + p].push_back((int)r);
    }
    std::vector<int32_t> row_ptr{0}, row_idx;
    std::vector<double> scale;
    for (int o = 0; o < pr.n_out; ++o) {
        for (int r : rows_of[o])
            row_idx.push_back(r);
        row_ptr.push_back((int32_t)row_idx.size());
        scale.push_back(o == 0 ? 1.0 : 2.0);
    }
    std::vector<int32_t> nblk(b.row_nblk.begin(), b.row_nblk.end());
    pr.n_rows = (int)b.row_param.size();
    pr.partial_bytes = align256((size_t)pr.n_rows * kGridMax * sizeof(double));

    auto up = [](void **dst, const void *src, size_t bytes) -> hipError_t {
        if (bytes == 0)
            bytes = 16;
        hipError_t e = hipMalloc(dst, bytes);
        if (e != hipSuccess)
            return e;
        if (src)
            return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
        return hipSuccess;
    };
    hipError_t e = hipSuccess;
    e = up((void **)&pr.d_ops, b.ops.data(), b.ops.size() * sizeof(DevOp));
    if (e == hipSuccess)
        e = up((void **)&pr.d_phases, b.phases.empty() ? nullptr : b.phases.data(),
               b.phases.size() * sizeof(DevPhase));
    if (e == hipSuccess)
        e = up((void **)&pr.d_vb, b.vb.empty() ? nullptr : b.vb.data(), b.vb.size() * sizeof(DevVBond));
    if (e == hipSuccess)
        e = up((void **)&pr.d_row_ptr, row_ptr.data(), row_ptr.size() * sizeof(int32_t));
    if (e == hipSuccess)
        e = up((void **)&pr.d_row_idx, row_idx.empty() ? nullptr : row_idx.data(),
               row_idx.size() * sizeof(int32_t));
    if (e == hipSuccess)
        e = up((void **)&pr.d_row_nblk, nblk.empty() ? nullptr : nblk.data(),
               nblk.size() * sizeof(int32_t));
    if (e == hipSuccess)
        e = up((void **)&pr.d_scale, scale.data(), scale.size() * sizeof(double));
    if (e == hipSuccess) {
        std::vector<int32_t> rp(b.row_param.begin(), b.row_param.end());
        e = up((void **)&pr.d_row_param, rp.empty() ? nullptr : rp.data(),
               rp.size() * sizeof(int32_t));
    }
    if (e != hipSuccess)
        return fail(HUBBARD_ERR_DEVICE, std::string("uploading plan: ") + hipGetErrorString(e));
    (void)ds;
    return HUBBARD_OK;
}

hubbard_status ensure_model(hubbard_model *h, int dev, DeviceState &ds)
{
    if (ds.d_model)
        return HUBBARD_OK;
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
        int lim = max_smem_per_block();
        const void *fns[] = {
            (const void *)k_pass<M_FWD, false, true, 1>,  (const void *)k_pass<M_REV, false, true, 1>,
            (const void *)k_pass<M_HAM, false, true, 1>,  (const void *)k_pass<M_EXP, false, true, 1>,
            (const void *)k_pass<M_FWD, true, true, 1>,   (const void *)k_pass<M_REV, true, true, 1>,
            (const void *)k_pass<M_HAM, true, true, 1>,   (const void *)k_pass<M_EXP, true, true, 1>,
            (const void *)k_pass<M_FWD, false, false, 1>, (const void *)k_pass<M_REV, false, false, 1>,
            (const void *)k_pass<M_HAM, false, false, 1>, (const void *)k_pass<M_EXP, false, false, 1>,
            (const void *)k_pass<M_FWD, true, false, 1>,  (const void *)k_pass<M_REV, true, false, 1>,
            (const void *)k_pass<M_HAM, true, false, 1>,  (const void *)k_pass<M_EXP, true, false, 1>,
            (const void *)k_pass<M_FWD, false, true, 2>,
            (const void *)k_pass<M_FWD, false, true, 1, true>,
            (const void *)k_pass<M_FWD, true, true, 1, true>,
            (const void *)k_pass<M_FWD, false, false, 1, true>,
            (const void *)k_pass<M_FWD, true, false, 1, true>,
            (const void *)k_pass<M_FWD, false, true, 2, true>,
            (const void *)k_pass<M_FWD, false, true, 1, false, OPS_NP>,
            (const void *)k_pass<M_FWD, false, true, 1, true, OPS_NP>,
            (const void *)k_pass<M_REV, false, true, 1, false, OPS_NP>,
            (const void *)k_pass<M_FWD, false, false, 1, false, OPS_NP>,
            (const void *)k_pass<M_FWD, false, false, 1, true, OPS_NP>,
            (const void *)k_pass<M_REV, false, false, 1, false, OPS_NP>};
        for (const void *f : fns)
            (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    });
    (void)dev;
    const Model &m = h->m;
    DevModel dm;
    std::memset(&dm, 0, sizeof(dm));
    dm.n = m.nq;
    dm.ns = m.ns;
    dm.general = m.general ? 1 : 0;
    dm.b0 = (uint32_t)m.neel;
    dm.U = m.U;
    for (int q = 0; q < kMaxQubits; ++q)
        dm.eps_q[q] = q < m.nq ? m.eps[q < m.ns ? q : q - m.ns] : 0.0;
    hipError_t e = hipMalloc((void **)&ds.d_model, sizeof(DevModel));
    if (e == hipSuccess)
        e = hipMemcpy(ds.d_model, &dm, sizeof(DevModel), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(ds.d_model);
        ds.d_model = nullptr;
        return fail(HUBBARD_ERR_DEVICE, std::string("uploading model: ") + hipGetErrorString(e));
    }
    return HUBBARD_OK;
}

hubbard_status get_program(hubbard_model *h, int kind, int layers, Program **out,
                           DeviceState **dsout)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(HUBBARD_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(h->mu);
    DeviceState &ds = h->dev[dev];
    hubbard_status st = ensure_model(h, dev, ds);
    if (st != HUBBARD_OK)
        return st;
    auto key = std::make_pair(kind, layers);
    auto it = ds.progs.find(key);
    if (it == ds.progs.end()) {
        std::unique_ptr<Program> pr(new Program());
        try {
            plan_program(h, kind, layers, max_smem_per_block(), *pr);
        } catch (const std::exception &ex) {
            return fail(HUBBARD_ERR_NOMEM, std::string("planning: ") + ex.what());
        }
        st = upload_program(h, ds, *pr);
        if (st != HUBBARD_OK)
            return st;
        it = ds.progs.emplace(key, std::move(pr)).first;
    }
    *out = it->second.get();
    *dsout = &ds;
    return HUBBARD_OK;
}

hubbard_status check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(HUBBARD_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return HUBBARD_OK;
}

// Timing mode: an event pair around one launch (events are created on first
// use and reused by later calls).
bool launch_mark(hubbard_model *h, int mode, hipStream_t s, bool end)
{
    if (!h || !h->timing)
        return false;
    const size_t i = end ? 2 * h->kmode.size() - 1 : 2 * h->kmode.size();
    if (!end) {
        if (h->kev.size() < i + 2) {
            hipEvent_t e0, e1;
            if (hipEventCreate(&e0) != hipSuccess)
                return false;
            if (hipEventCreate(&e1) != hipSuccess) {
                (void)hipEventDestroy(e0);
                return false;
            }
            h->kev.push_back(e0);
            h->kev.push_back(e1);
        }
        h->kmode.push_back(mode);
    }
    (void)hipEventRecord(h->kev[i], s);
    return true;
}

// Vector storage: the pass kernels find amplitude g of each vector at
// vec_offset(g, ilv) elements from its pointer; ilv = kPlainVec for
// contiguous vectors, else blocks of 2^ilv amplitudes with one-block gaps.
constexpr uint32_t kPlainVec = 32;
struct VecLayout {
    uint32_t ilv = kPlainVec;
};

// first_flags / last_flags: PassFlags added to the first / last pass of the
// list for this launch (PF_FROM_START, PF_NO_STORE).
template <int MODE>
void launch_list(const Program &pr, const DeviceState &ds, const PassList &pl, const double *theta,
                 const double2 *a, const double2 *b, double *partial, hipStream_t s,
                 hubbard_model *h, VecLayout vl = VecLayout(), int32_t first_flags = 0,
                 int32_t last_flags = 0)
{
    for (size_t i = 0; i < pl.pass.size(); ++i) {
        DevPass P = pl.pass[i];
        if (i == 0)
            P.flags |= first_flags;
        if (i + 1 == pl.pass.size())
            P.flags |= last_flags;
        const bool timed = launch_mark(h, MODE, s, false);
        // tiles of >= 16 amplitudes fill every register of every thread
        const bool full = pl.pass[i].k >= kRegBits;
        const bool two = pl.nt[i] == 2;
#define HV_LAUNCH_OPS(GEN, FULL, NT, ST, OPS)                                                   \
    hipLaunchKernelGGL((k_pass<MODE, GEN, FULL, NT, ST, OPS>), dim3(pl.grid[i]),               \
                       dim3(pl.threads[i]), pl.smem[i], s, P, pr.d_phases, pr.d_ops, pr.d_vb,   \
                       theta, ds.d_model, (double2 *)a, (double2 *)b, partial, kGridMax, vl.ilv)
#define HV_LAUNCH(GEN, FULL, NT, ST) HV_LAUNCH_OPS(GEN, FULL, NT, ST, OPS_HVA)
        if constexpr (MODE == M_FWD || MODE == M_REV) {
            // NP gate passes: hopping terms and mask phases, no diagonal sub-terms
            if (pr.np) {
                const bool st = MODE == M_FWD && (P.flags & PF_FROM_START) != 0;
                if (st) {
                    if (full)
                        HV_LAUNCH_OPS(false, true, 1, true, OPS_NP);
                    else
                        HV_LAUNCH_OPS(false, false, 1, true, OPS_NP);
                } else if (full) {
                    HV_LAUNCH_OPS(false, true, 1, false, OPS_NP);
                } else {
                    HV_LAUNCH_OPS(false, false, 1, false, OPS_NP);
                }
                if (timed)
                    launch_mark(h, MODE, s, true);
                continue;
            }
        }
        if constexpr (MODE == M_FWD) {
            // the first pass from the start state has kernels of its own
            const bool st = (P.flags & PF_FROM_START) != 0;
            if (two) {   // only planned for U-only models
                if (st)
                    HV_LAUNCH(false, true, 2, true);
                else
                    HV_LAUNCH(false, true, 2, false);
                if (timed)
                    launch_mark(h, MODE, s, true);
                continue;
            }
            if (st) {
                if (pr.general) {
                    if (full)
                        HV_LAUNCH(true, true, 1, true);
                    else
                        HV_LAUNCH(true, false, 1, true);
                } else {
                    if (full)
                        HV_LAUNCH(false, true, 1, true);
                    else
                        HV_LAUNCH(false, false, 1, true);
                }
                if (timed)
                    launch_mark(h, MODE, s, true);
                continue;
            }
        }
        if (pr.general) {
            if (full)
                HV_LAUNCH(true, true, 1, false);
            else
                HV_LAUNCH(true, false, 1, false);
        } else {
            if (full)
                HV_LAUNCH(false, true, 1, false);
            else
                HV_LAUNCH(false, false, 1, false);
        }
#undef HV_LAUNCH
#undef HV_LAUNCH_OPS
        if (timed)
            launch_mark(h, MODE, s, true);
    }
}

// from_start: psi is not read; the first pass starts from |b0> (the caller
// then skips the init kernel).  Needs at least one forward pass.
hubbard_status run_forward(const Program &pr, const DeviceState &ds, const double *theta,
                           double2 *psi, hipStream_t s, hubbard_model *h = nullptr,
                           VecLayout vl = VecLayout(), bool from_start = false)
{
    launch_list<M_FWD>(pr, ds, pr.fwd, theta, psi, nullptr, nullptr, s, h, vl,
                       from_start ? PF_FROM_START : 0);
    return check_launch("forward pass");
}

hubbard_status run_ham(const Program &pr, const DeviceState &ds, const double2 *psi, double2 *phi,
                       double *partial, hipStream_t s, hubbard_model *h = nullptr,
                       VecLayout vl = VecLayout())
{
    launch_list<M_HAM>(pr, ds, pr.ham, nullptr, psi, phi, partial, s, h, vl);
    return check_launch("hamiltonian pass");
}

hubbard_status run_init(const hubbard_model *h, double2 *psi, hipStream_t s,
                        VecLayout vl = VecLayout())
{
    const uint64_t dim = (uint64_t)1 << h->m.nq;
    uint64_t blocks = std::min<uint64_t>((dim + 255) / 256, 8192);
    hipLaunchKernelGGL(k_init_basis, dim3((unsigned)blocks), dim3(256), 0, s, psi, dim,
                       (uint64_t)h->m.neel, vl.ilv);
    return check_launch("init");
}

hubbard_status run_reduce(const Program &pr, const double *partial, double *E, double *grad,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce, dim3(pr.n_out), dim3(256), 0, s, partial, kGridMax, pr.d_row_ptr,
                       pr.d_row_idx, pr.d_row_nblk, pr.d_scale, E, grad, 1);
    return check_launch("reduce");
}

size_t vec_bytes(const hubbard_model *h) { return ((size_t)1 << h->m.nq) * 16u; }

// energy_grad's psi and lambda (2^n amplitudes each) share the first
// 2 * 2^n amplitudes of the workspace for n > kBlockBits: blocks of
// 2^kBlockBits amplitudes (1 MiB) of psi and lambda alternate.  A
// one-vector pass then streams over the whole 2 * 2^n region.  On MI355X
// at 32 qubits the interleave took the forward passes from 2.86 s to 2.62 s
// per evaluation (one-vector streaming over a single contiguous 64 GiB range
// ran at 5.1 TB/s in a probe, over both 64 GiB halves of a 128 GiB region
// at 6.1 TB/s); 1 MiB blocks beat 16 MiB ones by about 1 % per evaluation
// (the reverse passes; 64 KiB to 8 MiB blocks measured).
constexpr int kBlockBits = 16;
VecLayout grad_layout(const hubbard_model *h)
{
    VecLayout vl;
    if (h->m.nq > kBlockBits)
        vl.ilv = (uint32_t)kBlockBits;
    return vl;
}

// Phase marks: 0 before the forward passes, 1 after them, 2 after the H or
// expectation passes, 3 after the reverse passes.
void mark(hubbard_model *h, int i, hipStream_t s)
{
    if (!h->timing)
        return;
    if (!h->ev_ready) {
        for (int j = 0; j < 4; ++j)
            if (hipEventCreate(&h->ev[j]) != hipSuccess)
                return;
        h->ev_ready = true;
    }
    (void)hipEventRecord(h->ev[i], s);
    h->ev_used |= 1 << i;
}

}  // namespace

// ================================================================ batch

// Planning parameters of a batch (hubbard_batch_set_config; tuned and cached
// by the Python front end, which sets them before a batch is first planned):
//  - work items per instance pass: enough to spread a large instance over
//    many workgroups, few enough that each item streams several tiles; a
//    power of two, as the tile counts are, so every item gets the same
//    share (256 uneven instances with four lanes: 16, 32, 64, 128 items
//    took 14.1, 12.6, 13.0, 13.5 ms);
//  - lanes (streams): the caller's (lane 0, the longest forward schedules)
//    and the batch program's own: lane 1 for the instances with one pass
//    per schedule, lanes 2.. for shorter forward schedules.  At most four,
//    the hardware queues a process gets by default (with 32 work items, 2,
//    3, 4, 5 length groups took 13.0, 12.5, 12.8, 13.3 ms eager for 256
//    uneven instances; more streams than queues share queues).  One lane
//    puts every launch on the caller's stream.
constexpr int kBatchLanes = 4;
struct BatchConfig {
    int items = 32;
    int lanes = kBatchLanes;
};
std::mutex g_batch_cfg_mu;
BatchConfig g_batch_cfg;

BatchConfig batch_config()
{
    std::lock_guard<std::mutex> lk(g_batch_cfg_mu);
    return g_batch_cfg;
}

struct BatchLaunch {
    int mode;               // M_FWD, M_HAM or M_REV
    bool full;              // every item's tiles fill all registers of exactly `threads`
    bool start;             // first forward position: the passes build |b0> themselves
    int lane;               // stream of the launch (0 .. lanes-1)
    int item0, n_items;     // work items [item0, item0 + n_items)
    int threads, smem;
};

// Host layout of a batched evaluation, derived from the instances' programs
// only: every instance's passes in one array, the work items of each launch
// (launch j of a schedule runs pass j of every instance that has one), the
// workspace offsets, and for every output (energies first, then gradient
// entries) the segments of partial sums that the final reduction adds.
struct BatchLayout {
    std::vector<DevPass> passes;
    std::vector<DevWork> work;
    std::vector<BatchLaunch> launches;
    std::vector<int32_t> seg_ptr{0}, seg_cnt;
    std::vector<int64_t> seg_off;
    std::vector<double> scale;
    std::vector<int64_t> out_idx;
    std::vector<size_t> voff;   // byte offset of instance i's psi (lambda follows)
    size_t partial_at = 0;      // byte offset of the partial sums
    size_t n_partial = 0;       // doubles
    size_t ws_bytes = 0;
    bool general = false;       // any instance has eps or V terms: the general path for all
    bool np = false;            // any instance runs the NP circuit: gate kernels decode mask phases
};

hubbard_status batch_layout(const hubbard_t *hs, int n, const int64_t *toff,
                            const std::vector<const Program *> &progs, const BatchConfig &cfg,
                            BatchLayout &L)
{
    const int lim = max_smem_per_block();
    size_t at = 0;
    L.general = false;
    L.np = false;
    for (int i = 0; i < n; ++i) {
        L.general = L.general || progs[i]->general;
        L.np = L.np || progs[i]->np;
    }
    L.voff.resize(n);
    for (int i = 0; i < n; ++i) {
        L.voff[i] = at;
        at += 2 * align256(vec_bytes(hs[i]));
    }
    L.partial_at = at;
    // outputs: E of every instance, then each instance's gradient
    std::vector<size_t> gbase(n);
    size_t n_out = n;
    for (int i = 0; i < n; ++i) {
        gbase[i] = n_out;
        n_out += (size_t)hs[i]->m.n_params(progs[i]->layers);
    }
    std::vector<std::vector<std::pair<int64_t, int32_t>>> segs(n_out);
    L.scale.assign(n_out, 2.0);
    L.out_idx.resize(n_out);
    for (int i = 0; i < n; ++i) {
        L.scale[i] = 1.0;
        L.out_idx[i] = i;
        const size_t P = (size_t)hs[i]->m.n_params(progs[i]->layers);
        for (size_t p = 0; p < P; ++p)
            L.out_idx[gbase[i] + p] = toff[i] + (int64_t)p;
    }
    // pass arrays: per instance its forward, H and reverse passes
    std::vector<size_t> pbase(n);
    for (int i = 0; i < n; ++i) {
        pbase[i] = L.passes.size();
        for (const PassList *pl : {&progs[i]->fwd, &progs[i]->ham, &progs[i]->rev})
            L.passes.insert(L.passes.end(), pl->pass.begin(), pl->pass.end());
        // an instance's last reverse pass is needed for its reductions only;
        // the next evaluation starts from the start states again
        if (!progs[i]->rev.pass.empty())
            L.passes.back().flags |= PF_NO_STORE;
    }
    // lanes: instances grouped by forward length, each group's launch
    // sequence on its own stream, so that a group that has finished its
    // forward runs its H and reverse while longer ones still run theirs;
    // lane 1 holds the instances with one pass per schedule (whole state in
    // one tile: one workgroup runs the circuit)
    size_t fmax = 1;
    for (int i = 0; i < n; ++i)
        fmax = std::max(fmax, progs[i]->fwd.pass.size());
    std::vector<int> lane_of(n, 0);
    const int groups = cfg.lanes - 1;   // length groups of multi-pass instances
    for (int i = 0; i < n && cfg.lanes > 1; ++i) {
        const Program &pr = *progs[i];
        const bool single = pr.fwd.pass.size() == 1 && pr.ham.pass.size() == 1 &&
                            pr.rev.pass.size() == 1;
        // multi-pass instances: group q = 0 (longest) .. groups-1 by the
        // share of the longest forward schedule still ahead of them
        const int q = std::min<int>(groups - 1, (int)(groups * (fmax - pr.fwd.pass.size()) / fmax));
        lane_of[i] = single ? 1 : (q == 0 ? 0 : q + 1);
    }
    const int modes[3] = {M_FWD, M_HAM, M_REV};
    for (int ph = 0; ph < 3; ++ph) {
        size_t longest = 0;
        for (int i = 0; i < n; ++i) {
            const PassList &pl = ph == 0 ? progs[i]->fwd : ph == 1 ? progs[i]->ham : progs[i]->rev;
            longest = std::max(longest, pl.pass.size());
        }
        for (size_t j = 0; j < longest; ++j) {
            // pass j of every instance that has one; the widest pass sets the
            // workgroup size, and the passes whose tiles fill all registers of
            // exactly that many threads get a launch of their own on the
            // guard-free full-tile path
            std::vector<int> inst;
            int widest = 64;
            for (int i = 0; i < n; ++i) {
                const PassList &pl = ph == 0 ? progs[i]->fwd : ph == 1 ? progs[i]->ham : progs[i]->rev;
                if (j >= pl.pass.size())
                    continue;
                inst.push_back(i);
                widest = std::max(widest, 1 << pl.pass[j].tbits);
            }
            for (int lane = 0; lane < cfg.lanes; ++lane)
            for (int full = 1; full >= 0; --full) {
                BatchLaunch bl;
                bl.mode = modes[ph];
                bl.full = full != 0;
                bl.start = ph == 0 && j == 0;
                bl.lane = lane;
                bl.item0 = (int)L.work.size();
                bl.threads = 64;
                std::vector<const DevPass *> used;
                for (int i : inst) {
                    const Program &pr = *progs[i];
                    const PassList &pl = ph == 0 ? pr.fwd : ph == 1 ? pr.ham : pr.rev;
                    const DevPass &P = pl.pass[j];
                    const bool fills = P.k >= kRegBits && (1 << P.tbits) == widest;
                    if (fills != bl.full || lane_of[i] != bl.lane)
                        continue;
                    const size_t off = (ph == 0 ? 0 : ph == 1 ? pr.fwd.pass.size()
                                                               : pr.fwd.pass.size() + pr.ham.pass.size());
                    const uint64_t ntiles = (uint64_t)1 << P.nfree;
                    const uint32_t items = (uint32_t)std::min<uint64_t>(ntiles, (uint64_t)cfg.items);
                    const uint32_t per = (uint32_t)(ntiles / items);
                    const int nred = P.n_red;
                    const size_t part0 = L.n_partial;
                    L.n_partial += (size_t)nred * items;
                    for (int r = 0; r < nred; ++r) {
                        const int prm = pr.row_param[P.red_base + r];
                        const size_t o = prm < 0 ? (size_t)i : gbase[i] + (size_t)prm;
                        segs[o].push_back({(int64_t)(part0 + (size_t)r * items), (int32_t)items});
                    }
                    for (uint32_t b = 0; b < items; ++b) {
                        DevWork w;
                        std::memset(&w, 0, sizeof(w));
                        w.inst = i;
                        w.pass = (int32_t)(pbase[i] + off + j);
                        w.tile0 = b * per;
                        w.tile1 = (b + 1) * per;
                        w.part = (int64_t)(part0 + b);
                        w.stride = (int32_t)items;
                        L.work.push_back(w);
                    }
                    bl.threads = std::max(bl.threads, 1 << P.tbits);
                    used.push_back(&P);
                }
                bl.n_items = (int)L.work.size() - bl.item0;
                // longest items first: an instance that fits one tile runs its
                // whole circuit in one workgroup, which must not start last
                // (the order only maps workgroups to items; every item writes
                // its own partial slots)
                std::stable_sort(L.work.begin() + bl.item0, L.work.end(),
                                 [&](const DevWork &a, const DevWork &b) {
                                     auto cost = [&](const DevWork &w) {
                                         const DevPass &P = L.passes[w.pass];
                                         return (double)(P.n_ops + 1) * (w.tile1 - w.tile0) *
                                                (double)(1u << P.k);
                                     };
                                     return cost(a) > cost(b);
                                 });
                bl.smem = 0;
                for (const DevPass *P : used)
                    bl.smem = std::max(bl.smem, (int)smem_plan(P->k, P->n_ops, P->n_diag, P->n_red,
                                                               P->n_phases, bl.threads,
                                                               P->nfree == 0, true)
                                                    .total);
                if (bl.smem > lim)
                    return fail(HUBBARD_ERR_ARG,
                                "a batch instance needs more LDS than a workgroup may use");
                if (bl.n_items > 0)
                    L.launches.push_back(bl);
            }
        }
    }
    for (size_t o = 0; o < n_out; ++o) {
        for (const auto &sg : segs[o]) {
            L.seg_off.push_back(sg.first);
            L.seg_cnt.push_back(sg.second);
        }
        L.seg_ptr.push_back((int32_t)L.seg_off.size());
    }
    L.ws_bytes = L.partial_at + align256(std::max<size_t>(L.n_partial, 1) * sizeof(double));
    return HUBBARD_OK;
}

// Host-only programs of a batch (plans and pass lists, no device tables).
hubbard_status batch_host_programs(const hubbard_t *hs, int n, const int32_t *layers,
                                   std::vector<std::unique_ptr<Program>> &own,
                                   std::vector<const Program *> &progs)
{
    for (int i = 0; i < n; ++i) {
        std::unique_ptr<Program> pr(new Program());
        try {
            plan_program(hs[i], PROG_GRAD, layers[i], max_smem_per_block(), *pr);
            Builder b(hs[i]->m);
            build_lists(b, *pr);
        } catch (const std::exception &ex) {
            return fail(HUBBARD_ERR_NOMEM, std::string("planning: ") + ex.what());
        }
        progs.push_back(pr.get());
        own.push_back(std::move(pr));
    }
    return HUBBARD_OK;
}

struct BatchProgram {
    BatchLayout L;
    std::vector<uint64_t> uids;   // handles whose device tables the instances point into
    uint64_t last_use = 0;        // cache clock of the last call
    DevInstance *d_inst = nullptr;
    DevPass *d_passes = nullptr;
    DevWork *d_work = nullptr;
    int32_t *d_seg_ptr = nullptr, *d_seg_cnt = nullptr;
    int64_t *d_seg_off = nullptr, *d_out_idx = nullptr;
    double *d_scale = nullptr;
    int n = 0;
    // streams of lanes 1.. (default priority), forked from the caller's
    // stream by one event and joined back by one event each per call
    hipStream_t lane_s[kBatchLanes] = {};
    hipEvent_t fork = nullptr, join[kBatchLanes] = {};
    ~BatchProgram()
    {
        if (fork)
            (void)hipEventDestroy(fork);
        for (int l = 1; l < kBatchLanes; ++l) {
            if (join[l])
                (void)hipEventDestroy(join[l]);
            if (lane_s[l])
                (void)hipStreamDestroy(lane_s[l]);
        }
        (void)hipFree(d_inst);
        (void)hipFree(d_passes);
        (void)hipFree(d_work);
        (void)hipFree(d_seg_ptr);
        (void)hipFree(d_seg_cnt);
        (void)hipFree(d_seg_off);
        (void)hipFree(d_out_idx);
        (void)hipFree(d_scale);
    }
};

// Batch programs by their signature: the device, theta and workspace
// pointers (the program's work items point into them) and each instance's
// handle uid, tile generation, layer count and parameter offset.  A program
// points into its instances' device programs, so a change of any member's
// tiles (hubbard_set_tiles, hubbard_tune) or its destruction evicts every
// program that uses it; at most kMaxBatches programs are kept, the least
// recently called one is evicted first.  Eviction waits for the device to go
// idle before freeing (work queued with those tables may still run).
constexpr size_t kMaxBatches = 16;
std::mutex g_batch_mu;
std::map<std::string, std::unique_ptr<BatchProgram>> g_batches;
uint64_t g_batch_clock = 0;
std::atomic<uint64_t> g_next_uid{1};

// g_batch_mu held.  Frees the programs for which pred() holds.
template <typename Pred>
void evict_batches_locked(Pred pred)
{
    bool synced = false;
    for (auto it = g_batches.begin(); it != g_batches.end();) {
        if (!pred(*it->second)) {
            ++it;
            continue;
        }
        if (!synced) {
            (void)hipDeviceSynchronize();
            synced = true;
        }
        it = g_batches.erase(it);
    }
}

void evict_batches_of(uint64_t uid)
{
    std::lock_guard<std::mutex> lk(g_batch_mu);
    evict_batches_locked([uid](const BatchProgram &bp) {
        return std::find(bp.uids.begin(), bp.uids.end(), uid) != bp.uids.end();
    });
}

hubbard_status build_batch(const hubbard_t *hs, int n, const double *theta, const int64_t *toff,
                           const int32_t *layers, char *ws, const BatchConfig &cfg,
                           BatchProgram &bp)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return fail(HUBBARD_ERR_DEVICE, "no current device");
    bp.n = n;
    for (int i = 0; i < n; ++i)
        if (std::find(bp.uids.begin(), bp.uids.end(), hs[i]->uid) == bp.uids.end())
            bp.uids.push_back(hs[i]->uid);
    // the instances' device programs (cached per handle, device and layer count)
    std::vector<const Program *> progs(n);
    std::vector<DevInstance> insts(n);
    for (int i = 0; i < n; ++i) {
        Program *pr;
        DeviceState *ds;
        hubbard_status st = get_program(hs[i], PROG_GRAD, layers[i], &pr, &ds);
        if (st != HUBBARD_OK)
            return st;
        progs[i] = pr;
        DevInstance &I = insts[i];
        std::memset(&I, 0, sizeof(I));
        I.general = pr->general ? 1 : 0;
        I.phases = pr->d_phases;
        I.ops = pr->d_ops;
        I.vb = pr->d_vb;
        I.model = ds->d_model;
        I.theta = theta + toff[i];
    }
    hubbard_status st = batch_layout(hs, n, toff, progs, cfg, bp.L);
    if (st != HUBBARD_OK)
        return st;
    bool used[kBatchLanes] = {};
    for (const BatchLaunch &bl : bp.L.launches)
        used[bl.lane] = true;
    for (int l = 1; l < kBatchLanes; ++l) {
        if (!used[l])
            continue;
        if ((!bp.fork && hipEventCreateWithFlags(&bp.fork, hipEventDisableTiming) != hipSuccess) ||
            hipStreamCreateWithFlags(&bp.lane_s[l], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&bp.join[l], hipEventDisableTiming) != hipSuccess)
            return fail(HUBBARD_ERR_DEVICE, "creating the batch lane streams");
    }
    for (int i = 0; i < n; ++i) {
        insts[i].psi = ws + bp.L.voff[i];
        insts[i].lam = ws + bp.L.voff[i] + align256(vec_bytes(hs[i]));
    }
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
        const int lim = max_smem_per_block();
        const void *fns[] = {
#define HV_BATCH_FNS(GEN, FULL)                                                                 \
    (const void *)k_batch_pass<M_FWD, GEN, FULL, false>,                                        \
        (const void *)k_batch_pass<M_FWD, GEN, FULL, true>,                                     \
        (const void *)k_batch_pass<M_HAM, GEN, FULL, false>,                                    \
        (const void *)k_batch_pass<M_REV, GEN, FULL, false>,                                    \
        (const void *)k_batch_pass<M_FWD, GEN, FULL, false, OPS_ALL>,                           \
        (const void *)k_batch_pass<M_FWD, GEN, FULL, true, OPS_ALL>,                            \
        (const void *)k_batch_pass<M_REV, GEN, FULL, false, OPS_ALL>
            HV_BATCH_FNS(false, false), HV_BATCH_FNS(false, true), HV_BATCH_FNS(true, false),
            HV_BATCH_FNS(true, true)};
#undef HV_BATCH_FNS
        for (const void *f : fns)
            (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    });
    auto up = [](void **dst, const void *src, size_t bytes) -> hipError_t {
        hipError_t e = hipMalloc(dst, std::max<size_t>(bytes, 16));
        if (e == hipSuccess && bytes)
            e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
        return e;
    };
    const BatchLayout &L = bp.L;
    hipError_t e = up((void **)&bp.d_inst, insts.data(), insts.size() * sizeof(DevInstance));
    if (e == hipSuccess)
        e = up((void **)&bp.d_passes, L.passes.data(), L.passes.size() * sizeof(DevPass));
    if (e == hipSuccess)
        e = up((void **)&bp.d_work, L.work.data(), L.work.size() * sizeof(DevWork));
    if (e == hipSuccess)
        e = up((void **)&bp.d_seg_ptr, L.seg_ptr.data(), L.seg_ptr.size() * sizeof(int32_t));
    if (e == hipSuccess)
        e = up((void **)&bp.d_seg_cnt, L.seg_cnt.data(), L.seg_cnt.size() * sizeof(int32_t));
    if (e == hipSuccess)
        e = up((void **)&bp.d_seg_off, L.seg_off.data(), L.seg_off.size() * sizeof(int64_t));
    if (e == hipSuccess)
        e = up((void **)&bp.d_out_idx, L.out_idx.data(), L.out_idx.size() * sizeof(int64_t));
    if (e == hipSuccess)
        e = up((void **)&bp.d_scale, L.scale.data(), L.scale.size() * sizeof(double));
    if (e != hipSuccess)
        return fail(HUBBARD_ERR_DEVICE, std::string("uploading batch: ") + hipGetErrorString(e));
    return HUBBARD_OK;
}

// ===================================================================== ABI

namespace hv {
// For the library's other translation units (the sector form).
const Model *handle_model(hubbard_t h) { return h ? &h->m : nullptr; }
uint64_t handle_uid(hubbard_t h) { return h ? h->uid : 0; }
hubbard_status set_error(hubbard_status s, const std::string &msg) { return fail(s, msg); }
void sector_forget(uint64_t uid);
}  // namespace hv

extern "C" {

const char *hubbard_last_error(void) { return g_err.c_str(); }

hubbard_status hubbard_create(const hubbard_desc *d, hubbard_t *out)
{
    if (!d || !out)
        return fail(HUBBARD_ERR_ARG, "desc and out must not be NULL");
    *out = nullptr;
    hubbard_model *h = nullptr;
    try {
        h = new hubbard_model();
    } catch (...) {
        return fail(HUBBARD_ERR_NOMEM, "allocating handle");
    }
    std::string err = build_model(d->nx, d->ny, d->periodic_x, d->periodic_y, d->t_bond, d->U,
                                  d->V_bond, d->eps_site, d->bond_group, h->m);
    if (!err.empty()) {
        delete h;
        return fail(HUBBARD_ERR_ARG, err);
    }
    h->uid = g_next_uid.fetch_add(1);
    *out = h;
    return HUBBARD_OK;
}

hubbard_status hubbard_create_graph(const hubbard_graph_desc *d, hubbard_t *out)
{
    if (!d || !out)
        return fail(HUBBARD_ERR_ARG, "desc and out must not be NULL");
    *out = nullptr;
    hubbard_model *h = nullptr;
    try {
        h = new hubbard_model();
    } catch (...) {
        return fail(HUBBARD_ERR_NOMEM, "allocating handle");
    }
    std::string err = build_graph_model(d->n_sites, d->n_bonds, d->bond_i, d->bond_j, d->t_bond,
                                        d->U, d->V_bond, d->eps_site, d->bond_group,
                                        d->site_spin, h->m);
    if (!err.empty()) {
        delete h;
        return fail(HUBBARD_ERR_ARG, err);
    }
    h->uid = g_next_uid.fetch_add(1);
    *out = h;
    return HUBBARD_OK;
}

void hubbard_destroy(hubbard_t h)
{
    if (!h)
        return;
    evict_batches_of(h->uid);
    hv::sector_forget(h->uid);
    if (h->ev_ready)
        for (int j = 0; j < 4; ++j)
            (void)hipEventDestroy(h->ev[j]);
    for (hipEvent_t e : h->kev)
        (void)hipEventDestroy(e);
    for (auto &kv : h->dev) {
        (void)hipSetDevice(kv.first);
        kv.second.progs.clear();
        (void)hipFree(kv.second.d_model);
    }
    delete h;
}

hubbard_status hubbard_query(hubbard_t h, int32_t *n_qubits, int32_t *n_bonds, int32_t *n_groups,
                             int32_t *params_per_layer, uint64_t *neel_index)
{
    if (!h)
        return fail(HUBBARD_ERR_ARG, "NULL handle");
    if (n_qubits)
        *n_qubits = h->m.nq;
    if (n_bonds)
        *n_bonds = h->m.nb;
    if (n_groups)
        *n_groups = h->m.ngroups;
    if (params_per_layer)
        *params_per_layer = h->m.params_per_layer();
    if (neel_index)
        *neel_index = h->m.neel;
    return HUBBARD_OK;
}

hubbard_status hubbard_bonds(hubbard_t h, int32_t *bi, int32_t *bj, int32_t *group)
{
    if (!h)
        return fail(HUBBARD_ERR_ARG, "NULL handle");
    for (int b = 0; b < h->m.nb; ++b) {
        if (bi)
            bi[b] = h->m.bi[b];
        if (bj)
            bj[b] = h->m.bj[b];
        if (group)
            group[b] = h->m.slot[b] - 1;
    }
    return HUBBARD_OK;
}

hubbard_status hubbard_workspace_size(hubbard_t h, int32_t n_layers, int32_t op, size_t *bytes)
{
    if (!h || !bytes || n_layers < 0)
        return fail(HUBBARD_ERR_ARG, "bad arguments to hubbard_workspace_size");
    if (op != HUBBARD_OP_ENERGY && op != HUBBARD_OP_ENERGY_GRAD && op != HUBBARD_OP_OVERLAP_GRAD)
        return fail(HUBBARD_ERR_ARG, "unknown op");
    Program pr;
    try {
        plan_program(h, op == HUBBARD_OP_ENERGY ? PROG_ENERGY : PROG_GRAD, n_layers,
                     max_smem_per_block(), pr);   // overlap_grad runs the gradient program
    } catch (const std::exception &ex) {
        return fail(HUBBARD_ERR_NOMEM, ex.what());
    }
    Builder b(h->m);
    b.add(pr.h_fwd, 0, false, true);
    b.add(pr.h_ham, op != HUBBARD_OP_ENERGY ? 2 : 0, true);
    b.add(pr.h_rev, 1, false);
    b.add(pr.h_exp, 2, false);
    size_t partial = align256(b.row_param.size() * (size_t)kGridMax * sizeof(double));
    size_t nvec = (op == HUBBARD_OP_ENERGY) ? 1 : 2;
    *bytes = nvec * align256(vec_bytes(h)) + partial;
    if (op == HUBBARD_OP_OVERLAP_GRAD)   // the overlap's partial sums, its value, one spare
        *bytes += align256((size_t)kVecBlocks * sizeof(double2)) + 256;
    return HUBBARD_OK;
}

hubbard_status hubbard_init_neel(hubbard_t h, void *psi_dev, void *stream)
{
    if (!h || !psi_dev)
        return fail(HUBBARD_ERR_ARG, "NULL handle or psi");
    return run_init(h, (double2 *)psi_dev, (hipStream_t)stream);
}

hubbard_status ansatz_apply(hubbard_t h, const double *theta_dev, int32_t n_layers, void *psi_dev,
                            void *stream)
{
    if (!h || !psi_dev || n_layers < 0 || (n_layers > 0 && !theta_dev))
        return fail(HUBBARD_ERR_ARG, "bad arguments to ansatz_apply");
    if (n_layers == 0)
        return HUBBARD_OK;
    Program *pr;
    DeviceState *ds;
    hubbard_status st = get_program(h, PROG_ANSATZ, n_layers, &pr, &ds);
    if (st != HUBBARD_OK)
        return st;
    h->ev_used = 0;
    h->kmode.clear();
    mark(h, 0, (hipStream_t)stream);
    st = run_forward(*pr, *ds, theta_dev, (double2 *)psi_dev, (hipStream_t)stream, h);
    mark(h, 1, (hipStream_t)stream);
    return st;
}

hubbard_status hamiltonian_apply(hubbard_t h, const void *psi_dev, void *out_dev, void *stream)
{
    if (!h || !psi_dev || !out_dev)
        return fail(HUBBARD_ERR_ARG, "NULL argument to hamiltonian_apply");
    const char *a = (const char *)psi_dev, *b = (const char *)out_dev;
    const size_t nb = vec_bytes(h);
    if (a < b + nb && b < a + nb)
        return fail(HUBBARD_ERR_ARG, "out_dev overlaps psi_dev");
    Program *pr;
    DeviceState *ds;
    hubbard_status st = get_program(h, PROG_HAM, 0, &pr, &ds);
    if (st != HUBBARD_OK)
        return st;
    h->ev_used = 0;
    h->kmode.clear();
    mark(h, 1, (hipStream_t)stream);
    st = run_ham(*pr, *ds, (const double2 *)psi_dev, (double2 *)out_dev, nullptr,
                 (hipStream_t)stream, h);
    mark(h, 2, (hipStream_t)stream);
    return st;
}

hubbard_status energy(hubbard_t h, const double *theta_dev, int32_t n_layers, double *E_dev,
                      void *ws_dev, size_t ws_bytes, void *stream)
{
    if (!h || !E_dev || !ws_dev || n_layers < 0 || (n_layers > 0 && !theta_dev))
        return fail(HUBBARD_ERR_ARG, "bad arguments to energy");
    Program *pr;
    DeviceState *ds;
    hubbard_status st = get_program(h, PROG_ENERGY, n_layers, &pr, &ds);
    if (st != HUBBARD_OK)
        return st;
    const size_t vb = align256(vec_bytes(h));
    if (ws_bytes < vb + pr->partial_bytes)
        return fail(HUBBARD_ERR_SIZE, "workspace too small for energy");
    hipStream_t s = (hipStream_t)stream;
    double2 *psi = (double2 *)ws_dev;
    double *partial = (double *)((char *)ws_dev + vb);
    // the first forward pass starts from |b0> itself (no init pass)
    const bool from_start = !pr->fwd.pass.empty();
    if (!from_start && (st = run_init(h, psi, s)) != HUBBARD_OK)
        return st;
    h->ev_used = 0;
    h->kmode.clear();
    mark(h, 0, s);
    if ((st = run_forward(*pr, *ds, theta_dev, psi, s, h, VecLayout(), from_start)) != HUBBARD_OK)
        return st;
    mark(h, 1, s);
    launch_list<M_EXP>(*pr, *ds, pr->exp, nullptr, psi, nullptr, partial, s, h);
    if ((st = check_launch("expectation pass")) != HUBBARD_OK)
        return st;
    mark(h, 2, s);
    return run_reduce(*pr, partial, E_dev, nullptr, s);
}

}  // extern "C"

namespace {

// The launch sequence of energy_grad on given psi, lambda and partial-sum
// buffers.  th: the handle whose timing events are recorded, or NULL (no
// event is created or recorded).
hubbard_status grad_sequence(hubbard_model *h, hubbard_model *th, const Program &pr,
                             const DeviceState &ds, const double *theta_dev, double *E_dev,
                             double *grad_dev, double2 *psi, double2 *lam, double *partial,
                             VecLayout vl, hipStream_t s)
{
    hubbard_status st;
    // the first forward pass starts from |b0> itself (no init pass), and the
    // last reverse pass stores nothing: only its reductions are needed
    const bool from_start = !pr.fwd.pass.empty();
    if (!from_start && (st = run_init(h, psi, s, vl)) != HUBBARD_OK)
        return st;
    if (th) {
        th->ev_used = 0;
        th->kmode.clear();
        mark(th, 0, s);
    }
    if ((st = run_forward(pr, ds, theta_dev, psi, s, th, vl, from_start)) != HUBBARD_OK)
        return st;
    if (th)
        mark(th, 1, s);
    if ((st = run_ham(pr, ds, psi, lam, partial, s, th, vl)) != HUBBARD_OK)
        return st;
    if (th)
        mark(th, 2, s);
    launch_list<M_REV>(pr, ds, pr.rev, theta_dev, psi, lam, partial, s, th, vl, 0, PF_NO_STORE);
    if ((st = check_launch("reverse pass")) != HUBBARD_OK)
        return st;
    if (th)
        mark(th, 3, s);
    return run_reduce(pr, partial, E_dev, grad_dev, s);
}

// ------------------------------------------------- library-owned scratch --
// energy_grad_noalloc keeps psi, lambda and the partial sums in this array
// instead of a caller workspace: psi at offset 0 and lambda at
// kScratchVecBytes (2^20 amplitudes each, plain layout), the partial rows
// (kGridMax doubles each, up to kScratchRows) after them.  Each device that
// runs the library holds its own copy until the process ends.  In host code
// the name is only a stand-in for the symbol: kernels get the device
// address from hipGetSymbolAddress (per device, on that device's first
// call), never the name.
constexpr int kScratchQubits = 20;
constexpr size_t kScratchVecBytes = ((size_t)16) << kScratchQubits;
constexpr int kScratchRows = 128;
constexpr size_t kScratchBytes =
    2 * kScratchVecBytes + (size_t)kScratchRows * kGridMax * sizeof(double);   // 48 MiB
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, char *> g_scratch_ptr;   // device -> address of its copy of `scratch`

hubbard_status scratch_address(int dev, char **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        char *p = nullptr;
        hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HUBBARD_ERR_DEVICE,
                        std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        it = g_scratch_ptr.emplace(dev, p).first;
    }
    *out = it->second;
    return HUBBARD_OK;
}

// The handle's uploaded program of (kind, layers) on the current device, or
// NULL: looks only, never plans or uploads (no allocation).
Program *find_program(hubbard_model *h, int dev, int kind, int layers, DeviceState **dsout)
{
    std::lock_guard<std::mutex> lk(h->mu);
    auto d = h->dev.find(dev);
    if (d == h->dev.end() || !d->second.d_model)
        return nullptr;
    auto it = d->second.progs.find(std::make_pair(kind, layers));
    if (it == d->second.progs.end())
        return nullptr;
    *dsout = &d->second;
    return it->second.get();
}

}  // namespace

extern "C" {

hubbard_status energy_grad_noalloc(hubbard_t h, const double *theta_dev, int32_t n_layers,
                                   double *E_dev, double *grad_dev, void *stream)
{
    if (!h || !E_dev || n_layers < 0 || (n_layers > 0 && (!theta_dev || !grad_dev)))
        return fail(HUBBARD_ERR_ARG, "bad arguments to energy_grad_noalloc");
    if (h->m.nq > kScratchQubits)
        return fail(HUBBARD_ERR_SIZE, "energy_grad_noalloc: " + std::to_string(h->m.nq) +
                                          " qubits exceed the library scratch (at most " +
                                          std::to_string(kScratchQubits) + ")");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(HUBBARD_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    DeviceState *ds = nullptr;
    Program *pr = find_program(h, dev, PROG_GRAD, n_layers, &ds);
    if (!pr)
        return fail(HUBBARD_ERR_STATE, "energy_grad_noalloc: no uploaded plan for this handle, "
                                       "device and layer count (call energy_grad once first)");
    if (pr->n_rows > kScratchRows)
        return fail(HUBBARD_ERR_SIZE, "energy_grad_noalloc: " + std::to_string(pr->n_rows) +
                                          " reduction rows exceed the library scratch (at most " +
                                          std::to_string(kScratchRows) + ")");
    char *base = nullptr;
    hubbard_status st = scratch_address(dev, &base);
    if (st != HUBBARD_OK)
        return st;
    double2 *psi = (double2 *)base;
    double2 *lam = (double2 *)(base + kScratchVecBytes);
    double *partial = (double *)(base + 2 * kScratchVecBytes);
    return grad_sequence(h, nullptr, *pr, *ds, theta_dev, E_dev, grad_dev, psi, lam, partial,
                         VecLayout(), (hipStream_t)stream);
}

hubbard_status energy_grad(hubbard_t h, const double *theta_dev, int32_t n_layers, double *E_dev,
                           double *grad_dev, void *ws_dev, size_t ws_bytes, void *stream)
{
    if (!h || !E_dev || !ws_dev || n_layers < 0 || (n_layers > 0 && (!theta_dev || !grad_dev)))
        return fail(HUBBARD_ERR_ARG, "bad arguments to energy_grad");
    Program *pr;
    DeviceState *ds;
    hubbard_status st = get_program(h, PROG_GRAD, n_layers, &pr, &ds);
    if (st != HUBBARD_OK)
        return st;
    const size_t vb = align256(vec_bytes(h));
    if (ws_bytes < 2 * vb + pr->partial_bytes)
        return fail(HUBBARD_ERR_SIZE, "workspace too small for energy_grad");
    hipStream_t s = (hipStream_t)stream;
    // psi and lambda share the first 2 vb bytes (layout of grad_layout)
    const VecLayout vl = grad_layout(h);
    double2 *psi = (double2 *)ws_dev;
    double2 *lam = vl.ilv == kPlainVec ? (double2 *)((char *)ws_dev + vb)
                                       : psi + ((size_t)1 << vl.ilv);
    double *partial = (double *)((char *)ws_dev + 2 * vb);
    return grad_sequence(h, h, *pr, *ds, theta_dev, E_dev, grad_dev, psi, lam, partial, vl, s);
}

hubbard_status hubbard_batch_workspace_size(const hubbard_t *hs, int32_t n,
                                            const int32_t *n_layers, size_t *bytes)
{
    if (!hs || n < 1 || !n_layers || !bytes)
        return fail(HUBBARD_ERR_ARG, "bad arguments to hubbard_batch_workspace_size");
    for (int i = 0; i < n; ++i)
        if (!hs[i] || n_layers[i] < 0)
            return fail(HUBBARD_ERR_ARG, "bad instance " + std::to_string(i) + " in batch");
    std::vector<std::unique_ptr<Program>> own;
    std::vector<const Program *> progs;
    hubbard_status st = batch_host_programs(hs, n, n_layers, own, progs);
    if (st != HUBBARD_OK)
        return st;
    std::vector<int64_t> toff(n, 0);
    BatchLayout L;
    st = batch_layout(hs, n, toff.data(), progs, batch_config(), L);
    if (st != HUBBARD_OK)
        return st;
    *bytes = L.ws_bytes;
    return HUBBARD_OK;
}

hubbard_status energy_grad_batch(const hubbard_t *hs, int32_t n, const double *theta_dev,
                                 const int64_t *theta_off, const int32_t *n_layers,
                                 double *E_dev, double *grad_dev, void *ws_dev, size_t ws_bytes,
                                 void *stream)
{
    if (!hs || n < 1 || !theta_dev || !theta_off || !n_layers || !E_dev || !grad_dev || !ws_dev)
        return fail(HUBBARD_ERR_ARG, "bad arguments to energy_grad_batch");
    for (int i = 0; i < n; ++i) {
        if (!hs[i] || n_layers[i] < 0 || theta_off[i] < 0)
            return fail(HUBBARD_ERR_ARG, "bad instance " + std::to_string(i) + " in batch");
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    const BatchConfig cfg = batch_config();
    std::string key = std::to_string(dev) + ":" + std::to_string((uintptr_t)theta_dev) + ":" +
                      std::to_string((uintptr_t)ws_dev) + ":" + std::to_string(cfg.items) + "." +
                      std::to_string(cfg.lanes);
    for (int i = 0; i < n; ++i)
        key += ":" + std::to_string(hs[i]->uid) + "." + std::to_string(hs[i]->gen) + "/" +
               std::to_string(n_layers[i]) + "/" + std::to_string(theta_off[i]);
    hipStream_t s = (hipStream_t)stream;
    BatchProgram *bp = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_batch_mu);
        auto it = g_batches.find(key);
        if (it == g_batches.end()) {
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
                return fail(HUBBARD_ERR_STATE, "first call of a batch must happen outside graph "
                                               "capture (it uploads the batch tables)");
            if (g_batches.size() >= kMaxBatches) {
                const BatchProgram *lru = nullptr;
                for (const auto &kv : g_batches)
                    if (!lru || kv.second->last_use < lru->last_use)
                        lru = kv.second.get();
                evict_batches_locked([lru](const BatchProgram &bp) { return &bp == lru; });
            }
            std::unique_ptr<BatchProgram> nb(new BatchProgram());
            hubbard_status st = build_batch(hs, n, theta_dev, theta_off, n_layers,
                                            (char *)ws_dev, cfg, *nb);
            if (st != HUBBARD_OK)
                return st;
            it = g_batches.emplace(key, std::move(nb)).first;
        }
        bp = it->second.get();
        bp->last_use = ++g_batch_clock;
    }
    const BatchLayout &L = bp->L;
    if (ws_bytes < L.ws_bytes)
        return fail(HUBBARD_ERR_SIZE, "workspace too small for energy_grad_batch");
    double *partial = (double *)((char *)ws_dev + L.partial_at);
    if (bp->fork && hipEventRecord(bp->fork, s) != hipSuccess)
        return fail(HUBBARD_ERR_DEVICE, "forking the batch lane streams");
    for (int l = 1; l < kBatchLanes; ++l)
        if (bp->lane_s[l] && hipStreamWaitEvent(bp->lane_s[l], bp->fork, 0) != hipSuccess)
            return fail(HUBBARD_ERR_DEVICE, "forking the batch lane streams");
    for (const BatchLaunch &bl : L.launches) {
        const DevWork *w = bp->d_work + bl.item0;
        hipStream_t ls = bl.lane == 0 ? s : bp->lane_s[bl.lane];
#define HV_BATCH_LAUNCH(MODE, GEN, FULL, START, OPS)                                            \
    hipLaunchKernelGGL((k_batch_pass<MODE, GEN, FULL, START, OPS>), dim3(bl.n_items),          \
                       dim3(bl.threads), bl.smem, ls, bp->d_inst, bp->d_passes, w, partial)
#define HV_BATCH_GATES(MODE, GEN, FULL, START)                                                  \
    do {                                                                                        \
        if (L.np)                                                                               \
            HV_BATCH_LAUNCH(MODE, GEN, FULL, START, OPS_ALL);                                   \
        else                                                                                    \
            HV_BATCH_LAUNCH(MODE, GEN, FULL, START, OPS_HVA);                                   \
    } while (0)
#define HV_BATCH_MODE(GEN, FULL)                                                                \
    do {                                                                                        \
        if (bl.mode == M_FWD && bl.start)                                                       \
            HV_BATCH_GATES(M_FWD, GEN, FULL, true);                                             \
        else if (bl.mode == M_FWD)                                                              \
            HV_BATCH_GATES(M_FWD, GEN, FULL, false);                                            \
        else if (bl.mode == M_HAM)                                                              \
            HV_BATCH_LAUNCH(M_HAM, GEN, FULL, false, OPS_HVA);                                  \
        else                                                                                    \
            HV_BATCH_GATES(M_REV, GEN, FULL, false);                                            \
    } while (0)
        if (L.general) {
            if (bl.full)
                HV_BATCH_MODE(true, true);
            else
                HV_BATCH_MODE(true, false);
        } else {
            if (bl.full)
                HV_BATCH_MODE(false, true);
            else
                HV_BATCH_MODE(false, false);
        }
#undef HV_BATCH_MODE
#undef HV_BATCH_GATES
#undef HV_BATCH_LAUNCH
    }
    for (int l = 1; l < kBatchLanes; ++l)
        if (bp->lane_s[l] && (hipEventRecord(bp->join[l], bp->lane_s[l]) != hipSuccess ||
                              hipStreamWaitEvent(s, bp->join[l], 0) != hipSuccess))
            return fail(HUBBARD_ERR_DEVICE, "joining the batch lane streams");
    hipLaunchKernelGGL(k_reduce_seg, dim3((unsigned)L.scale.size()), dim3(256), 0, s, partial,
                       bp->d_seg_ptr, bp->d_seg_off, bp->d_seg_cnt, bp->d_scale, bp->d_out_idx, n,
                       E_dev, grad_dev);
    return check_launch("batch");
}

hubbard_status hubbard_plan_dump(hubbard_t h, int32_t n_layers, int32_t which, int32_t *buf,
                                 int64_t cap, int64_t *len)
{
    if (!h || !len || n_layers < 0 || which < 0 || which > 3)
        return fail(HUBBARD_ERR_ARG, "bad arguments to hubbard_plan_dump");
    Program pr;
    try {
        plan_program(h, which == 3 ? PROG_ENERGY : PROG_GRAD, n_layers, max_smem_per_block(), pr);
    } catch (const std::exception &ex) {
        return fail(HUBBARD_ERR_NOMEM, ex.what());
    }
    const std::vector<HostPass> &ps =
        which == 0 ? pr.h_fwd : which == 1 ? pr.h_ham : which == 2 ? pr.h_rev : pr.h_exp;
    std::vector<int32_t> out;
    out.push_back((int32_t)ps.size());
    for (const HostPass &p : ps) {
        out.push_back((int32_t)p.tile.size());
        for (int b : p.tile)
            out.push_back(b);
        out.push_back(p.flags);
        out.push_back((int32_t)p.ops.size());
        for (const HostOp &o : p.ops) {
            out.push_back(o.kind);
            out.push_back(o.param);
            out.push_back(o.p);
            out.push_back(o.q);
            out.push_back((int32_t)o.umask);
            out.push_back((int32_t)o.emask);
            out.push_back((int32_t)o.vbonds.size());
            for (int b : o.vbonds)
                out.push_back(b);
        }
    }
    *len = (int64_t)out.size();
    if (buf && cap >= (int64_t)out.size())
        std::memcpy(buf, out.data(), out.size() * sizeof(int32_t));
    else if (buf)
        return fail(HUBBARD_ERR_SIZE, "buffer too small for plan dump");
    return HUBBARD_OK;
}

hubbard_status hubbard_set_tiles(hubbard_t h, int32_t fwd_k, int32_t rev_k, int32_t c)
{
    if (!h || fwd_k < 2 || fwd_k > kMaxTileBits || rev_k < 2 || rev_k > kMaxTileBits || c < 0 ||
        c > fwd_k || c > rev_k)
        return fail(HUBBARD_ERR_ARG, "tile bits must be in [2, 13] and c <= k");
    // a hopping term on two qubits above the contiguous low bits needs two
    // more tile bits (unless a tile holds the whole state)
    for (int k : {fwd_k, rev_k})
        if (k - c < 2 && k < h->m.nq)
            return fail(HUBBARD_ERR_ARG, "a tile needs at least two bits beyond its c contiguous "
                                         "low bits (or all qubits)");
    // batches point into the device programs dropped below; evict them first
    // (lock order: the batch cache before a handle)
    evict_batches_of(h->uid);
    std::lock_guard<std::mutex> lk(h->mu);
    h->fwd_tc = TileConfig{fwd_k, c};
    h->rev_tc = TileConfig{rev_k, c};
    ++h->gen;
    for (auto &kv : h->dev)
        kv.second.progs.clear();
    return HUBBARD_OK;
}

hubbard_status hubbard_set_ansatz(hubbard_t h, int32_t ansatz)
{
    if (!h || (ansatz != HUBBARD_ANSATZ_HVA && ansatz != HUBBARD_ANSATZ_NP))
        return fail(HUBBARD_ERR_ARG, "ansatz must be HUBBARD_ANSATZ_HVA or HUBBARD_ANSATZ_NP");
    evict_batches_of(h->uid);   // lock order: the batch cache before a handle
    std::lock_guard<std::mutex> lk(h->mu);
    if (h->m.ansatz == ansatz)
        return HUBBARD_OK;
    h->m.ansatz = ansatz;
    ++h->gen;
    for (auto &kv : h->dev)
        kv.second.progs.clear();
    std::lock_guard<std::mutex> lk2(h->plan_mu);
    h->fwd_plans.clear();
    return HUBBARD_OK;
}

hubbard_status hubbard_param_count(hubbard_t h, int32_t n_layers, int64_t *count)
{
    if (!h || n_layers < 0 || !count)
        return fail(HUBBARD_ERR_ARG, "bad arguments to hubbard_param_count");
    *count = h->m.n_params(n_layers);
    return HUBBARD_OK;
}

hubbard_status hubbard_get_tiles(hubbard_t h, int32_t *cfg)
{
    if (!h || !cfg)
        return fail(HUBBARD_ERR_ARG, "NULL argument to hubbard_get_tiles");
    cfg[0] = h->fwd_tc.k;
    cfg[1] = h->rev_tc.k;
    cfg[2] = h->fwd_tc.c;
    return HUBBARD_OK;
}

hubbard_status hubbard_tune(hubbard_t h, int32_t n_layers, const double *theta_dev, void *ws_dev,
                            size_t ws_bytes, void *stream, int32_t reps, int32_t *table,
                            int32_t table_cap, int32_t *n_tried, float *table_ms)
{
    if (!h || n_layers < 1 || !theta_dev || !ws_dev || reps < 1 || !n_tried)
        return fail(HUBBARD_ERR_ARG, "bad arguments to hubbard_tune");
    hipStream_t s = (hipStream_t)stream;
    const int n = h->m.nq;
    std::vector<std::array<int, 3>> cands;
    for (int fk : {11, 12, 13})
        for (int rk : {10, 11, 12})
            for (int c : {4, 5}) {
                int f = std::min(fk, n), r = std::min(rk, n), cc = std::min(c, std::min(f, r));
                std::array<int, 3> x{f, r, cc};
                if (std::find(cands.begin(), cands.end(), x) == cands.end())
                    cands.push_back(x);
            }
    const TileConfig keep_f = h->fwd_tc, keep_r = h->rev_tc;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(HUBBARD_ERR_DEVICE, "creating tuning events");
    double *E = nullptr, *g = nullptr;
    const int P = h->m.n_params(n_layers);
    if (hipMalloc((void **)&E, sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&g, sizeof(double) * (size_t)P) != hipSuccess) {
        (void)hipFree(E);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return fail(HUBBARD_ERR_NOMEM, "tuning outputs");
    }
    float best = -1.0f;
    std::array<int, 3> bestc{keep_f.k, keep_r.k, keep_f.c};
    int tried = 0;
    hubbard_status st = HUBBARD_OK;
    for (const auto &cf : cands) {
        hubbard_set_tiles(h, cf[0], cf[1], cf[2]);
        size_t need = 0;
        if (hubbard_workspace_size(h, n_layers, HUBBARD_OP_ENERGY_GRAD, &need) != HUBBARD_OK ||
            need > ws_bytes)
            continue;
        if ((st = energy_grad(h, theta_dev, n_layers, E, g, ws_dev, ws_bytes, stream)) !=
            HUBBARD_OK)
            break;   // (also plans and uploads this configuration)
        float ms = 1e30f;
        for (int r = 0; r < reps; ++r) {
            (void)hipEventRecord(e0, s);
            energy_grad(h, theta_dev, n_layers, E, g, ws_dev, ws_bytes, stream);
            (void)hipEventRecord(e1, s);
            float t = 0.0f;
            if (hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
                st = fail(HUBBARD_ERR_DEVICE, "tuning timing");
                break;
            }
            ms = std::min(ms, t);
        }
        if (st != HUBBARD_OK)
            break;
        if (table && tried < table_cap) {
            table[3 * tried] = cf[0];
            table[3 * tried + 1] = cf[1];
            table[3 * tried + 2] = cf[2];
            if (table_ms)
                table_ms[tried] = ms;
        }
        ++tried;
        if (best < 0.0f || ms < best) {
            best = ms;
            bestc = cf;
        }
    }
    (void)hipFree(E);
    (void)hipFree(g);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *n_tried = tried;
    if (st != HUBBARD_OK) {
        // back to the configuration on entry (drops the candidate's programs)
        const std::string err = g_err;
        hubbard_set_tiles(h, keep_f.k, keep_r.k, keep_f.c);
        g_err = err;
        return st;
    }
    hubbard_set_tiles(h, bestc[0], bestc[1], bestc[2]);
    return HUBBARD_OK;
}

hubbard_status hubbard_batch_set_config(int32_t items, int32_t lanes)
{
    if (items < 1 || items > 4096 || (items & (items - 1)) != 0 || lanes < 1 ||
        lanes > kBatchLanes)
        return fail(HUBBARD_ERR_ARG, "batch items must be a power of two in [1, 4096] and "
                                     "lanes in [1, 4]");
    std::lock_guard<std::mutex> lk(g_batch_cfg_mu);
    g_batch_cfg.items = items;
    g_batch_cfg.lanes = lanes;
    return HUBBARD_OK;
}

hubbard_status hubbard_batch_get_config(int32_t *items, int32_t *lanes)
{
    if (!items || !lanes)
        return fail(HUBBARD_ERR_ARG, "NULL argument to hubbard_batch_get_config");
    const BatchConfig c = batch_config();
    *items = c.items;
    *lanes = c.lanes;
    return HUBBARD_OK;
}

hubbard_status hubbard_batch_cached(int32_t *count)
{
    if (!count)
        return fail(HUBBARD_ERR_ARG, "NULL count");
    std::lock_guard<std::mutex> lk(g_batch_mu);
    *count = (int32_t)g_batches.size();
    return HUBBARD_OK;
}

hubbard_status hubbard_set_timing(hubbard_t h, int32_t enable)
{
    if (!h)
        return fail(HUBBARD_ERR_ARG, "NULL handle");
    h->timing = enable != 0;
    return HUBBARD_OK;
}

hubbard_status hubbard_phase_ms(hubbard_t h, float *fwd_ms, float *ham_ms, float *rev_ms)
{
    if (!h || !fwd_ms || !ham_ms || !rev_ms)
        return fail(HUBBARD_ERR_ARG, "NULL argument to hubbard_phase_ms");
    *fwd_ms = *ham_ms = *rev_ms = -1.0f;
    if (!h->ev_ready)
        return fail(HUBBARD_ERR_STATE, "timing was not enabled before the last call");
    auto span = [&](int a, int b, float *out) -> hubbard_status {
        if ((h->ev_used & (1 << a)) && (h->ev_used & (1 << b))) {
            hipError_t e = hipEventSynchronize(h->ev[b]);
            if (e == hipSuccess)
                e = hipEventElapsedTime(out, h->ev[a], h->ev[b]);
            if (e != hipSuccess)
                return fail(HUBBARD_ERR_DEVICE, std::string("event timing: ") + hipGetErrorString(e));
        }
        return HUBBARD_OK;
    };
    hubbard_status st = span(0, 1, fwd_ms);
    if (st == HUBBARD_OK)
        st = span(1, 2, ham_ms);
    if (st == HUBBARD_OK)
        st = span(2, 3, rev_ms);
    return st;
}

hubbard_status hubbard_kernel_ms(hubbard_t h, int32_t mode, float *total_ms, int32_t *launches)
{
    if (!h || !total_ms || !launches || mode < 0 || mode > 3)
        return fail(HUBBARD_ERR_ARG, "bad arguments to hubbard_kernel_ms");
    *total_ms = 0.0f;
    *launches = 0;
    for (size_t i = 0; i < h->kmode.size(); ++i) {
        if (h->kmode[i] != mode)
            continue;
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(h->kev[2 * i + 1]);
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, h->kev[2 * i], h->kev[2 * i + 1]);
        if (e != hipSuccess)
            return fail(HUBBARD_ERR_DEVICE, std::string("event timing: ") + hipGetErrorString(e));
        *total_ms += ms;
        ++*launches;
    }
    return HUBBARD_OK;
}

}  // extern "C"

// ============================================================== drivers
// Host drivers built on the pass kernels and the vector kernels: overlaps
// (the fidelity of Sec. 3.4) and the Krylov ground state of H in the
// particle-number sector of a start vector (the reference energies and
// states against which Sec. 3.1 measures the VQE error and Sec. 3.4 the
// fidelity).

namespace {

size_t vec_partial_bytes() { return align256((size_t)kVecBlocks * sizeof(double2)); }

// Workgroup split of k_bit_moments for an n-qubit vector.
struct MomentLayout {
    int lo, mid, r, n_blk, stride;
    size_t partial_bytes;
};
MomentLayout moment_layout(int n)
{
    MomentLayout m;
    m.lo = std::min(kMomLo, n);
    m.mid = std::min(kMomMid, n - m.lo);
    m.r = m.lo + m.mid;
    m.n_blk = 1 << (n - m.r);
    m.stride = 1 + m.r * (m.r + 1) / 2;
    m.partial_bytes = align256((size_t)m.n_blk * m.stride * sizeof(double));
    return m;
}

unsigned vec_grid(uint64_t n)
{
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)kVecBlocks,
                                                               (n + kVecThreads - 1) / kVecThreads));
}

// <a|b> summed on the host in block order (waits for the stream).
hubbard_status host_dot(const double2 *a, const double2 *b, uint64_t n, double2 *partial,
                        hipStream_t s, double *re, double *im)
{
    const unsigned g = vec_grid(n);
    hipLaunchKernelGGL(k_vdot, dim3(g), dim3(kVecThreads), 0, s, a, b, n, partial);
    std::vector<double2> hp(g);
    hipError_t e = hipMemcpyAsync(hp.data(), partial, g * sizeof(double2),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return fail(HUBBARD_ERR_DEVICE, std::string("dot: ") + hipGetErrorString(e));
    double r = 0.0, i = 0.0;
    for (unsigned k = 0; k < g; ++k) {
        r += hp[k].x;
        i += hp[k].y;
    }
    *re = r;
    *im = i;
    return HUBBARD_OK;
}

// One step of the recurrence: w <- H v - alpha v - beta u with alpha =
// <v|H v> (computed unless given), returns ||w||^2.  has_alpha: use *alpha.
hubbard_status krylov_step(const hv::ApplyH &apply, const double2 *v, const double2 *u,
                           double2 *w, double beta, bool has_alpha, double *alpha,
                           double *wnorm2, double2 *partial, uint64_t n, hipStream_t s)
{
    hubbard_status st = apply(v, w);
    if (st != HUBBARD_OK)
        return st;
    if (!has_alpha) {
        double im = 0.0;
        if ((st = host_dot(v, w, n, partial, s, alpha, &im)) != HUBBARD_OK)
            return st;
    }
    const unsigned g = vec_grid(n);
    // beta = 0 on the first step: u is then v itself (any finite vector)
    hipLaunchKernelGGL(k_krylov_update, dim3(g), dim3(kVecThreads), 0, s, w, v, beta > 0.0 ? u : v,
                       *alpha, beta, n, partial);
    std::vector<double2> hp(g);
    hipError_t e = hipMemcpyAsync(hp.data(), partial, g * sizeof(double2),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return fail(HUBBARD_ERR_DEVICE, std::string("krylov update: ") + hipGetErrorString(e));
    double acc = 0.0;
    for (unsigned k = 0; k < g; ++k)
        acc += hp[k].x;
    *wnorm2 = acc;
    return HUBBARD_OK;
}

}  // namespace

namespace hv {

// The Lanczos recurrence on n amplitudes with the Hamiltonian given by
// `apply` (see hubbard_lanczos): buf holds three vectors of n, partial the
// vector kernels' block partials; gs (optional) receives the Ritz vector.
hubbard_status lanczos_run(const ApplyH &apply, uint64_t n, const double2 *start_dev,
                           int32_t max_iter, double tol, double *E0, int32_t *iters,
                           double *residual, double2 *gs_dev, double2 *const buf[3],
                           double2 *partial, hipStream_t s)
{
    hubbard_status st;
    const unsigned g = vec_grid(n);
    double nrm2 = 0.0, im = 0.0;
    if ((st = host_dot(start_dev, start_dev, n, partial, s,
                       &nrm2, &im)) != HUBBARD_OK)
        return st;
    if (!(nrm2 > 0.0) || !std::isfinite(nrm2))
        return fail(HUBBARD_ERR_ARG, "hubbard_lanczos: start vector has zero or non-finite norm");
    const double inv0 = 1.0 / std::sqrt(nrm2);
    // pass 1: the recurrence, alpha_j and beta_j, until the Ritz residual
    // beta_j |s_j| of the lowest Ritz pair is below tol (or an invariant
    // subspace: beta_j vanishes)
    std::vector<double> alpha, beta, svec;
    double lam = 0.0, res = 0.0;
    {
        double2 *v = buf[0], *u = buf[1], *w = buf[2];
        hipLaunchKernelGGL(k_vscale, dim3(g), dim3(kVecThreads), 0, s, v,
                           start_dev, inv0, n);
        double bprev = 0.0;
        for (int j = 0; j < max_iter; ++j) {
            double a = 0.0, w2 = 0.0;
            if ((st = krylov_step(apply, v, u, w, bprev, false, &a, &w2, partial, n, s)) !=
                HUBBARD_OK)
                return st;
            alpha.push_back(a);
            const double b = std::sqrt(w2);
            svec.assign(alpha.size(), 0.0);
            lam = tridiag_lowest(alpha.data(), beta.data(), (int)alpha.size(), svec.data());
            res = b * std::fabs(svec.back());
            const double scale = std::max(1.0, std::fabs(lam));
            if (res <= tol * scale || b <= 1e-14 * scale)
                break;
            beta.push_back(b);
            hipLaunchKernelGGL(k_vscale, dim3(g), dim3(kVecThreads), 0, s, u, w, 1.0 / b, n);
            std::swap(u, v);   // u <- v_j, v <- v_{j+1}
            bprev = b;
        }
    }
    *E0 = lam;
    if (iters)
        *iters = (int32_t)alpha.size();
    if (residual)
        *residual = res;
    if (!gs_dev)
        return check_launch("lanczos");
    // pass 2: the same recurrence with the stored coefficients (the same
    // arithmetic, hence the same vectors) accumulating the Ritz vector
    // x = sum_j s_j v_j, then normalised
    double2 *x = gs_dev;
    double2 *v = buf[0], *u = buf[1], *w = buf[2];
    hipLaunchKernelGGL(k_vscale, dim3(g), dim3(kVecThreads), 0, s, v, start_dev,
                       inv0, n);
    hipLaunchKernelGGL(k_vscale, dim3(g), dim3(kVecThreads), 0, s, x, v, svec[0], n);
    double bprev = 0.0;
    for (size_t j = 0; j + 1 < alpha.size(); ++j) {
        double a = alpha[j], w2 = 0.0;
        if ((st = krylov_step(apply, v, u, w, bprev, true, &a, &w2, partial, n, s)) !=
            HUBBARD_OK)
            return st;
        hipLaunchKernelGGL(k_vscale, dim3(g), dim3(kVecThreads), 0, s, u, w, 1.0 / beta[j], n);
        std::swap(u, v);
        hipLaunchKernelGGL(k_vaxpy, dim3(g), dim3(kVecThreads), 0, s, x, v, svec[j + 1], n);
        bprev = beta[j];
    }
    double xn = 0.0;
    if ((st = host_dot(x, x, n, partial, s, &xn, &im)) != HUBBARD_OK)
        return st;
    hipLaunchKernelGGL(k_vscale, dim3(g), dim3(kVecThreads), 0, s, x, x, 1.0 / std::sqrt(xn), n);
    return check_launch("lanczos");
}

size_t lanczos_partial_bytes() { return vec_partial_bytes(); }

}  // namespace hv

extern "C" {

hubbard_status hubbard_vector_workspace_size(hubbard_t h, int32_t op, size_t *bytes)
{
    if (!h || !bytes ||
        (op != HUBBARD_OP_OVERLAP && op != HUBBARD_OP_LANCZOS && op != HUBBARD_OP_SPIN_CORR))
        return fail(HUBBARD_ERR_ARG, "bad arguments to hubbard_vector_workspace_size");
    if (op == HUBBARD_OP_SPIN_CORR) {
        const MomentLayout ml = moment_layout(h->m.nq);
        *bytes = ml.partial_bytes + align256((size_t)h->m.nq * h->m.nq * sizeof(double));
        return HUBBARD_OK;
    }
    const size_t vb = align256(vec_bytes(h));
    *bytes = (op == HUBBARD_OP_LANCZOS ? 3 * vb : 0) + vec_partial_bytes();
    return HUBBARD_OK;
}

hubbard_status hubbard_overlap(hubbard_t h, const void *a_dev, const void *b_dev, double *out_dev,
                               void *ws_dev, size_t ws_bytes, void *stream)
{
    if (!h || !a_dev || !b_dev || !out_dev || !ws_dev)
        return fail(HUBBARD_ERR_ARG, "NULL argument to hubbard_overlap");
    if (ws_bytes < vec_partial_bytes())
        return fail(HUBBARD_ERR_SIZE, "workspace too small for hubbard_overlap");
    const uint64_t n = (uint64_t)1 << h->m.nq;
    const unsigned g = vec_grid(n);
    hipStream_t s = (hipStream_t)stream;
    double2 *partial = (double2 *)ws_dev;
    hipLaunchKernelGGL(k_vdot, dim3(g), dim3(kVecThreads), 0, s, (const double2 *)a_dev,
                       (const double2 *)b_dev, n, partial);
    hipLaunchKernelGGL(k_vsum, dim3(1), dim3(kVecThreads), 0, s, partial, (int)g,
                       (double2 *)out_dev);
    return check_launch("overlap");
}

hubbard_status hubbard_lanczos(hubbard_t h, const void *start_dev, int32_t max_iter, double tol,
                               double *E0, int32_t *iters, double *residual, void *gs_dev,
                               void *ws_dev, size_t ws_bytes, void *stream)
{
    if (!h || !start_dev || max_iter < 1 || !(tol > 0.0) || !E0 || !ws_dev)
        return fail(HUBBARD_ERR_ARG, "bad arguments to hubbard_lanczos");
    size_t need = 0;
    hubbard_vector_workspace_size(h, HUBBARD_OP_LANCZOS, &need);
    if (ws_bytes < need)
        return fail(HUBBARD_ERR_SIZE, "workspace too small for hubbard_lanczos");
    const size_t vb = align256(vec_bytes(h));
    const char *ws = (const char *)ws_dev;
    for (const void *p : {start_dev, (const void *)gs_dev}) {
        const char *q = (const char *)p;
        if (q && q < ws + need && ws < q + vec_bytes(h))
            return fail(HUBBARD_ERR_ARG, "start or state vector overlaps the workspace");
    }
    Program *pr;
    DeviceState *ds;
    hubbard_status st = get_program(h, PROG_HAM, 0, &pr, &ds);
    if (st != HUBBARD_OK)
        return st;
    hipStream_t s = (hipStream_t)stream;
    double2 *buf[3] = {(double2 *)ws_dev, (double2 *)(ws + vb), (double2 *)(ws + 2 * vb)};
    const hv::ApplyH apply = [&](const double2 *in, double2 *out) {
        return run_ham(*pr, *ds, in, out, nullptr, s);
    };
    return hv::lanczos_run(apply, (uint64_t)1 << h->m.nq, (const double2 *)start_dev, max_iter,
                           tol, E0, iters, residual, (double2 *)gs_dev, buf,
                           (double2 *)(ws + 3 * vb), s);
}

hubbard_status hubbard_tridiag_lowest(const double *a, const double *b, int32_t m, double *lam,
                                      double *vec)
{
    if (!a || (m > 1 && !b) || m < 1 || !lam)
        return fail(HUBBARD_ERR_ARG, "bad arguments to hubbard_tridiag_lowest");
    *lam = tridiag_lowest(a, b, m, vec);
    return HUBBARD_OK;
}

}  // extern "C"

// ================================================================== VQE
// The optimisation loop of Sec. 2.1 on the host: L-BFGS (lbfgs.cpp) over
// energy_grad evaluations, one start per call or many starts advanced in
// lockstep with one energy_grad_batch launch per round.

namespace {

LbfgsOptions vqe_options(const hubbard_vqe_opts *o)
{
    LbfgsOptions r;
    if (o) {
        r.max_steps = o->max_steps;
        r.history = o->history;
        r.e_tol = o->e_tol;
        r.g_tol = o->g_tol;
    }
    return r;
}

size_t vqe_eval_bytes(hubbard_t h, int32_t n_layers, int32_t n_starts)
{
    const size_t P = (size_t)h->m.n_params(n_layers);
    return align256((size_t)n_starts * sizeof(double)) +
           align256((size_t)n_starts * P * sizeof(double));
}

hubbard_status vqe_engine_bytes(hubbard_t h, int32_t n_layers, int32_t n_starts, size_t *bytes)
{
    if (n_starts == 1)
        return hubbard_workspace_size(h, n_layers, HUBBARD_OP_ENERGY_GRAD, bytes);
    std::vector<hubbard_t> hs(n_starts, h);
    std::vector<int32_t> ls(n_starts, n_layers);
    return hubbard_batch_workspace_size(hs.data(), n_starts, ls.data(), bytes);
}

}  // namespace

extern "C" {

hubbard_status hubbard_vqe_workspace_size(hubbard_t h, int32_t n_layers, int32_t n_starts,
                                          size_t *bytes)
{
    if (!h || !bytes || n_layers < 1 || n_starts < 1)
        return fail(HUBBARD_ERR_ARG, "bad arguments to hubbard_vqe_workspace_size");
    size_t eng = 0;
    hubbard_status st = vqe_engine_bytes(h, n_layers, n_starts, &eng);
    if (st != HUBBARD_OK)
        return st;
    *bytes = align256(eng) + vqe_eval_bytes(h, n_layers, n_starts);
    return HUBBARD_OK;
}

hubbard_status hubbard_vqe(hubbard_t h, int32_t n_layers, int32_t n_starts, double *theta_dev,
                           const hubbard_vqe_opts *opts, hubbard_vqe_result *results,
                           void *ws_dev, size_t ws_bytes, void *stream)
{
    if (!h || n_layers < 1 || n_starts < 1 || !theta_dev || !results || !ws_dev)
        return fail(HUBBARD_ERR_ARG, "bad arguments to hubbard_vqe");
    if (opts && (opts->history < 1 || opts->max_steps < 0 || !(opts->e_tol >= 0.0) ||
                 !(opts->g_tol >= 0.0)))
        return fail(HUBBARD_ERR_ARG, "bad hubbard_vqe_opts");
    size_t eng = 0, need = 0;
    hubbard_status st = vqe_engine_bytes(h, n_layers, n_starts, &eng);
    if (st != HUBBARD_OK)
        return st;
    eng = align256(eng);
    need = eng + vqe_eval_bytes(h, n_layers, n_starts);
    if (ws_bytes < need)
        return fail(HUBBARD_ERR_SIZE, "workspace too small for hubbard_vqe");
    const int P = h->m.n_params(n_layers);
    hipStream_t s = (hipStream_t)stream;
    double *E_dev = (double *)((char *)ws_dev + eng);
    double *G_dev = (double *)((char *)E_dev + align256((size_t)n_starts * sizeof(double)));
    std::vector<double> th((size_t)n_starts * P), E(n_starts), G((size_t)n_starts * P);
    hipError_t e = hipMemcpyAsync(th.data(), theta_dev, th.size() * sizeof(double),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return fail(HUBBARD_ERR_DEVICE, std::string("vqe: reading theta: ") + hipGetErrorString(e));
    const LbfgsOptions lo = vqe_options(opts);
    std::vector<Lbfgs> opt;
    opt.reserve(n_starts);
    for (int i = 0; i < n_starts; ++i)
        opt.emplace_back(th.data() + (size_t)i * P, P, lo);
    std::vector<int64_t> toff(n_starts);
    std::vector<int32_t> lay(n_starts, n_layers);
    std::vector<hubbard_t> hs(n_starts, h);
    for (int i = 0; i < n_starts; ++i)
        toff[i] = (int64_t)i * P;
    for (;;) {
        bool active = false;
        for (int i = 0; i < n_starts; ++i) {
            // finished starts stay at their final iterate (evaluated with the
            // others: one launch sequence for all)
            const std::vector<double> &t = opt[i].trial_point();
            std::copy(t.begin(), t.end(), th.begin() + (size_t)i * P);
            active = active || opt[i].state() == LBFGS_EVALUATE;
        }
        if (!active)
            break;
        e = hipMemcpyAsync(theta_dev, th.data(), th.size() * sizeof(double),
                           hipMemcpyHostToDevice, s);
        if (e != hipSuccess)
            return fail(HUBBARD_ERR_DEVICE, std::string("vqe: theta: ") + hipGetErrorString(e));
        st = n_starts == 1
                 ? energy_grad(h, theta_dev, n_layers, E_dev, G_dev, ws_dev, eng, stream)
                 : energy_grad_batch(hs.data(), n_starts, theta_dev, toff.data(), lay.data(),
                                     E_dev, G_dev, ws_dev, eng, stream);
        if (st != HUBBARD_OK)
            return st;
        e = hipMemcpyAsync(E.data(), E_dev, E.size() * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(G.data(), G_dev, G.size() * sizeof(double),
                               hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            return fail(HUBBARD_ERR_DEVICE, std::string("vqe: evaluation: ") +
                                                hipGetErrorString(e));
        for (int i = 0; i < n_starts; ++i)
            if (opt[i].state() == LBFGS_EVALUATE)
                opt[i].tell(E[i], G.data() + (size_t)i * P);
    }
    for (int i = 0; i < n_starts; ++i) {
        const std::vector<double> &x = opt[i].iterate();
        std::copy(x.begin(), x.end(), th.begin() + (size_t)i * P);
        hubbard_vqe_result &r = results[i];
        std::memset(&r, 0, sizeof(r));
        r.E = opt[i].value();
        r.grad_norm = opt[i].grad_norm();
        r.steps = opt[i].n_steps();
        r.evals = opt[i].n_evals();
        r.reason = opt[i].state();
    }
    e = hipMemcpyAsync(theta_dev, th.data(), th.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return fail(HUBBARD_ERR_DEVICE, std::string("vqe: writing theta: ") + hipGetErrorString(e));
    return HUBBARD_OK;
}

struct hubbard_lbfgs {
    Lbfgs opt;
    hubbard_lbfgs(const double *x0, int n, const LbfgsOptions &o) : opt(x0, n, o) {}
};

hubbard_status hubbard_lbfgs_create(const double *x0, int32_t n, const hubbard_vqe_opts *opts,
                                    hubbard_lbfgs_t *out)
{
    if (!x0 || n < 1 || !out)
        return fail(HUBBARD_ERR_ARG, "bad arguments to hubbard_lbfgs_create");
    try {
        *out = new hubbard_lbfgs(x0, n, vqe_options(opts));
    } catch (...) {
        return fail(HUBBARD_ERR_NOMEM, "allocating the optimiser");
    }
    return HUBBARD_OK;
}

hubbard_status hubbard_lbfgs_tell(hubbard_lbfgs_t L, double f, const double *g, int32_t *state,
                                  double *x_next)
{
    if (!L || !g || !state || !x_next)
        return fail(HUBBARD_ERR_ARG, "bad arguments to hubbard_lbfgs_tell");
    *state = L->opt.tell(f, g);
    const std::vector<double> &t = L->opt.trial_point();
    std::copy(t.begin(), t.end(), x_next);
    return HUBBARD_OK;
}

hubbard_status hubbard_lbfgs_result(hubbard_lbfgs_t L, hubbard_vqe_result *res)
{
    if (!L || !res)
        return fail(HUBBARD_ERR_ARG, "bad arguments to hubbard_lbfgs_result");
    std::memset(res, 0, sizeof(*res));
    res->E = L->opt.value();
    res->grad_norm = L->opt.grad_norm();
    res->steps = L->opt.n_steps();
    res->evals = L->opt.n_evals();
    res->reason = L->opt.state();
    return HUBBARD_OK;
}

void hubbard_lbfgs_destroy(hubbard_lbfgs_t L) { delete L; }

}  // extern "C"

// ========================================================== observables
// The overlap loss of Eq. (5)/(6) with its adjoint gradient, and the spin
// correlations of Eq. (17).

extern "C" {

hubbard_status overlap_grad(hubbard_t h, const double *theta_dev, int32_t n_layers,
                            const void *ref_dev, double *out_dev, double *grad_dev, void *ws_dev,
                            size_t ws_bytes, void *stream)
{
    if (!h || !ref_dev || !out_dev || !ws_dev || n_layers < 0 ||
        (n_layers > 0 && (!theta_dev || !grad_dev)))
        return fail(HUBBARD_ERR_ARG, "bad arguments to overlap_grad");
    Program *pr;
    DeviceState *ds;
    hubbard_status st = get_program(h, PROG_GRAD, n_layers, &pr, &ds);
    if (st != HUBBARD_OK)
        return st;
    const size_t vb = align256(vec_bytes(h));
    const size_t need = 2 * vb + pr->partial_bytes + vec_partial_bytes() + 256;
    if (ws_bytes < need)
        return fail(HUBBARD_ERR_SIZE, "workspace too small for overlap_grad");
    const char *ws = (const char *)ws_dev, *rf = (const char *)ref_dev;
    if (rf < ws + need && ws < rf + vec_bytes(h))
        return fail(HUBBARD_ERR_ARG, "ref_dev overlaps the workspace");
    hipStream_t s = (hipStream_t)stream;
    double2 *psi = (double2 *)ws_dev;
    double2 *lam = (double2 *)((char *)ws_dev + vb);
    double *partial = (double *)((char *)ws_dev + 2 * vb);
    double2 *vpart = (double2 *)((char *)partial + pr->partial_bytes);
    double2 *c = (double2 *)((char *)vpart + vec_partial_bytes());
    double *spare = (double *)(c + 1);
    const uint64_t n = (uint64_t)1 << h->m.nq;
    const unsigned g = vec_grid(n);
    // psi(theta), plain layout
    const bool from_start = !pr->fwd.pass.empty();
    if (!from_start && (st = run_init(h, psi, s)) != HUBBARD_OK)
        return st;
    h->ev_used = 0;
    h->kmode.clear();
    if ((st = run_forward(*pr, *ds, theta_dev, psi, s, h, VecLayout(), from_start)) != HUBBARD_OK)
        return st;
    // c = <ref|psi>, lambda = c ref = P psi (P the projector on ref)
    hipLaunchKernelGGL(k_vdot, dim3(g), dim3(kVecThreads), 0, s, (const double2 *)ref_dev,
                       (const double2 *)psi, n, vpart);
    hipLaunchKernelGGL(k_vsum, dim3(1), dim3(kVecThreads), 0, s, vpart, (int)g, c);
    hipLaunchKernelGGL(k_vscale_dev, dim3(g), dim3(kVecThreads), 0, s, lam,
                       (const double2 *)ref_dev, (const double2 *)c, n);
    // the energy's reverse sweep with H replaced by P: dF/dtheta (the
    // reduction's energy output reads rows of H passes that did not run and
    // goes to a spare slot)
    launch_list<M_REV>(*pr, *ds, pr->rev, theta_dev, psi, lam, partial, s, h, VecLayout(), 0,
                       PF_NO_STORE);
    if ((st = check_launch("overlap reverse pass")) != HUBBARD_OK)
        return st;
    if ((st = run_reduce(*pr, partial, spare, grad_dev, s)) != HUBBARD_OK)
        return st;
    const int P = h->m.n_params(n_layers);
    hipLaunchKernelGGL(k_overlap_finish, dim3(1), dim3(kVecThreads), 0, s, (const double2 *)c,
                       grad_dev, P, out_dev);
    return check_launch("overlap_grad");
}

hubbard_status hubbard_spin_correlation(hubbard_t h, const void *psi_dev, double *C_dev,
                                        double *Sz_dev, void *ws_dev, size_t ws_bytes,
                                        void *stream)
{
    if (!h || !psi_dev || !C_dev || !Sz_dev || !ws_dev)
        return fail(HUBBARD_ERR_ARG, "NULL argument to hubbard_spin_correlation");
    size_t need = 0;
    hubbard_vector_workspace_size(h, HUBBARD_OP_SPIN_CORR, &need);
    if (ws_bytes < need)
        return fail(HUBBARD_ERR_SIZE, "workspace too small for hubbard_spin_correlation");
    const int n = h->m.nq;
    const MomentLayout ml = moment_layout(n);
    hipStream_t s = (hipStream_t)stream;
    double *partial = (double *)ws_dev;
    double *Q = (double *)((char *)ws_dev + ml.partial_bytes);
    const int W = 1 + kMomMid + kMomMid * (kMomMid - 1) / 2;
    const int smem = (1 << ml.lo) * W * (int)sizeof(double);
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
        (void)hipFuncSetAttribute((const void *)k_bit_moments,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  max_smem_per_block());
    });
    hipLaunchKernelGGL(k_bit_moments, dim3(ml.n_blk), dim3(1 << ml.lo), smem, s,
                       (const double2 *)psi_dev, ml.lo, ml.mid, partial);
    hipLaunchKernelGGL(k_moments_final, dim3(n * (n + 1) / 2), dim3(kVecThreads), 0, s, partial,
                       ml.n_blk, ml.r, n, Q);
    hipLaunchKernelGGL(k_spin_corr, dim3(1), dim3(kVecThreads), 0, s, Q, h->m.ns, C_dev, Sz_dev);
    return check_launch("spin correlation");
}

}  // extern "C"
