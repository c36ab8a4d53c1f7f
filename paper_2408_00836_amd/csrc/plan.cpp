// plan.cpp -- turns the circuit of Eq. (3)/(7) and the operator H into
// fused tile passes over the state vector.  Host only.
//
// A pass loads tiles of 2^k amplitudes whose index bits are a chosen set S of
// k qubits (always containing the c lowest bits, so every load is a run of
// 2^c contiguous amplitudes), applies a sequence of operations whose qubits
// all lie in S, and writes the tiles back.  Diagonal operations act
// element-wise and fit any tile.
//
// Ordering rule: two operations must keep their relative order iff they share
// a qubit and are not both diagonal.  Hopping terms on disjoint qubit pairs are
// fermion-parity-even bilinears on disjoint modes and commute; diagonal terms
// commute with each other.  The diagonal of a layer is split into one
// sub-term per site (U n_up n_dn + eps n) and one per V bond, so a spin-up
// gate only waits for the sub-terms on its own sites.
#include <stdexcept>
#include <algorithm>
#include <cstdint>
#include <functional>
#include <tuple>
#include <vector>

#include "hubvqe.hpp"

namespace hv {

namespace {

inline uint32_t qbit(int q) { return 1u << q; }

// Diagonal ops (OP_DIAG, OP_MASK) commute with each other and fit any tile.
inline bool diagonal(const HostOp &o) { return o.kind != OP_HOP; }

bool conflicts(const HostOp &a, const HostOp &b)
{
    if (diagonal(a) && diagonal(b))
        return false;
    return (a.qmask & b.qmask) != 0;
}

struct Closure {
    uint32_t S = 0;
    std::vector<int> inc;
    int hops = 0;
};

// Grow a tile set from `seed`, repeatedly taking the ready hop that adds the
// fewest new qubits, and return the ops that this tile can apply in order.
Closure grow(const std::vector<HostOp> &ops, const std::vector<int> &active,
             const std::vector<char> &done, uint32_t seed, int k)
{
    (void)done;
    Closure cl;
    cl.S = seed;
    if (__builtin_popcount(cl.S) > k)
        return cl;
    std::vector<char> in(ops.size(), 0);
    for (;;) {
        uint32_t bg = 0, bd = 0;   // qubits of blocked hops / blocked diagonals
        int best = -1, best_new = 99;
        for (int i : active) {
            if (in[i])
                continue;
            const HostOp &o = ops[i];
            if (diagonal(o)) {
                if (o.qmask & bg)
                    bd |= o.qmask;
                else
                    in[i] = 1;
                continue;
            }
            if ((o.qmask & bg) || (o.qmask & bd)) {
                bg |= o.qmask;
                continue;
            }
            uint32_t u = cl.S | o.qmask;
            int nw = __builtin_popcount(u) - __builtin_popcount(cl.S);
            if (__builtin_popcount(u) <= k && nw < best_new) {
                best_new = nw;
                best = i;
            }
            bg |= o.qmask;   // until included, later ops must wait for it
        }
        if (best < 0)
            break;
        in[best] = 1;
        cl.S |= ops[best].qmask;
    }
    // Final in-order check: an op is applied only if no earlier op it must
    // follow is left for a later pass.
    uint32_t bg = 0, bd = 0;
    for (int i : active) {
        const HostOp &o = ops[i];
        bool ok = in[i] && !(o.qmask & bg) && (diagonal(o) || !(o.qmask & bd));
        if (ok) {
            cl.inc.push_back(i);
            if (o.kind == OP_HOP)
                ++cl.hops;
        } else if (diagonal(o)) {
            bd |= o.qmask;
        } else {
            bg |= o.qmask;
        }
    }
    return cl;
}

// Fill a tile set up to k bits, lowest free bits first (longer contiguous run).
std::vector<int> finish_tile(uint32_t S, int n, int k)
{
    for (int b = 0; b < n && __builtin_popcount(S) < k; ++b)
        S |= qbit(b);
    std::vector<int> tile;
    for (int b = 0; b < n; ++b)
        if (S & qbit(b))
            tile.push_back(b);
    return tile;
}

// Merge diagonal sub-terms of the same parameter inside a pass when no
// conflicting op sits between them, so each tile multiplies once per run.
void merge_diagonals(std::vector<HostOp> &ops)
{
    std::vector<HostOp> out;
    for (const HostOp &o : ops) {
        if (o.kind == OP_DIAG) {
            int target = -1;
            for (int j = (int)out.size() - 1; j >= 0; --j) {
                if (out[j].kind == OP_DIAG && out[j].param == o.param) {
                    target = j;
                    break;
                }
                if (conflicts(out[j], o))
                    break;
            }
            if (target >= 0) {
                HostOp &d = out[target];
                // Moving o back to `target` is valid: everything between
                // commutes with it.  Everything between also commutes with the
                // merged op's other part, which was already there.
                d.qmask |= o.qmask;
                d.umask |= o.umask;
                d.emask |= o.emask;
                d.vbonds.insert(d.vbonds.end(), o.vbonds.begin(), o.vbonds.end());
                continue;
            }
        }
        out.push_back(o);
    }
    ops.swap(out);
}

}  // namespace

// The NP circuit of Eq. (8) (Sec. 2.2.1): R_z on every qubit, as the phase
// gate exp(i th n_q) (R_z up to a global phase), then per layer, for every
// on-site pair and then every bond of every hopping group (spin up, then
// spin down), U_NP(theta, phi) = exp(i theta K_pq) exp(i phi n_p n_q): a
// hopping rotation with t = 1 and a MASK phase with coefficient -1.
std::vector<HostOp> np_circuit_ops(const Model &m, int layers)
{
    std::vector<HostOp> ops;
    for (int q = 0; q < m.nq; ++q) {
        HostOp d;
        d.kind = OP_MASK;
        d.param = q;
        d.qmask = qbit(q);
        d.t = -1.0;
        ops.push_back(d);
    }
    int k = m.lead_params();
    auto term = [&](int a, int c) {
        HostOp h;
        h.kind = OP_HOP;
        h.param = k;
        h.p = std::min(a, c);
        h.q = std::max(a, c);
        h.qmask = qbit(a) | qbit(c);
        h.t = 1.0;
        ops.push_back(h);
        HostOp d;
        d.kind = OP_MASK;
        d.param = k + 1;
        d.qmask = qbit(a) | qbit(c);
        d.t = -1.0;
        ops.push_back(d);
        k += 2;
    };
    for (int l = 0; l < layers; ++l) {
        for (int i = 0; i < m.ns; ++i)
            term(m.qubit(i, 0), m.qubit(i, 1));
        for (int s = 1; s <= m.ngroups; ++s)
            for (int b = 0; b < m.nb; ++b)
                if (m.slot[b] == s)
                    for (int spin = 0; spin < 2; ++spin)
                        term(m.qubit(m.bi[b], spin), m.qubit(m.bj[b], spin));
    }
    return ops;
}

std::vector<HostOp> circuit_ops(const Model &m, int layers)
{
    if (m.ansatz == 1)
        return np_circuit_ops(m, layers);
    std::vector<HostOp> ops;
    const int per = m.params_per_layer();
    for (int l = 0; l < layers; ++l) {
        const int p0 = l * per;
        for (int i = 0; i < m.ns; ++i) {
            HostOp d;
            d.kind = OP_DIAG;
            d.param = p0;
            uint32_t both = qbit(m.qubit(i, 0)) | qbit(m.qubit(i, 1));
            d.qmask = both;
            if (m.U != 0.0)
                d.umask = qbit(m.qubit(i, 0));
            if (m.eps[i] != 0.0)
                d.emask = both;
            if (d.umask || d.emask)
                ops.push_back(d);
        }
        for (int b = 0; b < m.nb; ++b) {
            if (m.V[b] == 0.0)
                continue;
            HostOp d;
            d.kind = OP_DIAG;
            d.param = p0;
            d.qmask = qbit(m.qubit(m.bi[b], 0)) | qbit(m.qubit(m.bi[b], 1)) |
                      qbit(m.qubit(m.bj[b], 0)) | qbit(m.qubit(m.bj[b], 1));
            d.vbonds.push_back(b);
            ops.push_back(d);
        }
        for (int s = 1; s < per; ++s) {
            for (int b = 0; b < m.nb; ++b) {
                if (m.slot[b] != s)
                    continue;
                for (int spin = 0; spin < 2; ++spin) {
                    HostOp h;
                    h.kind = OP_HOP;
                    h.param = p0 + s;
                    int a = m.qubit(m.bi[b], spin), c = m.qubit(m.bj[b], spin);
                    h.p = std::min(a, c);
                    h.q = std::max(a, c);
                    h.qmask = qbit(a) | qbit(c);
                    h.t = m.t[b];
                    ops.push_back(h);
                }
            }
        }
    }
    return ops;
}

std::vector<HostPass> plan_forward(const Model &m, int layers, const TileConfig &tc)
{
    return plan_ops(circuit_ops(m, layers), m.nq, tc);
}

std::vector<HostPass> plan_ops(const std::vector<HostOp> &ops, int n, const TileConfig &tc)
{
    std::vector<HostPass> passes;
    if (ops.empty())
        return passes;
    const int k = std::min(tc.k, n);
    const int c = std::min(tc.c, k);
    if (n <= k) {
        HostPass p;
        p.tile = finish_tile(0, n, n);
        p.ops = ops;
        merge_diagonals(p.ops);
        plan_phases(p);
        passes.push_back(p);
        return passes;
    }
    uint32_t C = 0;
    for (int b = 0; b < c; ++b)
        C |= qbit(b);
    std::vector<char> done(ops.size(), 0);
    size_t first = 0;
    const size_t window = 480;
    // candidate passes from the current state: one closure per seed (no
    // seed, and the qubits of each ready hop), best first
    auto candidates = [&](const std::vector<char> &dn, size_t from, size_t max_seeds) {
        std::vector<int> active;
        for (size_t i = from; i < ops.size() && active.size() < window; ++i)
            if (!dn[i])
                active.push_back((int)i);
        std::vector<uint32_t> seeds{0u};
        uint32_t bg = 0, bd = 0;
        for (int i : active) {
            const HostOp &o = ops[i];
            if (diagonal(o)) {
                if (o.qmask & bg)
                    bd |= o.qmask;
                continue;
            }
            if (!((o.qmask & bg) || (o.qmask & bd)))
                seeds.push_back(o.qmask);
            bg |= o.qmask;
            if (seeds.size() > max_seeds)
                break;
        }
        std::vector<Closure> out;
        for (uint32_t sd : seeds) {
            Closure cl = grow(ops, active, dn, C | sd, k);
            if (!cl.inc.empty())
                out.push_back(std::move(cl));
        }
        std::stable_sort(out.begin(), out.end(), [](const Closure &a, const Closure &b) {
            return a.hops > b.hops || (a.hops == b.hops && a.inc.size() > b.inc.size());
        });
        return out;
    };
    while (first < ops.size()) {
        std::vector<Closure> cands = candidates(done, first, 48);
        // Lookahead: among the best few candidates keep the one that, with
        // the best follow-up passes (searched `depth` deep over the same
        // number of candidates), applies the most hops in total.
        std::function<int(const std::vector<char> &, size_t, int)> future =
            [&](const std::vector<char> &dn0, size_t from, int depth) -> int {
            size_t f = from;
            while (f < ops.size() && dn0[f])
                ++f;
            if (depth == 0 || f >= ops.size())
                return 0;
            std::vector<Closure> nc = candidates(dn0, f, 24);
            int bestv = 0;
            const size_t bw = std::min<size_t>(nc.size(), (size_t)tc.lookahead);
            for (size_t ci = 0; ci < bw; ++ci) {
                std::vector<char> dn = dn0;
                for (int i : nc[ci].inc)
                    dn[i] = 1;
                bestv = std::max(bestv, nc[ci].hops + future(dn, f, depth - 1));
            }
            return bestv;
        };
        if (cands.empty())
            throw std::runtime_error("no hopping term fits a tile of " + std::to_string(k) +
                                     " bits with " + std::to_string(c) + " fixed low bits");
        Closure best = cands.front();
        if (tc.lookahead > 0 && cands.size() > 1) {
            int best_score = -1;
            const size_t beam = std::min<size_t>(cands.size(), (size_t)tc.lookahead);
            for (size_t ci = 0; ci < beam; ++ci) {
                std::vector<char> dn = done;
                for (int i : cands[ci].inc)
                    dn[i] = 1;
                const int score = cands[ci].hops + future(dn, first, tc.depth);
                if (score > best_score) {
                    best_score = score;
                    best = cands[ci];
                }
            }
        }
        HostPass p;
        p.tile = finish_tile(best.S, n, k);
        for (int i : best.inc) {
            p.ops.push_back(ops[i]);
            done[i] = 1;
        }
        merge_diagonals(p.ops);
        plan_phases(p);
        passes.push_back(p);
        while (first < ops.size() && done[first])
            ++first;
    }
    return passes;
}

std::vector<HostPass> plan_hamiltonian(const Model &m, const TileConfig &tc)
{
    const int n = m.nq;
    const int k = std::min(tc.k, n);
    const int c = std::min(tc.c, k);
    HostOp diag;
    diag.kind = OP_DIAG;
    diag.param = -1;
    for (int i = 0; i < m.ns; ++i) {
        diag.umask |= qbit(m.qubit(i, 0));
        if (m.eps[i] != 0.0)
            diag.emask |= qbit(m.qubit(i, 0)) | qbit(m.qubit(i, 1));
    }
    diag.qmask = (n == 32) ? 0xffffffffu : ((1u << n) - 1u);
    for (int b = 0; b < m.nb; ++b)
        if (m.V[b] != 0.0)
            diag.vbonds.push_back(b);
    std::vector<HostOp> terms;
    for (int b = 0; b < m.nb; ++b)
        for (int spin = 0; spin < 2; ++spin) {
            HostOp h;
            h.kind = OP_HOP;
            int a = m.qubit(m.bi[b], spin), cq = m.qubit(m.bj[b], spin);
            h.p = std::min(a, cq);
            h.q = std::max(a, cq);
            h.qmask = qbit(a) | qbit(cq);
            h.t = m.t[b];
            terms.push_back(h);
        }
    std::vector<HostPass> passes;
    uint32_t C = 0;
    for (int b = 0; b < c; ++b)
        C |= qbit(b);
    std::vector<char> used(terms.size(), 0);
    size_t left = terms.size();
    bool first = true;
    while (left > 0 || first) {
        uint32_t bestS = C;
        int bestCount = -1;
        std::vector<uint32_t> seeds{0u};
        for (size_t i = 0; i < terms.size(); ++i)
            if (!used[i])
                seeds.push_back(terms[i].qmask);
        for (uint32_t sd : seeds) {
            uint32_t S = C | sd;
            if (__builtin_popcount(S) > k)
                continue;
            std::vector<char> take(terms.size(), 0);
            for (;;) {
                int bi = -1, bn = 99;
                for (size_t i = 0; i < terms.size(); ++i) {
                    if (used[i] || take[i])
                        continue;
                    uint32_t u = S | terms[i].qmask;
                    int nw = __builtin_popcount(u) - __builtin_popcount(S);
                    if (__builtin_popcount(u) <= k && nw < bn) {
                        bn = nw;
                        bi = (int)i;
                    }
                }
                if (bi < 0)
                    break;
                take[bi] = 1;
                S |= terms[bi].qmask;
            }
            int cnt = 0;
            for (size_t i = 0; i < terms.size(); ++i)
                cnt += (!used[i] && (terms[i].qmask & ~S) == 0);
            if (cnt > bestCount) {
                bestCount = cnt;
                bestS = S;
            }
        }
        HostPass p;
        p.tile = finish_tile(bestS, n, k);
        uint32_t Sf = 0;
        for (int b : p.tile)
            Sf |= qbit(b);
        if (first)
            p.ops.push_back(diag);
        for (size_t i = 0; i < terms.size(); ++i)
            if (!used[i] && (terms[i].qmask & ~Sf) == 0) {
                used[i] = 1;
                --left;
                p.ops.push_back(terms[i]);
            }
        if (!first && p.ops.empty())
            throw std::runtime_error("no Hamiltonian term fits a tile of " + std::to_string(k) +
                                     " bits with " + std::to_string(c) + " fixed low bits");
        p.flags = first ? PF_HAM_FIRST : 0;
        first = false;
        plan_phases(p);
        passes.push_back(p);
    }
    passes.back().flags |= PF_HAM_LAST;
    return passes;
}

void plan_phases(HostPass &p)
{
    const int k = (int)p.tile.size();
    const int rbits = std::min(k, kRegBits);
    int loc[kMaxQubits];
    for (int b = 0; b < kMaxQubits; ++b)
        loc[b] = -1;
    for (int j = 0; j < k; ++j)
        loc[p.tile[j]] = j;
    // the same ops with tile-local qubit masks (ordering only needs tile bits:
    // every hopping term of the pass lies in the tile)
    std::vector<HostOp> lops = p.ops;
    for (HostOp &o : lops) {
        uint32_t m = 0;
        for (int b = 0; b < kMaxQubits; ++b)
            if ((o.qmask >> b) & 1u)
                if (loc[b] >= 0)
                    m |= 1u << loc[b];
        o.qmask = m;
    }
    // low local bits that the load/store layout keeps on lanes 0..15
    uint32_t io_forbid = 0;
    for (int b = 0; b < std::min(4, k - kRegBits); ++b)
        io_forbid |= 1u << b;
    // Thread-id bits beyond the 6 lane bits index the waves of a workgroup.
    // A re-layout that keeps the wave bits fixed moves data only inside each
    // wave and needs no workgroup barrier, so the wave bits go on the tile
    // bits (other than the coalescing ones) that the fewest hopping terms
    // touch.
    const int wb = std::max(0, k - rbits - 6);
    std::vector<int> touch(k, 0);
    for (const HostOp &o : lops)
        if (o.kind == OP_HOP)
            for (int b = 0; b < k; ++b)
                touch[b] += (o.qmask >> b) & 1u;
    auto wave_rank = [&](int b) {
        // never on the coalescing bits: a wave's loads stay 256-byte runs
        int io = ((io_forbid >> b) & 1u) ? 1 : 0;
        return std::make_tuple(io, touch[b], -b);
    };
    auto pick_wave = [&](uint32_t excl) {
        std::vector<int> cand;
        for (int b = 0; b < k; ++b)
            if (!((excl >> b) & 1u))
                cand.push_back(b);
        std::sort(cand.begin(), cand.end(),
                  [&](int a, int b) { return wave_rank(a) < wave_rank(b); });
        std::vector<int> w(cand.begin(), cand.begin() + std::min<int>(wb, (int)cand.size()));
        std::sort(w.begin(), w.end());
        return w;
    };
    auto bits_of = [](const std::vector<int> &v) {
        uint32_t m = 0;
        for (int b : v)
            m |= 1u << b;
        return m;
    };
    const std::vector<int> W0 = pick_wave(0u);
    // register set of size rbits containing S and avoiding W (and, if it can,
    // the low bits the load/store layout needs on lanes)
    auto pad = [&](uint32_t S, uint32_t W) {
        std::vector<int> regs;
        for (int b = 0; b < k; ++b)
            if ((S >> b) & 1u)
                regs.push_back(b);
        for (int pass = 0; pass < 2; ++pass)
            for (int b = k - 1; b >= 0 && (int)regs.size() < rbits; --b) {
                const uint32_t bit = 1u << b;
                if ((S & bit) || (W & bit) || (pass == 0 && (io_forbid & bit)))
                    continue;
                regs.push_back(b);
                S |= bit;
            }
        std::sort(regs.begin(), regs.end());
        return regs;
    };
    auto layout_for = [&](uint32_t S) {
        HostPhase ph;
        ph.wave = (S & bits_of(W0)) ? pick_wave(S) : W0;
        ph.regs = pad(S, bits_of(ph.wave));
        return ph;
    };
    auto io_ok = [&](const HostPhase &ph) {
        for (int b : ph.regs)
            if ((io_forbid >> b) & 1u)
                return false;
        return true;
    };
    auto io_phase = [&](const std::vector<int> &wave, int at) {
        HostPhase io;
        io.wave = wave;
        io.regs = pad(0u, bits_of(wave));
        io.op_begin = io.op_end = at;
        return io;
    };

    std::vector<HostPhase> phases;
    std::vector<HostOp> ordered;
    std::vector<char> done(lops.size(), 0);
    size_t left = lops.size();
    while (left > 0) {
        std::vector<int> active;
        for (size_t i = 0; i < lops.size(); ++i)
            if (!done[i])
                active.push_back((int)i);
        std::vector<uint32_t> seeds{0u};
        {
            uint32_t bg = 0, bd = 0;
            for (int i : active) {
                const HostOp &o = lops[i];
                if (diagonal(o)) {
                    if (o.qmask & bg)
                        bd |= o.qmask;
                    continue;
                }
                if (!((o.qmask & bg) || (o.qmask & bd)))
                    seeds.push_back(o.qmask);
                bg |= o.qmask;
            }
        }
        Closure best;
        best.hops = -1;
        for (uint32_t sd : seeds) {
            Closure cl = grow(lops, active, done, sd, rbits);
            if (cl.inc.empty())
                continue;
            if (cl.hops > best.hops || (cl.hops == best.hops && cl.inc.size() > best.inc.size()))
                best = cl;
        }
        HostPhase ph = layout_for(best.S);
        ph.op_begin = (int)ordered.size();
        for (int i : best.inc) {
            ordered.push_back(p.ops[i]);
            done[i] = 1;
            --left;
        }
        ph.op_end = (int)ordered.size();
        // a phase with the previous one's layout extends it
        if (!phases.empty() && phases.back().regs == ph.regs && phases.back().wave == ph.wave)
            phases.back().op_end = ph.op_end;
        else
            phases.push_back(ph);
    }
    if (phases.empty() || !io_ok(phases.front()))
        phases.insert(phases.begin(), io_phase(phases.empty() ? W0 : phases.front().wave, 0));
    // the store layout must be load-compatible and keep the load layout's
    // wave bits, so that consecutive tiles never share LDS slots across waves
    if (!io_ok(phases.back()) || phases.back().wave != phases.front().wave)
        phases.push_back(io_phase(phases.front().wave, (int)ordered.size()));
    p.ops.swap(ordered);
    p.phases.swap(phases);
}

std::vector<HostPass> reversed_passes(std::vector<HostPass> ps)
{
    std::reverse(ps.begin(), ps.end());
    for (HostPass &p : ps) {
        const int n = (int)p.ops.size();
        std::reverse(p.ops.begin(), p.ops.end());
        std::reverse(p.phases.begin(), p.phases.end());
        for (HostPhase &ph : p.phases) {
            int b = n - ph.op_end, e = n - ph.op_begin;
            ph.op_begin = b;
            ph.op_end = e;
        }
    }
    return ps;
}

}  // namespace hv
