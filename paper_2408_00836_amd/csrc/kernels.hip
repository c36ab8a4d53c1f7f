// kernels.hip -- gfx950 kernels of the Hubbard state-vector engine.
//
// A pass streams the complex128 state vector (and, for the adjoint and H
// passes, a second vector) through registers in tiles of 2^k amplitudes.
// The tile's index bits are the pass's chosen qubits; the other n-k bits (the
// tile id) are spread over the grid with a grid-stride loop.  Tile bits
// 0..c-1 are the low bits of the amplitude index, and the load/store layout
// puts them on lanes 0..15, so every global access is a run of >= 256
// contiguous bytes.
//
// Inside a tile each thread holds 16 amplitudes in registers (four
// "register bits" of the tile index).  A pass is a sequence of phases; every
// hopping term of a phase acts on two of its register bits, so it runs
// entirely in registers.  Between phases the tile is re-laid out through one
// LDS exchange (XOR-swizzled slots against bank conflicts).
//
// Operations (see hubvqe.hpp):
//   OP_HOP   exp(-i th (-t)(a+_p a_q + h.c.)) on the pairs x <-> x^(2^p+2^q)
//            with exactly one of p, q occupied.  On such a pair the term is
//            s * [[0,1],[1,0]] with the Jordan-Wigner sign
//            s = (-1)^popcount(x & between(p,q)), so the gate is the rotation
//            (cos(th t), i s sin(th t)); no other amplitude changes.
//   OP_DIAG  exp(-i th D_sub) with D_sub = U * #{doubly occupied sites in the
//            op's set} + sum eps over its qubits + sum V_b n_i n_j over its bonds.
// No MFMA: nothing here is a dense contraction; the bound is HBM bandwidth.
#include <hip/hip_runtime.h>

#include "hubvqe.hpp"
#include "phase.hpp"

namespace hv {

enum Mode { M_FWD = 0, M_REV = 1, M_HAM = 2, M_EXP = 3 };

// Bit deposit: the low bits of x go, in order, to the set bits of mask.  x and
// mask are wave-uniform wherever this is called, so it runs on the scalar unit.
__device__ __forceinline__ uint32_t pdep32(uint32_t x, uint32_t mask)
{
    uint32_t r = 0;
    for (uint32_t m = mask; m; m &= m - 1u) {
        if (x & 1u)
            r |= m & (0u - m);
        x >>= 1;
    }
    return r;
}

// Diagonal sub-term value D_sub(g); GEN: the model has eps or V terms.
// etab: the op's eight nibble tables of its eps sum (LDS); vb: its V bond
// classes (see DevVBond).
template <bool GEN, typename OpT, typename MT, typename VbT>
__device__ __forceinline__ double diag_value(const OpT &op, uint32_t g, const MT *M,
                                             const VbT *vb, const double *etab)
{
    const uint32_t dn = (uint32_t)((uint64_t)g >> M->ns);
    double d = M->U * (double)__popc(g & dn & op.umask);
    if constexpr (GEN) {
#pragma unroll
        for (int k = 0; k < 8; ++k)
            d += etab[k * 16 + ((g >> (4 * k)) & 15u)];
        const uint32_t smask = (1u << M->ns) - 1u;
        const uint32_t U = g & smask, D = dn & smask;
        for (int v = op.v_begin; v < op.v_end; ++v) {
            const uint32_t src = vb[v].src;
            const int32_t delta = vb[v].delta;
            const uint32_t Us = delta >= 0 ? U >> delta : U << -delta;
            const uint32_t Ds = delta >= 0 ? D >> delta : D << -delta;
            const int cnt = __popc(U & Us & src) + __popc(U & Ds & src) + __popc(D & Us & src) +
                            __popc(D & Ds & src);
            d += vb[v].V * (double)cnt;
        }
    }
    return d;
}

// The general diagonal sub-term D_sub at the 16 registers of a thread:
// g_j = gt | goff(j).  The eps sum is additive over disjoint bits, so the
// thread's part is looked up once and each register bit's part once; the V
// classes are the outer loop, so that no loop runs inside the unrolled
// register loop.
template <typename Layout, typename OpT, typename MT, typename VbT>
__device__ __forceinline__ void diag_values(const OpT &op, uint32_t gt, const Layout &L,
                                            const MT *M, const VbT *vb, const double *etab,
                                            double (&dv)[kRegs])
{
    const uint32_t ns = M->ns;
    double et = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        et += etab[k * 16 + ((gt >> (4 * k)) & 15u)];
    double er[kRegBits];
#pragma unroll
    for (int i = 0; i < kRegBits; ++i) {
        const uint32_t b = L.gb[i];   // one global bit, or 0 (phantom register bit)
        const int p = b ? __builtin_ctz(b) : 0;
        er[i] = b ? etab[(p >> 2) * 16 + (1u << (p & 3))] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kRegs; ++j) {
        double e = et;
#pragma unroll
        for (int i = 0; i < kRegBits; ++i)
            if ((j >> i) & 1)
                e += er[i];
        const uint32_t g = gt | L.goff(j);
        dv[j] = M->U * (double)__popc(g & (g >> ns) & op.umask) + e;
    }
    const uint32_t smask = (1u << ns) - 1u;
    for (int c = op.v_begin; c < op.v_end; ++c) {
        const uint32_t src = vb[c].src;
        const int32_t delta = vb[c].delta;
        const double V = vb[c].V;
#pragma unroll
        for (int j = 0; j < kRegs; ++j) {
            const uint32_t g = gt | L.goff(j);
            const uint32_t U = g & smask, D = (g >> ns) & smask;
            const uint32_t Us = delta >= 0 ? U >> delta : U << -delta;
            const uint32_t Ds = delta >= 0 ? D >> delta : D << -delta;
            const int cnt = __popc(U & Us & src) + __popc(U & Ds & src) + __popc(D & Us & src) +
                            __popc(D & Ds & src);
            dv[j] += V * (double)cnt;
        }
    }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double im_conj_mul(double2 a, double2 b)
{
    return a.x * b.y - a.y * b.x;   // Im(conj(a) b)
}

__device__ __forceinline__ double re_conj_mul(double2 a, double2 b)
{
    return a.x * b.x + a.y * b.y;   // Re(conj(a) b)
}

// (x, y) <- (c x + i s y, i s x + c y)
__device__ __forceinline__ void rotate(double2 &x, double2 &y, double c, double s)
{
    double2 a = x, b = y;
    x = make_double2(c * a.x - s * b.y, c * a.y + s * b.x);
    y = make_double2(c * b.x - s * a.y, c * b.y + s * a.x);
}

// Per-op context of a hopping term applied in registers.  The Jordan-Wigner
// sign of a pair is (-1)^(par_thread + par_reg): the thread/tile part is
// folded into sn and t once per op; the register part is a wave-uniform bit
// of the op's flip mask (precomputed from the phase layout), applied by one
// XOR of the sign bit -- no loads and no branches per pair.
template <int NT>
struct PairCtx {
    double cs;             // cos of the rotation
    double sn[NT];         // sin, times the thread part of the sign, per tile
    double t[NT];          // (-t_b) times the thread part of the sign, per tile
    uint32_t flip;         // bit j: register j's part of the sign is odd
    double acc[NT];        // reduction of the op (register part of the sign applied)
};

// One register pair (J, JJ) of a hopping term.  Register sets: forward and
// expectation passes hold NT tiles of one vector (set t = tile t); reverse
// and H passes hold one tile of two vectors (set 0 = psi, set 1 = lambda or
// phi).
template <int MODE, int NT, int NS, int J, int JJ>
__device__ __forceinline__ void pair_op(double2 (&v)[NS][kRegs], PairCtx<NT> &x)
{
    const uint32_t fb = (x.flip >> J) & 1u;   // wave-uniform
    if constexpr (MODE == 0) {            // forward gate
#pragma unroll
        for (int t = 0; t < NT; ++t)
            rotate(v[t][J], v[t][JJ], x.cs, flip_sign(x.sn[t], fb));
    } else if constexpr (MODE == 1) {     // reverse: reduce, then un-apply
        const double w = im_conj_mul(v[1][J], v[0][JJ]) + im_conj_mul(v[1][JJ], v[0][J]);
        x.acc[0] += flip_sign(w, fb);
        const double ss = flip_sign(x.sn[0], fb);
        rotate(v[0][J], v[0][JJ], x.cs, ss);
        rotate(v[1][J], v[1][JJ], x.cs, ss);
    } else if constexpr (MODE == 2) {     // phi += (-t) s (swap) psi
        const double w = flip_sign(x.t[0], fb);
        v[1][J].x += w * v[0][JJ].x;
        v[1][J].y += w * v[0][JJ].y;
        v[1][JJ].x += w * v[0][J].x;
        v[1][JJ].y += w * v[0][J].y;
    } else {                              // expectation
#pragma unroll
        for (int t = 0; t < NT; ++t)
            x.acc[t] += flip_sign(re_conj_mul(v[t][J], v[t][JJ]), fb);
    }
}

template <int MODE, int NT, int NS, int A, int B, int X>
__device__ __forceinline__ void pair_at(double2 (&v)[NS][kRegs], PairCtx<NT> &x)
{
    constexpr int C = (A != 0 && B != 0) ? 0 : ((A != 1 && B != 1) ? 1 : 2);
    constexpr int D = 6 - A - B - C;   // the fourth register bit
    constexpr int J = (1 << A) | ((X & 1) << C) | (((X >> 1) & 1) << D);
    pair_op<MODE, NT, NS, J, J ^ ((1 << A) | (1 << B))>(v, x);
}

template <int MODE, int NT, int NS, int A, int B>
__device__ __forceinline__ void pairs4(double2 (&v)[NS][kRegs], PairCtx<NT> &x)
{
    pair_at<MODE, NT, NS, A, B, 0>(v, x);
    pair_at<MODE, NT, NS, A, B, 1>(v, x);
    pair_at<MODE, NT, NS, A, B, 2>(v, x);
    pair_at<MODE, NT, NS, A, B, 3>(v, x);
}

template <int MODE, int NT, int NS>
__device__ __forceinline__ void hop_regs(int pair, double2 (&v)[NS][kRegs], PairCtx<NT> &x)
{
    switch (pair) {
    case 0: pairs4<MODE, NT, NS, 0, 1>(v, x); break;
    case 1: pairs4<MODE, NT, NS, 0, 2>(v, x); break;
    case 2: pairs4<MODE, NT, NS, 0, 3>(v, x); break;
    case 3: pairs4<MODE, NT, NS, 1, 2>(v, x); break;
    case 4: pairs4<MODE, NT, NS, 1, 3>(v, x); break;
    default: pairs4<MODE, NT, NS, 2, 3>(v, x); break;
    }
}

// Register part of a phase's layout, held in scalar registers: goff(j) is
// register j's global-index bits, roff(j) its LDS byte offset relative to
// the thread's slot.  Both are linear in the bits of j (see DevPhase).
struct RegLayout {
    uint32_t gb[kRegBits], sb[kRegBits];
    __device__ __forceinline__ uint32_t goff(int j) const
    {
        uint32_t r = 0;
#pragma unroll
        for (int i = 0; i < kRegBits; ++i)
            if ((j >> i) & 1)
                r |= gb[i];
        return r;
    }
    __device__ __forceinline__ uint32_t roff(int j) const
    {
        uint32_t r = 0;
#pragma unroll
        for (int i = 0; i < kRegBits; ++i)
            if ((j >> i) & 1)
                r ^= sb[i];
        return r;
    }
};

template <typename PhT>
__device__ __forceinline__ RegLayout reg_layout(const PhT &ph)
{
    RegLayout r;
#pragma unroll
    for (int i = 0; i < kRegBits; ++i) {
        r.gb[i] = ph.gb[i];
        r.sb[i] = ph.sb[i];
    }
    return r;
}

// Re-lay the tile out from one phase's register layout to the next through
// LDS: every register goes to the slot of its tile-local index and comes
// back from the slot of its new one.  xf/xt are the thread's slot byte
// offsets in the old and new layouts.
// If the wave bits stay fixed (cross == false) every wave reads back exactly
// the slots it wrote, in program order, so no workgroup barrier is needed;
// every LDS slot a wave touches between cross-wave exchanges is its own.
template <int NS, bool FULL>
__device__ __forceinline__ void relayout(double2 (&v)[NS][kRegs], char *xbuf, uint32_t xf,
                                         const RegLayout &from, uint32_t xt, const RegLayout &to,
                                         bool cross, uint32_t valid)
{
#pragma unroll
    for (int w = 0; w < NS; ++w) {
        if (cross && w > 0)
            __syncthreads();   // the previous set's reads are done everywhere
#pragma unroll
        for (int j = 0; j < kRegs; ++j)
            if (FULL || ((valid >> j) & 1u))
                *(double2 *)(xbuf + (xf ^ from.roff(j))) = v[w][j];
        if (cross)
            __syncthreads();
        else
            __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int j = 0; j < kRegs; ++j)
            if (FULL || ((valid >> j) & 1u))
                v[w][j] = *(const double2 *)(xbuf + (xt ^ to.roff(j)));
        __builtin_amdgcn_wave_barrier();
    }
}

// Sum of x over each aligned group of four lanes (the same value in every
// lane of the group), by DPP quad permutations of the two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double y)
{
    const long long b = __double_as_longlong(y);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double quad_sum(double x)
{
    x += dpp_f64<0xB1>(x);   // quad_perm [1,0,3,2]: lane ^ 1
    x += dpp_f64<0x4E>(x);   // quad_perm [2,3,0,1]: lane ^ 2
    return x;
}

// Where a workgroup's reduction rows go: row r of the pass at
// base[r * stride] (a column of the partial array that a second-stage
// reduction sums in a fixed order).
struct Sink {
    double *base;     // row 0 of this workgroup's partial column
    int64_t stride;   // distance between rows
};

// Sum of x over the workgroup, valid in thread 0 (fixed shuffle tree, then
// the waves in order).  All threads must call it.
__device__ __forceinline__ double block_sum(double x, double *wsum)
{
    const int T = blockDim.x, tid = threadIdx.x;
    for (int off = (T < 64 ? T : 64) >> 1; off > 0; off >>= 1)
        x += __shfl_xor(x, off);
    if ((tid & 63) == 0)
        wsum[tid >> 6] = x;
    __syncthreads();
    double tot = 0.0;
    if (tid == 0)
        for (int w = 0; w < (T + 63) / 64; ++w)
            tot += wsum[w];
    __syncthreads();
    return tot;
}

// A value the optimiser must treat as freshly computed here (an empty asm
// that claims to modify it), so that work derived from it stays where it is
// written instead of being hoisted into long-lived registers.
__device__ __forceinline__ uint32_t opaque(uint32_t x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Global-index bits of a tile-local index x: tile bits 0..c-1 are global bits
// 0..c-1, the others are deposited over hi_mask (the tile's bits, ascending).
__device__ __forceinline__ uint32_t tile_global(uint32_t x, int c, uint32_t hi_mask)
{
    const uint32_t cmask = (1u << c) - 1u;
    return pdep32(x >> c, hi_mask) | (x & cmask);
}

// Tile id -> its global bits, advanced by a fixed step: adding the deposited
// step with every non-free bit set carries straight through those bits.
__device__ __forceinline__ uint32_t tile_advance(uint32_t base, uint32_t step_dep,
                                                 uint32_t free_mask)
{
    return (uint32_t)((((uint64_t)(base | ~free_mask)) + step_dep) & free_mask);
}

// Element offset of amplitude g of a vector stored in blocks of 2^ilv
// amplitudes with a gap of one block after each (ilv = 32: plain contiguous
// storage); a second vector may fill the gaps.  Inserting a zero bit is
// linear: the offset of a | b (disjoint bits) is the OR of their offsets, so
// a thread's part is mapped once per tile and a register's part, uniform
// over the wave, on the scalar unit.
__device__ __forceinline__ uint64_t vec_offset(uint64_t g, uint32_t ilv)
{
    return g + ((g >> ilv) << ilv);
}

// One pass over the tiles [tile0, tile_end) with stride tstep.  FULL: all
// threads own amplitudes and all 16 registers hold one (tiles of >= 16
// amplitudes launched with exactly 2^tbits threads): no per-register guards.
// NT = 2 (forward passes only): every iteration takes the tiles tl and
// tl + tstep, which needs tile_end - tile0 to be a multiple of 2 tstep; the
// op stream is then decoded once for two tiles.
// Vector element access through a possibly address-space-qualified type
// (member by member: the vector type's own copy operations take generic
// references only).
template <typename Vec>
__device__ __forceinline__ double2 vload(const Vec *p)
{
    return make_double2(p->x, p->y);
}
template <typename Vec>
__device__ __forceinline__ void vstore(Vec *p, double2 v)
{
    p->x = v.x;
    p->y = v.y;
}

// Vec and the table types: address-space qualified where the caller knows
// more than the pointer types say (see k_batch_pass).
// OPS: which op kinds the op loop decodes (OPS_HVA: hopping terms and
// diagonal sub-terms; OPS_NP: hopping terms and mask phases; OPS_ALL: all
// three).  A kind a kernel does not decode costs it no registers.
template <int MODE, bool GEN, bool FULL, int NT, bool START = false, int OPS = OPS_HVA,
          typename Vec = double2,
          typename PhT = DevPhase, typename OpT = DevOp, typename VbT = DevVBond,
          typename ThT = double, typename MT = DevModel>
__device__ __forceinline__ void run_pass(const DevPass &P, const PhT *__restrict__ phases,
                                         const OpT *__restrict__ ops,
                                         const VbT *__restrict__ vb,
                                         const ThT *__restrict__ theta,
                                         const MT *__restrict__ M, Vec *__restrict__ v0,
                                         Vec *__restrict__ v1, char *smem, uint64_t tile0,
                                         uint64_t tstep, uint64_t tile_end, uint32_t ilv,
                                         const Sink &sink)
{
    constexpr int NV = (MODE == M_FWD || MODE == M_EXP) ? 1 : 2;   // vectors per tile
    constexpr int NS = NT * NV;                                     // register sets
    static_assert(NS <= 2 && (NT == 1 || NV == 1), "at most two register sets");
    const int T = blockDim.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // a batch workgroup may be wider than this pass's 2^tbits threads: the
    // extra threads keep zero registers and only join the barriers
    const bool act = FULL || tid < (1 << P.tbits);
    const bool ham_first = (MODE == M_HAM) && (P.flags & PF_HAM_FIRST);
    const bool ham_last = (MODE == M_HAM) && (P.flags & PF_HAM_LAST);
    const int n_red = (MODE == M_EXP) ? 1 : P.n_red;
    const bool single = (P.nfree == 0);
    const SmemPlan sp = smem_plan(P.k, P.n_ops, P.n_diag, n_red, P.n_phases, T, single, GEN);
    char *xbuf = smem + sp.xbuf;
    uint2 *ltab = (uint2 *)(smem + sp.ltab);
    uint2 *wtab = (uint2 *)(smem + sp.wtab);
    double2 *opc = (double2 *)(smem + sp.opc);
    double2 *dtab = (double2 *)(smem + sp.dtab);
    double *etab = (double *)(smem + sp.etab);
    double2 *cis = (double2 *)(smem + sp.cis);
    double *red = (double *)(smem + sp.red);
    const int R = (int)sp.rows;            // accumulators per reduction row
    const bool quad = !single && T >= 4;   // rows hold sums over four lanes

    const PhT *ph = phases + P.phase_begin;
    // ---- per-workgroup set-up: lane and wave parts of every phase's
    // tile-local index, as global bits and as LDS slot byte offsets
    const double sign = (MODE == M_REV) ? -1.0 : 1.0;
    {
        for (int i = tid; i < P.n_phases * 64; i += T) {
            const uint32_t lp = pdep32((uint32_t)(i & 63), ph[i >> 6].lmask);
            ltab[i] = make_uint2(tile_global(lp, P.c, P.hi_mask), slot(lp, P.swz[0], P.swz[1]) << 4);
        }
        for (int i = tid; i < P.n_phases * kMaxWaves; i += T) {
            const uint32_t wp = pdep32((uint32_t)(i % kMaxWaves), ph[i / kMaxWaves].wmask);
            wtab[i] = make_uint2(tile_global(wp, P.c, P.hi_mask), slot(wp, P.swz[0], P.swz[1]) << 4);
        }
        if constexpr (MODE == M_FWD || MODE == M_REV) {
            for (int o = tid; o < P.n_ops; o += T) {
                const OpT &op = ops[P.op_begin + o];
                if (op.kind == OP_HOP) {
                    double s, c;
                    sincos(theta[op.param] * op.t, &s, &c);
                    opc[o] = make_double2(c, sign * s);
                } else if (OPS != OPS_HVA && op.kind == OP_MASK) {
                    // exp(-i sign th coef) on the amplitudes with every mask bit set
                    double s, c;
                    sincos(theta[op.param] * op.t, &s, &c);
                    opc[o] = make_double2(c, -sign * s);
                }
            }
            if constexpr (!GEN) {
                for (int o = 0; o < P.n_ops; ++o) {
                    const OpT &op = ops[P.op_begin + o];
                    if (op.kind != OP_DIAG)
                        continue;
                    for (int m = tid; m < kDiagTab; m += T) {
                        double s, c;
                        sincos(theta[op.param] * (M->U * (double)m), &s, &c);
                        dtab[op.dtab * kDiagTab + m] = make_double2(c, -sign * s);
                    }
                }
            } else if (P.n_diag > 0) {
                build_cis(cis, tid, T);
            }
        }
        if constexpr (GEN) {
            // eps sum of each diag op over its qubits, per index nibble
            for (int o = 0; o < P.n_ops; ++o) {
                const OpT &op = ops[P.op_begin + o];
                if (op.kind != OP_DIAG)
                    continue;
                for (int t = tid; t < 128; t += T) {
                    const int k = t >> 4;
                    const uint32_t v = (uint32_t)(t & 15) & ((op.emask >> (4 * k)) & 15u);
                    double e = 0.0;
                    for (int j = 0; j < 4; ++j)
                        if ((v >> j) & 1u)
                            e += M->eps_q[4 * k + j];
                    etab[op.dtab * 128 + t] = e;
                }
            }
        }
        for (int r = tid; r < n_red * R; r += T)
            red[r] = 0.0;
    }
    __syncthreads();
    double *wsum = red + n_red * R;

    const uint64_t ntiles = tile_end;
    const uint32_t valid = FULL ? 0xFFFFu : ph[0].valid;
    const uint32_t step_dep = pdep32((uint32_t)tstep, P.free_mask);
    double eacc = 0.0;
    double2 v[NS][kRegs];

    // the thread's part of phase q's layout: global bits and slot offset
    auto thread_part = [&](int q) __attribute__((always_inline)) {
        const uint2 a = ltab[q * 64 + lane], b = wtab[q * kMaxWaves + wave];
        return make_uint2(a.x | b.x, a.y ^ b.y);
    };
    const uint2 tp0 = thread_part(0);
    const RegLayout L0 = reg_layout(ph[0]);
    // START (forward only): the input is |b0>; nothing is read
    constexpr bool from_start = (MODE == M_FWD) && START;
    const bool no_store = (MODE == M_REV) && (P.flags & PF_NO_STORE);
    const uint32_t b0 = M->b0;

    // Registers of a tile smaller than 16 amplitudes that hold nothing are
    // zero, so they add nothing to any reduction.
    auto load_tiles = [&](double2 (&dst)[NS][kRegs], const uint32_t (&bs)[NT])
                          __attribute__((always_inline)) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if constexpr (from_start) {   // |b0>: one amplitude 1, the others 0
                const uint32_t gt = bs[t] | tp0.x;
#pragma unroll
                for (int j = 0; j < kRegs; ++j)
                    dst[t][j] = make_double2(
                        (FULL || (act && ((valid >> j) & 1u))) && (gt | L0.goff(j)) == b0 ? 1.0
                                                                                           : 0.0,
                        0.0);
                continue;
            }
            const uint64_t ga = vec_offset(bs[t] | tp0.x, ilv);
#pragma unroll
            for (int j = 0; j < kRegs; ++j) {
                if constexpr (!FULL) {
                    dst[t * NV][j] = make_double2(0.0, 0.0);
                    if constexpr (NV == 2)
                        dst[1][j] = make_double2(0.0, 0.0);
                }
                if (FULL || (act && ((valid >> j) & 1u))) {
                    const uint64_t g = ga | vec_offset(L0.goff(j), ilv);
                    dst[t * NV][j] = vload(v0 + g);
                    if constexpr (NV == 2) {
                        if (!ham_first)
                            dst[1][j] = vload(v1 + g);
                        else if constexpr (FULL)
                            dst[1][j] = make_double2(0.0, 0.0);
                    }
                }
            }
        }
    };
    // One-vector, one-tile passes prefetch the next tile into a second
    // register set while the current one is computed.
    constexpr bool PREFETCH = (NS == 1);
    double2 nxt[NS][kRegs];
    uint32_t bases[NT];
    bases[0] = pdep32((uint32_t)tile0, P.free_mask);
#pragma unroll
    for (int t = 1; t < NT; ++t)
        bases[t] = tile_advance(bases[t - 1], step_dep, P.free_mask);
    if (PREFETCH && tile0 < ntiles)
        load_tiles(nxt, bases);

    for (uint64_t tl = tile0; tl < ntiles; tl += NT * tstep) {
        uint32_t nbases[NT];
        nbases[0] = tile_advance(bases[NT - 1], step_dep, P.free_mask);
#pragma unroll
        for (int t = 1; t < NT; ++t)
            nbases[t] = tile_advance(nbases[t - 1], step_dep, P.free_mask);
        if constexpr (PREFETCH) {
#pragma unroll
            for (int j = 0; j < kRegs; ++j)
                v[0][j] = nxt[0][j];
            if (tl + tstep < ntiles)
                load_tiles(nxt, nbases);
        } else {
            load_tiles(v, bases);
        }
        uint2 tp = tp0;
        RegLayout L = L0;
        uint32_t gthr[NT];   // the thread's global bits in each tile
#pragma unroll
        for (int t = 0; t < NT; ++t)
            gthr[t] = bases[t] | tp.x;
        for (int q = 0; q < P.n_phases; ++q) {
            const PhT &phq = ph[q];
            if (q > 0) {
                const uint2 tn = thread_part(q);
                const RegLayout Ln = reg_layout(phq);
                relayout<NS, FULL>(v, xbuf, tp.y, L, tn.y, Ln, phq.cross != 0,
                                   act ? valid : 0u);
                tp = tn;
                L = Ln;
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    gthr[t] = bases[t] | tp.x;
            }
            for (int o = phq.op_begin; o < phq.op_end; ++o) {
                const OpT &op = ops[P.op_begin + o];
                double racc = 0.0;   // this op's reduction (thread part)
                if (OPS != OPS_NP && op.kind == OP_DIAG) {
                    double th_op = 0.0;
                    if constexpr (GEN && (MODE == M_FWD || MODE == M_REV))
                        th_op = theta[op.param];
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        // recomputed per op: hoisted out of the op loop, the
                        // 16 indices would only occupy (or spill) registers
                        const uint32_t gt = opaque(gthr[t]);
                        // general diagonal: D_sub at each register, computed
                        // together (the expectation passes keep the per-register
                        // form, which needs fewer registers there)
                        constexpr bool DV = GEN && MODE != M_EXP;
                        double dv[kRegs];
                        if constexpr (DV)
                            diag_values(op, gt, L, M, vb, etab + op.dtab * 128, dv);
#pragma unroll
                        for (int j = 0; j < kRegs; ++j) {
                            if (!FULL && !((valid >> j) & 1u))
                                continue;
                            const uint32_t g = gt | L.goff(j);
                            double2 &a = v[t * NV][j];
                            if constexpr (MODE == M_FWD || MODE == M_REV) {
                                double2 phs;
                                double d = 0.0;
                                if constexpr (!GEN) {
                                    const uint32_t dbl = g & (g >> M->ns) & op.umask;
                                    phs = dtab[op.dtab * kDiagTab + __popc(dbl)];
                                    if constexpr (MODE == M_REV)
                                        d = M->U * (double)__popc(dbl);
                                } else {
                                    d = dv[j];
                                    phs = cis_neg(sign * th_op * d, cis);
                                }
                                if constexpr (MODE == M_REV) {
                                    racc += d * im_conj_mul(v[1][j], a);
                                    v[1][j] = cmul(v[1][j], phs);
                                }
                                a = cmul(a, phs);
                            } else if constexpr (MODE == M_HAM) {
                                const double d =
                                    GEN ? dv[j] : diag_value<GEN>(op, g, M, vb, etab + op.dtab * 128);
                                v[1][j].x += d * a.x;
                                v[1][j].y += d * a.y;
                            } else {
                                eacc += diag_value<GEN>(op, g, M, vb, etab + op.dtab * 128) *
                                        (a.x * a.x + a.y * a.y);
                            }
                        }
                    }
                } else if (OPS != OPS_HVA && op.kind == OP_MASK) {
                    // coef * [every bit of the mask set]: the phase (fwd/rev)
                    // on those registers, and in the reverse the bracket
                    // coef * sum Im(conj(lambda) psi) over them
                    if constexpr (MODE == M_FWD || MODE == M_REV) {
                        const double2 ph = opc[o];
                        const uint32_t mask = op.between;
                        // the mask's bits among the phase's register bits
                        // select registers (uniform), the rest select threads
                        uint32_t mreg = 0, rbits = 0;
#pragma unroll
                        for (int i = 0; i < kRegBits; ++i) {
                            rbits |= L.gb[i];
                            if (L.gb[i] & mask)
                                mreg |= 1u << i;
                        }
                        const uint32_t mthr = mask & ~rbits;
#pragma unroll
                        for (int t = 0; t < NT; ++t) {
                            if ((gthr[t] & mthr) != mthr)
                                continue;
#pragma unroll
                            for (int j = 0; j < kRegs; ++j) {
                                if (((uint32_t)j & mreg) != mreg)
                                    continue;
                                if (!FULL && !((valid >> j) & 1u))
                                    continue;
                                double2 &a = v[t * NV][j];
                                if constexpr (MODE == M_REV) {
                                    racc += op.t * im_conj_mul(v[1][j], a);
                                    v[1][j] = cmul(v[1][j], ph);
                                }
                                a = cmul(a, ph);
                            }
                        }
                    }
                } else {
                    PairCtx<NT> x;
                    x.flip = op.flip;
                    double cs = 0.0, sn = 0.0;
                    if constexpr (MODE == M_FWD || MODE == M_REV) {
                        const double2 c2 = opc[o];
                        cs = c2.x;
                        sn = c2.y;
                    }
                    x.cs = cs;
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        // thread and tile part of the Jordan-Wigner sign
                        const bool podd = (__popc(gthr[t] & op.between) & 1u) != 0;
                        x.t[t] = podd ? op.t : -op.t;   // (-t) times that part of the sign
                        x.sn[t] = podd ? -sn : sn;
                        x.acc[t] = 0.0;
                    }
                    hop_regs<MODE, NT, NS>(op.pair, v, x);
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        racc += x.t[t] * x.acc[t];   // (-t) s summed
                    if constexpr (MODE == M_EXP)
                        eacc += 2.0 * racc;
                }
                if constexpr (MODE == M_REV) {
                    if (single) {
                        const double tot = block_sum(racc, wsum);
                        if (tid == 0)
                            red[op.red] += tot;
                    } else if (quad) {
                        const double qs = quad_sum(racc);
                        if ((tid & 3) == 0)
                            red[op.red * R + (tid >> 2)] += qs;
                    } else {
                        red[op.red * R + tid] += racc;
                    }
                }
            }
        }
        // ---- store from the last phase's layout
        if constexpr (MODE != M_EXP) {
#pragma unroll
            for (int t = 0; t < NT && !no_store; ++t) {
                const uint64_t ga = vec_offset(opaque(gthr[t]), ilv);
#pragma unroll
                for (int j = 0; j < kRegs; ++j) {
                    if (FULL || (act && ((valid >> j) & 1u))) {
                        const uint64_t g = ga | vec_offset(L.goff(j), ilv);
                        if constexpr (MODE == M_FWD || MODE == M_REV)
                            vstore(v0 + g, v[t * NV][j]);
                        if constexpr (NV == 2)
                            vstore(v1 + g, v[1][j]);
                        if (MODE == M_HAM && ham_last)
                            eacc += re_conj_mul(v[0][j], v[1][j]);
                    }
                }
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
            bases[t] = nbases[t];
    }
    __syncthreads();
    if (MODE == M_EXP || (MODE == M_HAM && n_red > 0)) {
        const double tot = block_sum(eacc, wsum);
        if (tid == 0)
            red[0] = tot;
        __syncthreads();
    } else if (!single) {
        // accumulators -> row sums in red[r * R], fixed tree order
        for (int r = 0; r < n_red; ++r) {
            double *row = red + r * R;
            for (int s = R >> 1; s > 0; s >>= 1) {
                __syncthreads();
                if (tid < s)
                    row[tid] += row[tid + s];
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        const int rstride = (MODE == M_EXP || MODE == M_HAM || single) ? 1 : R;
        for (int r = 0; r < n_red; ++r)
            sink.base[r * sink.stride] = red[r * rstride];
    }
    __syncthreads();
}

template <int MODE, bool GEN, bool FULL, int NT, bool START, int OPS>
__global__ void __launch_bounds__(512)
k_pass(DevPass P, const DevPhase *__restrict__ phases, const DevOp *__restrict__ ops,
       const DevVBond *__restrict__ vb, const double *__restrict__ theta,
       const DevModel *__restrict__ M, double2 *__restrict__ v0, double2 *__restrict__ v1,
       double *__restrict__ partial, int stride, uint32_t ilv)
{
    extern __shared__ __align__(16) char smem[];
    const Sink sink{partial + (size_t)P.red_base * stride + blockIdx.x, stride};
    run_pass<MODE, GEN, FULL, NT, START, OPS>(P, phases, ops, vb, theta, M, v0, v1, smem, blockIdx.x,
                                  gridDim.x, (uint64_t)1 << P.nfree, ilv, sink);
}

// ------------------------------------------------------------------ batch --
// A batched evaluation is a sequence of launches per lane (a group of
// instances with its own stream): one launch per pass index of the forward,
// H and reverse schedules, each running that pass of every instance of the
// lane that has one (the first forward launch builds the start states in
// registers), with each instance's tiles split into work items over many
// workgroups; then one reduction of the partial rows.  No workgroup waits
// for another.

// GEN: the launch runs the general-diagonal path for every instance (a
// batch with any eps or V term; the path also holds for U-only instances,
// whose eps tables are zero and V classes empty), else the U-only path.
// FULL: every item's tiles fill all registers of exactly the launch's
// threads (the guard-free path; a launch of its own keeps the two paths'
// registers apart).
// An instance's pointers come from memory, so the compiler cannot see where
// they point: every access would be a flat one (vector loads for the
// wave-uniform op fields, completion counted together with LDS).  The
// vectors are global memory, the tables read-only for the launch (scalar
// loads where uniform).
typedef __attribute__((address_space(1))) double2 global_double2;
typedef const __attribute__((address_space(4))) DevPhase const_phase;
typedef const __attribute__((address_space(4))) DevOp const_op;
typedef const __attribute__((address_space(4))) DevVBond const_vbond;
typedef const __attribute__((address_space(4))) double const_double;
typedef const __attribute__((address_space(4))) DevModel const_model;

// START (forward, first schedule position): every instance's first pass
// builds its start state |b0> in registers; nothing is read.
template <int MODE, bool GEN, bool FULL, bool START, int OPS>
__global__ void __launch_bounds__(512)
k_batch_pass(const DevInstance *__restrict__ inst, const DevPass *__restrict__ passes,
             const DevWork *__restrict__ work, double *__restrict__ partial)
{
    extern __shared__ __align__(16) char smem[];
    const DevWork w = work[blockIdx.x];
    const DevInstance I = inst[w.inst];
    const DevPass P = passes[w.pass];
    const Sink sink{partial + w.part, w.stride};
    run_pass<MODE, GEN, FULL, 1, START, OPS, global_double2>(
        P, (const_phase *)I.phases, (const_op *)I.ops, (const_vbond *)I.vb,
        (const_double *)I.theta, (const_model *)I.model, (global_double2 *)I.psi,
        (global_double2 *)I.lam, smem, w.tile0, 1, w.tile1, 32u, sink);
}
#define HV_BATCH(MODE, GEN, FULL, START, OPS)                                                   \
    template __global__ void k_batch_pass<MODE, GEN, FULL, START, OPS>(                         \
        const DevInstance *, const DevPass *, const DevWork *, double *);
// batches with NP instances decode all three op kinds in their gate passes
#define HV_BATCH_ALL(GEN, FULL)                                                                 \
    HV_BATCH(M_FWD, GEN, FULL, false, OPS_HVA)                                                  \
    HV_BATCH(M_FWD, GEN, FULL, true, OPS_HVA)                                                   \
    HV_BATCH(M_HAM, GEN, FULL, false, OPS_HVA)                                                  \
    HV_BATCH(M_REV, GEN, FULL, false, OPS_HVA)                                                  \
    HV_BATCH(M_FWD, GEN, FULL, false, OPS_ALL)                                                  \
    HV_BATCH(M_FWD, GEN, FULL, true, OPS_ALL)                                                   \
    HV_BATCH(M_REV, GEN, FULL, false, OPS_ALL)
HV_BATCH_ALL(false, false)
HV_BATCH_ALL(false, true)
HV_BATCH_ALL(true, false)
HV_BATCH_ALL(true, true)
#undef HV_BATCH_ALL
#undef HV_BATCH

// out = scale[o] * sum over segments seg_ptr[o] .. seg_ptr[o+1] of the
// seg_cnt[s] partials starting at seg_off[s], in a fixed order; output o goes
// to E[out_idx[o]] for o < n_e and to grad[out_idx[o]] otherwise.
__global__ void __launch_bounds__(256)
k_reduce_seg(const double *__restrict__ partial, const int32_t *__restrict__ seg_ptr,
             const int64_t *__restrict__ seg_off, const int32_t *__restrict__ seg_cnt,
             const double *__restrict__ scale, const int64_t *__restrict__ out_idx, int n_e,
             double *__restrict__ E, double *__restrict__ grad)
{
    __shared__ double sm[256];
    const int o = blockIdx.x, tid = threadIdx.x, T = blockDim.x;
    double acc = 0.0;
    for (int sg = seg_ptr[o]; sg < seg_ptr[o + 1]; ++sg) {
        const double *p = partial + seg_off[sg];
        for (int b = tid; b < seg_cnt[sg]; b += T)
            acc += p[b];
    }
    sm[tid] = acc;
    for (int st = T >> 1; st > 0; st >>= 1) {
        __syncthreads();
        if (tid < st)
            sm[tid] += sm[tid + st];
    }
    if (tid == 0) {
        const double v = scale[o] * sm[0];
        if (o < n_e)
            E[out_idx[o]] = v;
        else
            grad[out_idx[o]] = v;
    }
}

#define HV_INSTANTIATE(MODE, GEN, FULL, NT, ST)                                               \
    HV_INSTANTIATE_OPS(MODE, GEN, FULL, NT, ST, OPS_HVA)
#define HV_INSTANTIATE_OPS(MODE, GEN, FULL, NT, ST, OPS)                                      \
    template __global__ void k_pass<MODE, GEN, FULL, NT, ST, OPS>(                              \
        DevPass, const DevPhase *, const DevOp *, const DevVBond *, const double *,             \
        const DevModel *, double2 *, double2 *, double *, int, uint32_t);
#define HV_INSTANTIATE_ALL(GEN, FULL)                                                           \
    HV_INSTANTIATE(M_FWD, GEN, FULL, 1, false)                                                  \
    HV_INSTANTIATE(M_FWD, GEN, FULL, 1, true)                                                   \
    HV_INSTANTIATE(M_REV, GEN, FULL, 1, false)                                                  \
    HV_INSTANTIATE(M_HAM, GEN, FULL, 1, false)                                                  \
    HV_INSTANTIATE(M_EXP, GEN, FULL, 1, false)
HV_INSTANTIATE_ALL(false, true)
HV_INSTANTIATE_ALL(true, true)
HV_INSTANTIATE_ALL(false, false)
HV_INSTANTIATE_ALL(true, false)
// two tiles per iteration: forward passes over full tiles, U-only models
// (the general diagonal's per-amplitude sincos needs the registers)
HV_INSTANTIATE(M_FWD, false, true, 2, false)
HV_INSTANTIATE(M_FWD, false, true, 2, true)
// gate passes of the NP circuit: hopping terms and mask phases only
HV_INSTANTIATE_OPS(M_FWD, false, true, 1, false, OPS_NP)
HV_INSTANTIATE_OPS(M_FWD, false, true, 1, true, OPS_NP)
HV_INSTANTIATE_OPS(M_REV, false, true, 1, false, OPS_NP)
HV_INSTANTIATE_OPS(M_FWD, false, false, 1, false, OPS_NP)
HV_INSTANTIATE_OPS(M_FWD, false, false, 1, true, OPS_NP)
HV_INSTANTIATE_OPS(M_REV, false, false, 1, false, OPS_NP)
#undef HV_INSTANTIATE_ALL
#undef HV_INSTANTIATE_OPS
#undef HV_INSTANTIATE

// ---------------------------------------------------------- vector kernels --
// Streaming kernels over whole state vectors (n complex128 amplitudes) for
// the drivers of the library (the Krylov ground state and overlaps):
// HBM-bound, one grid-stride loop each, kVecThreads threads per block.
// Reductions are deterministic: every block sums its share of the grid
// stride in a fixed tree order into one partial, and the partials are added
// in block order afterwards.

// Sum of (x, y) over the block in a fixed tree order; valid in thread 0.
__device__ __forceinline__ double2 block_sum2(double x, double y, double2 *sm)
{
    const int tid = threadIdx.x;
    sm[tid] = make_double2(x, y);
    for (int s = kVecThreads / 2; s > 0; s >>= 1) {
        __syncthreads();
        if (tid < s) {
            sm[tid].x += sm[tid + s].x;
            sm[tid].y += sm[tid + s].y;
        }
    }
    __syncthreads();
    return sm[0];
}

// partial[block] = sum over the block's share of conj(a_i) b_i.
__global__ void __launch_bounds__(kVecThreads)
k_vdot(const double2 *__restrict__ a, const double2 *__restrict__ b, uint64_t n,
       double2 *__restrict__ partial)
{
    __shared__ double2 sm[kVecThreads];
    double re = 0.0, im = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kVecThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride) {
        const double2 x = a[i], y = b[i];
        re += re_conj_mul(x, y);
        im += im_conj_mul(x, y);
    }
    const double2 t = block_sum2(re, im, sm);
    if (threadIdx.x == 0)
        partial[blockIdx.x] = t;
}

// Three-term Krylov recurrence: w <- w - alpha v - beta u, and
// partial[block].x = sum over the block's share of |w_i|^2 (new w).
__global__ void __launch_bounds__(kVecThreads)
k_krylov_update(double2 *__restrict__ w, const double2 *__restrict__ v,
                const double2 *__restrict__ u, double alpha, double beta, uint64_t n,
                double2 *__restrict__ partial)
{
    __shared__ double2 sm[kVecThreads];
    double acc = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kVecThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride) {
        double2 x = w[i];
        const double2 y = v[i], z = u[i];
        x.x = fma(-beta, z.x, fma(-alpha, y.x, x.x));
        x.y = fma(-beta, z.y, fma(-alpha, y.y, x.y));
        w[i] = x;
        acc = fma(x.x, x.x, fma(x.y, x.y, acc));
    }
    const double2 t = block_sum2(acc, 0.0, sm);
    if (threadIdx.x == 0)
        partial[blockIdx.x] = t;
}

// dst <- s * src (dst may be src).
__global__ void __launch_bounds__(kVecThreads)
k_vscale(double2 *dst, const double2 *src, double s, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * kVecThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride) {
        const double2 x = src[i];
        dst[i] = make_double2(s * x.x, s * x.y);
    }
}

// y <- y + a x (real a).
__global__ void __launch_bounds__(kVecThreads)
k_vaxpy(double2 *__restrict__ y, const double2 *__restrict__ x, double a, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * kVecThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride) {
        double2 t = y[i];
        const double2 z = x[i];
        t.x = fma(a, z.x, t.x);
        t.y = fma(a, z.y, t.y);
        y[i] = t;
    }
}

// out[0] = the nblk partials added in block order (one block of one thread
// group: the fixed second stage of the reductions above).
__global__ void __launch_bounds__(kVecThreads)
k_vsum(const double2 *__restrict__ partial, int nblk, double2 *__restrict__ out)
{
    __shared__ double2 sm[kVecThreads];
    double re = 0.0, im = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kVecThreads) {
        re += partial[b].x;
        im += partial[b].y;
    }
    const double2 t = block_sum2(re, im, sm);
    if (threadIdx.x == 0)
        out[0] = t;
}

// dst <- c * src with the complex scalar c read from device memory (the
// adjoint seed of the overlap loss: lambda = <ref|psi> ref).
__global__ void __launch_bounds__(kVecThreads)
k_vscale_dev(double2 *__restrict__ dst, const double2 *__restrict__ src,
             const double2 *__restrict__ c, uint64_t n)
{
    const double2 z = c[0];
    const uint64_t stride = (uint64_t)gridDim.x * kVecThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n; i += stride)
        dst[i] = cmul(z, src[i]);
}

// Overlap loss from F = |c|^2, c = <ref|psi>: out = (f, F) with
// f = log10(1 - F), and the gradient of F (adjoint sweep) turned into the
// gradient of f: df = -dF / ((1 - F) ln 10).
__global__ void __launch_bounds__(kVecThreads)
k_overlap_finish(const double2 *__restrict__ c, double *__restrict__ grad, int P,
                 double *__restrict__ out)
{
    const double F = c[0].x * c[0].x + c[0].y * c[0].y;
    const double s = -1.0 / ((1.0 - F) * 2.302585092994045684);   // ln 10
    for (int k = threadIdx.x; k < P; k += blockDim.x)
        grad[k] *= s;
    if (threadIdx.x == 0) {
        out[0] = log10(1.0 - F);
        out[1] = F;
    }
}

// ----------------------------------------------- occupation second moments --
// Q[a][b] = sum over amplitudes of |psi_x|^2 bit_a(x) bit_b(x) for every pair
// of qubits (the diagonal holds the occupations <n_a>): every diagonal
// observable quadratic in occupations -- the spin correlations of Eq. (17)
// among them -- follows from Q.  One HBM read of psi.
//
// A workgroup covers 2^(LO+MID) consecutive amplitudes: the thread id gives
// the LO low bits, a loop over j gives the MID bits above them, and the bits
// above LO+MID (the block index) are fixed in the workgroup.  Because j is
// uniform across the workgroup, a thread accumulates the mass c, the
// moments M[a] of the loop bits and their pair moments Qm[a][b] with
// branches that never diverge; the workgroup then forms the moment matrix of
// its LO+MID low bits and its mass, and k_moments_final combines the
// workgroups with their fixed high bits.  Fixed summation orders throughout.
constexpr int kMomPairs = kMomMid * (kMomMid - 1) / 2;
__device__ __forceinline__ int mom_pair(int a, int b)   // a < b < kMomMid
{
    return a * (2 * kMomMid - a - 1) / 2 + (b - a - 1);
}

// partial[blk * (1 + R*(R+1)/2)]: the mass, then the upper triangle (row
// major, diagonal included) of the workgroup's R x R moment matrix, R = LO + MID.
__global__ void __launch_bounds__(256)
k_bit_moments(const double2 *__restrict__ psi, int LO, int MID, double *__restrict__ partial)
{
    extern __shared__ __align__(16) char smem[];
    const int T = 1 << LO, t = threadIdx.x;
    const int R = LO + MID, stride = 1 + R * (R + 1) / 2;
    double c = 0.0, M[kMomMid], Q[kMomPairs];
#pragma unroll
    for (int a = 0; a < kMomMid; ++a)
        M[a] = 0.0;
#pragma unroll
    for (int a = 0; a < kMomPairs; ++a)
        Q[a] = 0.0;
    const uint64_t base = (uint64_t)blockIdx.x << R;
    for (uint32_t j = 0; j < (1u << MID); ++j) {
        const double2 v = psi[base | ((uint64_t)j << LO) | (uint32_t)t];
        const double p = v.x * v.x + v.y * v.y;
        c += p;
#pragma unroll
        for (int a = 0; a < kMomMid; ++a) {
            if (!((j >> a) & 1u))
                continue;
            M[a] += p;
#pragma unroll
            for (int b = a + 1; b < kMomMid; ++b)
                if ((j >> b) & 1u)
                    Q[mom_pair(a, b)] += p;
        }
    }
    // per-thread values to LDS: [T][1 + MID + pairs]
    const int W = 1 + kMomMid + kMomPairs;
    double *lds = (double *)smem;
    lds[t * W] = c;
#pragma unroll
    for (int a = 0; a < kMomMid; ++a)
        lds[t * W + 1 + a] = M[a];
#pragma unroll
    for (int a = 0; a < kMomPairs; ++a)
        lds[t * W + 1 + kMomMid + a] = Q[a];
    __syncthreads();
    double *out = partial + (size_t)blockIdx.x * stride;
    // entry e: 0 = mass, then (a, b), a <= b < R, row major
    for (int e = t; e < stride; e += T) {
        int a = 0, b = 0;
        if (e > 0) {
            int r = e - 1;
            while (r >= R - a) {
                r -= R - a;
                ++a;
            }
            b = a + r;
        }
        double acc = 0.0;
        for (int u = 0; u < T; ++u) {
            const double *row = lds + u * W;
            double v;
            if (e == 0)
                v = row[0];
            else if (b < LO)        // both in the thread id
                v = ((u >> a) & (u >> b) & 1) ? row[0] : 0.0;
            else if (a < LO)        // thread bit a, loop bit b
                v = ((u >> a) & 1) ? row[1 + (b - LO)] : 0.0;
            else if (a == b)        // loop bit a
                v = row[1 + (a - LO)];
            else                    // loop bits a < b
                v = row[1 + kMomMid + mom_pair(a - LO, b - LO)];
            acc += v;
        }
        out[e] = acc;
    }
}

// Q (n x n, both triangles) from the workgroup partials: block e handles one
// pair a <= b; bits >= R are bits of the workgroup index.
__global__ void __launch_bounds__(kVecThreads)
k_moments_final(const double *__restrict__ partial, int n_blk, int R, int n,
                double *__restrict__ Q)
{
    __shared__ double2 sm[kVecThreads];
    int e = blockIdx.x, a = 0;
    while (e >= n - a) {
        e -= n - a;
        ++a;
    }
    const int b = a + e;
    const int stride = 1 + R * (R + 1) / 2;
    // index of (a, b) in a workgroup's upper triangle
    auto tri = [R](int x, int y) { return 1 + x * R - x * (x - 1) / 2 + (y - x); };
    double acc = 0.0;
    for (int k = threadIdx.x; k < n_blk; k += kVecThreads) {
        const double *row = partial + (size_t)k * stride;
        double v;
        if (b < R)
            v = row[tri(a, b)];
        else if (a < R)
            v = ((k >> (b - R)) & 1) ? row[tri(a, a)] : 0.0;
        else
            v = ((k >> (a - R)) & (k >> (b - R)) & 1) ? row[0] : 0.0;
        acc += v;
    }
    const double2 tot = block_sum2(acc, 0.0, sm);
    if (threadIdx.x == 0) {
        Q[a * n + b] = tot.x;
        Q[b * n + a] = tot.x;
    }
}

// Eq. (17) from Q (spin-blocked qubits: site i up = i, down = i + ns):
// Sz_i = (<n_i,up> - <n_i,dn>)/2,
// <Sz_i Sz_j> = (Q[iu][ju] - Q[iu][jd] - Q[id][ju] + Q[id][jd]) / 4,
// C_ij = <Sz_i Sz_j> - Sz_i Sz_j.
__global__ void __launch_bounds__(kVecThreads)
k_spin_corr(const double *__restrict__ Q, int ns, double *__restrict__ C, double *__restrict__ Sz)
{
    const int n = 2 * ns;
    for (int e = threadIdx.x; e < ns * ns; e += blockDim.x) {
        const int i = e / ns, j = e % ns;
        const int iu = i, id = i + ns, ju = j, jd = j + ns;
        const double ss = 0.25 * (Q[iu * n + ju] - Q[iu * n + jd] - Q[id * n + ju] + Q[id * n + jd]);
        const double si = 0.5 * (Q[iu * n + iu] - Q[id * n + id]);
        const double sj = 0.5 * (Q[ju * n + ju] - Q[jd * n + jd]);
        C[e] = ss - si * sj;
        if (j == 0)
            Sz[i] = si;
    }
}

// ------------------------------------------------------------ misc kernels --

__global__ void k_init_basis(double2 *__restrict__ psi, uint64_t dim, uint64_t b0, uint32_t ilv)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += stride)
        psi[vec_offset(i, ilv)] = make_double2(i == b0 ? 1.0 : 0.0, 0.0);
}

// out[o] = scale[o] * sum over rows row_idx[row_ptr[o] .. row_ptr[o+1]) of the
// first row_nblk[row] entries of that partial row, in a fixed order.
__global__ void __launch_bounds__(256)
k_reduce(const double *__restrict__ partial, int stride, const int32_t *__restrict__ row_ptr,
         const int32_t *__restrict__ row_idx, const int32_t *__restrict__ row_nblk,
         const double *__restrict__ scale, double *__restrict__ out0, double *__restrict__ out1,
         int split)
{
    __shared__ double sm[256];
    const int o = blockIdx.x, tid = threadIdx.x, T = blockDim.x;
    double acc = 0.0;
    for (int r = row_ptr[o]; r < row_ptr[o + 1]; ++r) {
        const int row = row_idx[r];
        const double *p = partial + (size_t)row * stride;
        for (int b = tid; b < row_nblk[row]; b += T)
            acc += p[b];
    }
    sm[tid] = acc;
    for (int s = T >> 1; s > 0; s >>= 1) {
        __syncthreads();
        if (tid < s)
            sm[tid] += sm[tid + s];
    }
    if (tid == 0) {
        double v = scale[o] * sm[0];
        if (o < split)
            out0[o] = v;
        else
            out1[o - split] = v;
    }
}

}  // namespace hv
