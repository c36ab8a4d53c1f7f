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

// LDS slot of tile-local index l: the low four bits are XORed with a fold of
// the higher bits so that lanes whose indices differ only in high bits land
// in different banks.  A bijection on [0, 2^k).
__device__ __forceinline__ uint32_t slot(uint32_t l)
{
    return l ^ (((l >> 4) ^ (l >> 8)) & 15u);
}

// Tile-local index bits of this thread: the lane id deposited over lmask and
// the wave id over wmask (masks are wave-uniform: scalar loops).
__device__ __forceinline__ uint32_t thread_local_index(uint32_t lmask, uint32_t wmask, int tid)
{
    return pdep32((uint32_t)(tid & 63), lmask) | pdep32((uint32_t)(tid >> 6), wmask);
}

// Diagonal sub-term value D_sub(g); GEN: the model has eps or V terms.
template <bool GEN>
__device__ __forceinline__ double diag_value(const DevOp &op, uint32_t g, const DevModel *M,
                                             const DevVBond *vb)
{
    uint32_t up = g & op.umask;
    uint32_t dn = (uint32_t)((uint64_t)g >> M->ns) & op.umask;
    double d = M->U * (double)__popc(up & dn);
    if constexpr (GEN) {
        uint32_t e = g & op.emask;
        d += M->eps_byte[0][e & 255u] + M->eps_byte[1][(e >> 8) & 255u] +
             M->eps_byte[2][(e >> 16) & 255u] + M->eps_byte[3][(e >> 24) & 255u];
        for (int v = op.v_begin; v < op.v_end; ++v) {
            const DevVBond &B = vb[v];
            int ni = (int)((g >> B.q[0]) & 1u) + (int)((g >> B.q[1]) & 1u);
            int nj = (int)((g >> B.q[2]) & 1u) + (int)((g >> B.q[3]) & 1u);
            d += B.V * (double)(ni * nj);
        }
    }
    return d;
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
struct PairCtx {
    double cs, sn, t;      // rotation (cos, thread-signed sin); thread-signed (-t)
    uint32_t flip;         // bit j: register j's part of the sign is odd
    double acc;            // reduction of the op (register part of the sign applied)
};

__device__ __forceinline__ double flip_sign(double x, uint32_t bit)
{
    return __longlong_as_double(__double_as_longlong(x) ^ ((long long)bit << 63));
}

template <int MODE, int NV, int J, int JJ>
__device__ __forceinline__ void pair_op(double2 (&v)[NV][kRegs], PairCtx &x)
{
    const uint32_t fb = (x.flip >> J) & 1u;   // wave-uniform
    if constexpr (MODE == 0) {            // forward gate
        rotate(v[0][J], v[0][JJ], x.cs, flip_sign(x.sn, fb));
    } else if constexpr (MODE == 1) {     // reverse: reduce, then un-apply
        const double w =
            im_conj_mul(v[NV - 1][J], v[0][JJ]) + im_conj_mul(v[NV - 1][JJ], v[0][J]);
        x.acc += flip_sign(w, fb);
        const double ss = flip_sign(x.sn, fb);
        rotate(v[0][J], v[0][JJ], x.cs, ss);
        rotate(v[NV - 1][J], v[NV - 1][JJ], x.cs, ss);
    } else if constexpr (MODE == 2) {     // phi += (-t) s (swap) psi
        const double w = flip_sign(x.t, fb);
        v[NV - 1][J].x += w * v[0][JJ].x;
        v[NV - 1][J].y += w * v[0][JJ].y;
        v[NV - 1][JJ].x += w * v[0][J].x;
        v[NV - 1][JJ].y += w * v[0][J].y;
    } else {                              // expectation
        x.acc += flip_sign(re_conj_mul(v[0][J], v[0][JJ]), fb);
    }
}

template <int MODE, int NV, int A, int B, int X>
__device__ __forceinline__ void pair_at(double2 (&v)[NV][kRegs], PairCtx &x)
{
    constexpr int C = (A != 0 && B != 0) ? 0 : ((A != 1 && B != 1) ? 1 : 2);
    constexpr int D = 6 - A - B - C;   // the fourth register bit
    constexpr int J = (1 << A) | ((X & 1) << C) | (((X >> 1) & 1) << D);
    pair_op<MODE, NV, J, J ^ ((1 << A) | (1 << B))>(v, x);
}

template <int MODE, int NV, int A, int B>
__device__ __forceinline__ void pairs4(double2 (&v)[NV][kRegs], PairCtx &x)
{
    pair_at<MODE, NV, A, B, 0>(v, x);
    pair_at<MODE, NV, A, B, 1>(v, x);
    pair_at<MODE, NV, A, B, 2>(v, x);
    pair_at<MODE, NV, A, B, 3>(v, x);
}

template <int MODE, int NV>
__device__ __forceinline__ void hop_regs(int pair, double2 (&v)[NV][kRegs], PairCtx &x)
{
    switch (pair) {
    case 0: pairs4<MODE, NV, 0, 1>(v, x); break;
    case 1: pairs4<MODE, NV, 0, 2>(v, x); break;
    case 2: pairs4<MODE, NV, 0, 3>(v, x); break;
    case 3: pairs4<MODE, NV, 1, 2>(v, x); break;
    case 4: pairs4<MODE, NV, 1, 3>(v, x); break;
    default: pairs4<MODE, NV, 2, 3>(v, x); break;
    }
}

// Re-lay the tile out from one phase's register layout to the next through
// LDS.  slot() is linear over GF(2) and a thread's local bits never overlap
// a register's, so slot(tl | roff) = slot(tl) ^ slot(roff): one vector XOR
// per register, the register part computed on the scalar unit.
// If the wave bits stay fixed (cross == 0) every wave reads back exactly the
// slots it wrote, in program order, so no workgroup barrier is needed; every
// LDS slot a wave touches between cross-wave exchanges is its own.
template <int NV>
__device__ __forceinline__ void relayout(double2 (&v)[NV][kRegs], char *xbuf, uint32_t tl_from,
                                         const DevPhase &from, uint32_t tl_to,
                                         const DevPhase &to, uint32_t valid)
{
    const uint32_t xf = slot(tl_from) << 4, xt = slot(tl_to) << 4;
    const bool cross = to.cross != 0;
#pragma unroll
    for (int w = 0; w < NV; ++w) {
        if (cross && w > 0)
            __syncthreads();   // the previous vector's reads are done everywhere
#pragma unroll
        for (int j = 0; j < kRegs; ++j)
            if ((valid >> j) & 1u)
                *(double2 *)(xbuf + (xf ^ (slot(from.roff[j]) << 4))) = v[w][j];
        if (cross)
            __syncthreads();
        else
            __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int j = 0; j < kRegs; ++j)
            if ((valid >> j) & 1u)
                v[w][j] = *(const double2 *)(xbuf + (xt ^ (slot(to.roff[j]) << 4)));
        __builtin_amdgcn_wave_barrier();
    }
}

// Where a pass's reduction rows go: the partial array of the two-stage
// reduction (row r, block b at partial[(red_base + r) * stride + b]), or, for
// a batched instance, straight into its outputs (row_param != nullptr).
struct Sink {
    double *partial;
    int stride, block;
    const int32_t *row_param;
    double *E, *grad;
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

template <int MODE, bool GEN>
__device__ __forceinline__ void run_pass(const DevPass &P, const DevPhase *__restrict__ phases,
                                         const DevOp *__restrict__ ops,
                                         const DevVBond *__restrict__ vb,
                                         const double *__restrict__ theta,
                                         const DevModel *__restrict__ M, double2 *__restrict__ v0,
                                         double2 *__restrict__ v1, char *smem, uint64_t tile0,
                                         uint64_t tstep, const Sink &sink)
{
    constexpr int NV = (MODE == M_FWD || MODE == M_EXP) ? 1 : 2;
    const int T = blockDim.x, tid = threadIdx.x;
    // a batch workgroup may be wider than this pass's 2^tbits threads: the
    // extra threads keep zero registers and only join the barriers
    const bool act = tid < (1 << P.tbits);
    const bool ham_first = (MODE == M_HAM) && (P.flags & PF_HAM_FIRST);
    const bool ham_last = (MODE == M_HAM) && (P.flags & PF_HAM_LAST);
    const int n_red = (MODE == M_REV) ? P.n_red : (MODE == M_EXP) ? 1 : P.n_red;
    const bool single = (P.nfree == 0);
    const SmemPlan sp = smem_plan(P.k, P.c, P.n_ops, P.n_diag, n_red, T, single);
    char *xbuf = smem + sp.xbuf;
    uint32_t *offs = (uint32_t *)(smem + sp.offs);
    double2 *opc = (double2 *)(smem + sp.opc);
    double2 *dtab = (double2 *)(smem + sp.dtab);
    double *red = (double *)(smem + sp.red);

    // ---- per-workgroup set-up
    const double sign = (MODE == M_REV) ? -1.0 : 1.0;
    {
        const int nhi = P.k - P.c;
        for (int i = tid; i < (1 << nhi); i += T)
            offs[i] = pdep32((uint32_t)i, P.hi_mask);
        if constexpr (MODE == M_FWD || MODE == M_REV) {
            for (int o = tid; o < P.n_ops; o += T) {
                const DevOp op = ops[P.op_begin + o];
                if (op.kind == OP_HOP) {
                    double s, c;
                    sincos(theta[op.param] * op.t, &s, &c);
                    opc[o] = make_double2(c, sign * s);
                }
            }
            if constexpr (!GEN) {
                for (int o = 0; o < P.n_ops; ++o) {
                    const DevOp op = ops[P.op_begin + o];
                    if (op.kind != OP_DIAG)
                        continue;
                    for (int m = tid; m < kDiagTab; m += T) {
                        double s, c;
                        sincos(theta[op.param] * (M->U * (double)m), &s, &c);
                        dtab[op.dtab * kDiagTab + m] = make_double2(c, -sign * s);
                    }
                }
            }
        }
        if (single) {
            for (int r = tid; r < n_red; r += T)
                red[r] = 0.0;
        } else {
            for (int r = 0; r < n_red; ++r)
                red[r * T + tid] = 0.0;
        }
    }
    __syncthreads();
    double *wsum = red + n_red * (single ? 1 : T);

    const uint32_t cmask = (1u << P.c) - 1u;
    const uint64_t ntiles = (uint64_t)1 << P.nfree;
    const DevPhase *ph = phases + P.phase_begin;
    const uint32_t valid = ph[0].valid;
    double eacc = 0.0;
    double2 v[NV][kRegs];
    // the first phase's layout is the load layout; its thread part of the
    // global index is the same for every tile
    const uint32_t tloc0 = thread_local_index(ph[0].lmask, ph[0].wmask, tid);
    const uint32_t gthr0 = offs[tloc0 >> P.c] | (tloc0 & cmask);
    // Registers of a tile smaller than 16 amplitudes that hold nothing are
    // zero, so they add nothing to any reduction.
    auto load_tile = [&](double2 (&dst)[NV][kRegs], uint64_t t) __attribute__((always_inline)) {
        const uint32_t gb = pdep32((uint32_t)t, P.free_mask) | gthr0;
#pragma unroll
        for (int j = 0; j < kRegs; ++j) {
            dst[0][j] = make_double2(0.0, 0.0);
            if constexpr (NV == 2)
                dst[NV - 1][j] = make_double2(0.0, 0.0);
            if (act && ((valid >> j) & 1u)) {
                const uint64_t g = gb | ph[0].goff[j];
                dst[0][j] = v0[g];
                if constexpr (NV == 2)
                    if (!ham_first)
                        dst[NV - 1][j] = v1[g];
            }
        }
    };
    // One-vector passes prefetch the next tile into a second register set
    // while the current one is computed (the registers are there: occupancy
    // is bounded by LDS, not by VGPRs, for these kernels).
    constexpr bool PREFETCH = (NV == 1);
    double2 nxt[NV][kRegs];
    if (PREFETCH && tile0 < ntiles)
        load_tile(nxt, tile0);

    for (uint64_t tl = tile0; tl < ntiles; tl += tstep) {
        const uint32_t base = pdep32((uint32_t)tl, P.free_mask);
        uint32_t tloc = tloc0;
        uint32_t gthr = base | gthr0;
        if constexpr (PREFETCH) {
#pragma unroll
            for (int j = 0; j < kRegs; ++j)
                v[0][j] = nxt[0][j];
            if (tl + tstep < ntiles)
                load_tile(nxt, tl + tstep);
        } else {
            load_tile(v, tl);
        }
        for (int q = 0; q < P.n_phases; ++q) {
            if (q > 0) {
                const uint32_t tnew = thread_local_index(ph[q].lmask, ph[q].wmask, tid);
                relayout<NV>(v, xbuf, tloc, ph[q - 1], tnew, ph[q], act ? valid : 0u);
                tloc = tnew;
                gthr = base | offs[tloc >> P.c] | (tloc & cmask);
            }
            for (int o = ph[q].op_begin; o < ph[q].op_end; ++o) {
                const DevOp op = ops[P.op_begin + o];
                double dacc = 0.0;   // reverse: this op's Im <lambda|D_sub|psi>
                if (op.kind == OP_DIAG) {
#pragma unroll
                    for (int j = 0; j < kRegs; ++j) {
                        if (!((valid >> j) & 1u))
                            continue;
                        const uint32_t g = gthr | ph[q].goff[j];
                        if constexpr (MODE == M_FWD || MODE == M_REV) {
                            double2 phs;
                            if constexpr (!GEN) {
                                uint32_t up = g & op.umask;
                                uint32_t dn = (uint32_t)((uint64_t)g >> M->ns) & op.umask;
                                phs = dtab[op.dtab * kDiagTab + __popc(up & dn)];
                            } else {
                                double s, c;
                                sincos(theta[op.param] * diag_value<GEN>(op, g, M, vb), &s, &c);
                                phs = make_double2(c, -sign * s);
                            }
                            if constexpr (MODE == M_REV) {
                                double d = diag_value<GEN>(op, g, M, vb);
                                dacc += d * im_conj_mul(v[NV - 1][j], v[0][j]);
                                v[NV - 1][j] = cmul(v[NV - 1][j], phs);
                            }
                            v[0][j] = cmul(v[0][j], phs);
                        } else if constexpr (MODE == M_HAM) {
                            double d = diag_value<GEN>(op, g, M, vb);
                            v[NV - 1][j].x += d * v[0][j].x;
                            v[NV - 1][j].y += d * v[0][j].y;
                        } else {
                            double2 a = v[0][j];
                            eacc += diag_value<GEN>(op, g, M, vb) * (a.x * a.x + a.y * a.y);
                        }
                    }
                    if constexpr (MODE == M_REV) {
                        if (single) {
                            const double tot = block_sum(dacc, wsum);
                            if (tid == 0)
                                red[op.red] += tot;
                        } else {
                            red[op.red * T + tid] += dacc;
                        }
                    }
                } else {
                    PairCtx x;
                    const bool podd =
                        ((__popc(tloc & op.bm_local) + __popc((uint32_t)tl & op.bm_free)) & 1u) != 0;
                    x.flip = op.flip;
                    x.t = podd ? op.t : -op.t;   // (-t) times the thread part of the sign
                    x.acc = 0.0;
                    if constexpr (MODE == M_FWD || MODE == M_REV) {
                        x.cs = opc[o].x;
                        x.sn = podd ? -opc[o].y : opc[o].y;
                    } else {
                        x.cs = x.sn = 0.0;
                    }
                    hop_regs<MODE, NV>(op.pair, v, x);
                    // (-t) s summed: thread part of s applied here
                    const double red_op = x.t * x.acc;
                    if constexpr (MODE == M_REV) {
                        if (single) {
                            const double tot = block_sum(red_op, wsum);
                            if (tid == 0)
                                red[op.red] += tot;
                        } else {
                            red[op.red * T + tid] += red_op;
                        }
                    }
                    if constexpr (MODE == M_EXP)
                        eacc += 2.0 * red_op;
                }
            }
        }
        // ---- store from the last phase's layout
        const DevPhase &pl = ph[P.n_phases - 1];
        if constexpr (MODE != M_EXP) {
#pragma unroll
            for (int j = 0; j < kRegs; ++j) {
                if (act && ((valid >> j) & 1u)) {
                    const uint64_t g = gthr | pl.goff[j];
                    if constexpr (MODE == M_FWD || MODE == M_REV)
                        v0[g] = v[0][j];
                    if constexpr (NV == 2)
                        v1[g] = v[NV - 1][j];
                    if (MODE == M_HAM && ham_last)
                        eacc += re_conj_mul(v[0][j], v[NV - 1][j]);
                }
            }
        }
    }
    __syncthreads();
    if (MODE == M_EXP || (MODE == M_HAM && n_red > 0)) {
        const double tot = block_sum(eacc, wsum);
        if (tid == 0)
            red[0] = tot;
        __syncthreads();
    } else if (!single) {
        // per-thread rows -> row sums in red[r * T]
        for (int r = 0; r < n_red; ++r) {
            double *row = red + r * T;
            for (int s = T >> 1; s > 0; s >>= 1) {
                __syncthreads();
                if (tid < s)
                    row[tid] += row[tid + s];
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        const int rstride = (MODE == M_EXP || MODE == M_HAM || single) ? 1 : T;
        for (int r = 0; r < n_red; ++r) {
            const double val = red[r * rstride];
            if (sink.row_param) {
                const int prm = sink.row_param[P.red_base + r];
                if (prm < 0)
                    sink.E[0] = val;
                else
                    sink.grad[prm] += 2.0 * val;
            } else {
                sink.partial[(size_t)(P.red_base + r) * sink.stride + sink.block] = val;
            }
        }
    }
    __syncthreads();
}

template <int MODE, bool GEN>
__global__ void __launch_bounds__(512)
k_pass(DevPass P, const DevPhase *__restrict__ phases, const DevOp *__restrict__ ops,
       const DevVBond *__restrict__ vb, const double *__restrict__ theta,
       const DevModel *__restrict__ M, double2 *__restrict__ v0, double2 *__restrict__ v1,
       double *__restrict__ partial, int stride)
{
    extern __shared__ __align__(16) char smem[];
    Sink sink{partial, stride, (int)blockIdx.x, nullptr, nullptr, nullptr};
    run_pass<MODE, GEN>(P, phases, ops, vb, theta, M, v0, v1, smem, blockIdx.x, gridDim.x, sink);
}

// Persistent batch kernel: each workgroup claims whole instances from a
// work counter (instances are listed largest first) and runs the instance's
// initial state, forward passes, H passes and reverse passes itself, looping
// over all tiles of every pass, so no synchronisation between workgroups is
// needed.  Results go straight into the instance's E and gradient.  The
// counter must be zero at launch (k_fill_u32 before this kernel).
__global__ void __launch_bounds__(512)
k_batch(const DevInstance *__restrict__ inst, const DevPass *__restrict__ passes, int n_inst,
        unsigned int *__restrict__ counter)
{
    extern __shared__ __align__(16) char smem_all[];
    int *claim = (int *)smem_all;   // first 16 bytes; the passes use the rest
    char *smem = smem_all + 16;
    const int T = blockDim.x, tid = threadIdx.x;
    for (;;) {
        if (tid == 0)
            *claim = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int i = *claim;
        __syncthreads();
        if (i >= n_inst)
            break;
        const DevInstance I = inst[i];
        double2 *psi = (double2 *)I.psi, *lam = (double2 *)I.lam;
        for (uint64_t b = tid; b < I.dim; b += T)
            psi[b] = make_double2(b == I.neel ? 1.0 : 0.0, 0.0);
        for (int p = tid; p < I.n_params; p += T)
            I.grad[p] = 0.0;
        __syncthreads();
        Sink sink{nullptr, 0, 0, I.row_param, I.E, I.grad};
        const DevPass *ps = passes + I.pass_begin;
        for (int p = 0; p < I.n_fwd; ++p) {
            if (I.general)
                run_pass<M_FWD, true>(ps[p], I.phases, I.ops, I.vb, I.theta, I.model, psi, lam,
                                      smem, 0, 1, sink);
            else
                run_pass<M_FWD, false>(ps[p], I.phases, I.ops, I.vb, I.theta, I.model, psi, lam,
                                       smem, 0, 1, sink);
        }
        ps += I.n_fwd;
        for (int p = 0; p < I.n_ham; ++p) {
            if (I.general)
                run_pass<M_HAM, true>(ps[p], I.phases, I.ops, I.vb, I.theta, I.model, psi, lam,
                                      smem, 0, 1, sink);
            else
                run_pass<M_HAM, false>(ps[p], I.phases, I.ops, I.vb, I.theta, I.model, psi, lam,
                                       smem, 0, 1, sink);
        }
        ps += I.n_ham;
        for (int p = 0; p < I.n_rev; ++p) {
            if (I.general)
                run_pass<M_REV, true>(ps[p], I.phases, I.ops, I.vb, I.theta, I.model, psi, lam,
                                      smem, 0, 1, sink);
            else
                run_pass<M_REV, false>(ps[p], I.phases, I.ops, I.vb, I.theta, I.model, psi, lam,
                                       smem, 0, 1, sink);
        }
    }
}

__global__ void k_fill_u32(unsigned int *p, unsigned int v, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = v;
}

#define HV_INSTANTIATE(MODE, GEN)                                                          \
    template __global__ void k_pass<MODE, GEN>(DevPass, const DevPhase *, const DevOp *,   \
                                               const DevVBond *, const double *,           \
                                               const DevModel *, double2 *, double2 *,     \
                                               double *, int);
HV_INSTANTIATE(M_FWD, false)
HV_INSTANTIATE(M_REV, false)
HV_INSTANTIATE(M_HAM, false)
HV_INSTANTIATE(M_EXP, false)
HV_INSTANTIATE(M_FWD, true)
HV_INSTANTIATE(M_REV, true)
HV_INSTANTIATE(M_HAM, true)
HV_INSTANTIATE(M_EXP, true)
#undef HV_INSTANTIATE

// ------------------------------------------------------------ misc kernels --

__global__ void k_init_basis(double2 *__restrict__ psi, uint64_t dim, uint64_t b0)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += stride)
        psi[i] = make_double2(i == b0 ? 1.0 : 0.0, 0.0);
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
