// sector.hip -- the particle-number sector form of the HVA circuit on gfx950.
//
// H (Eq. (1)/(2)/(15)/(16)) and every gate of the Eq. (7) layer keep the
// numbers of spin-up and spin-down electrons, so the circuit state prepared
// from the checkerboard basis state |b0> (Sec. 2.1) has nonzero amplitudes
// only on the basis states with b0's (N_up, N_dn).  This file stores only
// those: the state is the matrix Psi[r_dn][r_up] of C(Ns, N_dn) x C(Ns, N_up)
// complex128 amplitudes, r_s the rank of the spin-s site pattern among the
// patterns with N_s electrons in increasing numeric order (at 4x4 half
// filling 12870 x 12870 = 1.66e8 amplitudes, 2.6 GB, against 2^32 and
// 64 GiB for the full vector).
//
// A hopping term of spin s changes only the spin-s pattern, so in the layout
// whose rows are indexed by the other spin (layout A: rows r_dn, columns r_up;
// layout B: the transpose) every spin-s gate acts inside rows, with the same
// pairing of columns in every row.  A row pass holds one row per workgroup
// in registers and applies a run of gates to it; a gate's partner amplitudes
// come through LDS, each active element writing its value to its pair slot
// and reading the partner's from the neighbouring slot (pair slots and the
// Jordan-Wigner sign precomputed per gate and rank on the host).  Between
// runs of the two spins the state is transposed (A <-> B).  The diagonal
// phase acts element-wise in either layout.
//
// Schedule of L layers: [D_0, up_0] (A), [dn_0, D_1, dn_1] (B),
// [up_1, D_2, up_2] (A), ...: within a layer the up and down hops commute,
// so each row pass carries the second half of one layer and the first half
// of the next, L + 1 row passes and L transposes per sweep.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/hubbard.h"
#include "hubvqe.hpp"
#include "phase.hpp"

namespace hv {

// engine.hip: the handle's model, its unique id, the thread's last error,
// the Lanczos recurrence on a Hamiltonian given as a callback
const Model *handle_model(hubbard_t h);
uint64_t handle_uid(hubbard_t h);
hubbard_status set_error(hubbard_status s, const std::string &msg);
using ApplyH = std::function<hubbard_status(const double2 *, double2 *)>;
hubbard_status lanczos_run(const ApplyH &apply, uint64_t n, const double2 *start_dev,
                           int32_t max_iter, double tol, double *E0, int32_t *iters,
                           double *residual, double2 *gs_dev, double2 *const buf[3],
                           double2 *partial, hipStream_t s);
size_t lanczos_partial_bytes();

namespace sec {

constexpr int kT = 1024;                  // threads of a row workgroup
constexpr int kWaves = kT / 64;
constexpr int kMaxRed = 16;               // reduction slots of one row pass
constexpr int kGrid = 1024;               // at most this many row workgroups
constexpr int kMaxRows = 13 * kT;         // longest row: C(16, 8) = 12870
constexpr int kZero = 16;                 // zeroed LDS slots (one per bank group) read by inactive elements

// Register tile of a row of n elements over kT threads: rpt_of(n) elements
// per thread (element t + j kT in thread t).  A gate's code table holds
// rp_of(rpt) >= rpt codes per thread in chunks of cw_of(rpt) consecutive
// codes: element j of thread t is entry code_index(rpt, t, j), so that a
// thread reads a chunk with one LDS load and a wave's loads are contiguous.
__host__ __device__ constexpr int rpt_of(int n)
{
    return n <= kT ? 1 : n <= 2 * kT ? 2 : n <= 4 * kT ? 4 : n <= 8 * kT ? 8 : 13;
}
__host__ __device__ constexpr int rp_of(int rpt) { return rpt == 13 ? 16 : (rpt < 2 ? 2 : rpt); }
__host__ __device__ constexpr int cw_of(int rpt) { return rp_of(rpt) < 8 ? rp_of(rpt) : 8; }
__host__ __device__ constexpr int code_index(int rpt, int t, int j)
{
    return ((j / cw_of(rpt)) * kT + t) * cw_of(rpt) + j % cw_of(rpt);
}

enum { S_FWD = 0, S_REV = 1, S_HAM = 2 };
enum { SOP_HOP = 0, SOP_DIAG = 1 };
enum { SF_NO_STORE = 1, SF_NEGATE = 2 };

// One operation of a row pass (32 bytes).  HOP: the gate exp(-i th t h) of
// one bond and spin (h = a+_i a_j + h.c. on that spin's sites); DIAG: the
// layer's diagonal exp(-i th D).
struct SecOp {
    int32_t kind;
    int32_t param;    // theta index
    int32_t tab;      // HOP: offset of its code table (kT rp_of(rpt) entries)
    int32_t red;      // REV: reduction slot of the parameter within the pass
    double t;         // HOP: t_b
    int32_t nxt[2];   // the HOP op that follows this one in the pass's list in
                      // forward [0] and reverse [1] execution order, wrapping
                      // around (its code table is fetched while this op runs)
};

// Device constants of a model's sector.
struct SecModel {
    int32_t ns, nvb;
    int32_t n[2];              // patterns of each spin
    double U;
    const uint32_t *pat[2];    // site pattern of each rank
    const double *base[2];     // sum_i eps_i p_i + sum_b V_b p_i p_j of each rank
    const uint16_t *code;      // per gate: LDS slot | sign << 15 (a zero slot: not active)
                               // of every column, at code_index (kT rp_of(rpt) entries)
    int32_t vi[kMaxBonds], vj[kMaxBonds];
    double vV[kMaxBonds];
};

// D of the basis state with row pattern rp and column pattern cp:
// U #(doubly occupied) + base(rp) + base(cp) + sum_b V_b (rp_i cp_j + cp_i rp_j).
template <typename MT>
__device__ __forceinline__ double diag_d(const MT *M, uint32_t rp, double rb, uint32_t cp,
                                         double cb)
{
    double d = M->U * (double)__popc(rp & cp) + rb + cb;
    for (int v = 0; v < M->nvb; ++v) {
        const int i = M->vi[v], j = M->vj[v];
        const uint32_t x = (((rp >> i) & (cp >> j)) | ((cp >> i) & (rp >> j))) & 1u;
        const uint32_t y = ((rp >> i) & (cp >> j) & (cp >> i) & (rp >> j)) & 1u;
        d += M->vV[v] * (double)(x + y);
    }
    return d;
}

// The value is final here: the work that produced it stays before the next
// workgroup barrier instead of being sunk past it (which would keep the
// inputs, a partner value each, live across the barrier).
__device__ __forceinline__ void pin(double2 &v) { asm volatile("" : "+v"(v.x), "+v"(v.y)); }
__device__ __forceinline__ void pin(double &v) { asm volatile("" : "+v"(v)); }

// x <- x m + q, and acc <- acc + m q, computed in the registers of x (acc):
// the register tile is updated in place.  (Left to itself the allocator
// writes an op's results to fresh registers and copies the whole tile back
// at the end of the op: twice the tile's registers and a copy per element.)
__device__ __forceinline__ void fma_ip(double &x, double m, double q)
{
    asm("v_fma_f64 %0, %0, %1, %2" : "+v"(x) : "v"(m), "v"(q));
}
__device__ __forceinline__ void fmac_ip(double &acc, double m, double q)
{
    asm("v_fma_f64 %0, %1, %2, %0" : "+v"(acc) : "v"(m), "v"(q));
}

// x from another lane of the same 16-lane row (DPP control CTRL), both
// 32-bit halves.
template <int CTRL>
__device__ __forceinline__ double row_dpp(double y)
{
    const long long b = __double_as_longlong(y);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double lane_value(double y, int l)
{
    const long long b = __double_as_longlong(y);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum of x over the wave, the same value in every lane: each 16-lane row
// summed by lane permutations (no LDS traffic), then the four rows' sums.
__device__ __forceinline__ double wave_sum(double x)
{
    x += row_dpp<0xB1>(x);    // quad_perm [1,0,3,2]: pairs
    x += row_dpp<0x4E>(x);    // quad_perm [2,3,0,1]: quads
    x += row_dpp<0x141>(x);   // row_half_mirror: the other quad of the half row
    x += row_dpp<0x140>(x);   // row_mirror: the other half of the row
    return (lane_value(x, 0) + lane_value(x, 16)) + (lane_value(x, 32) + lane_value(x, 48));
}

// A thread's gate codes, two 16-bit codes per register (LDS slot | sign <<
// 15; an element the gate leaves alone has a zero slot, at or above the
// first zero slot nz, with sign 0).
template <int RPT>
struct Codes {
    uint32_t w[rp_of(RPT) / 2];
    __device__ __forceinline__ uint32_t get(int j) const { return (w[j >> 1] >> (16 * (j & 1))) & 0xFFFFu; }
};

typedef const __attribute__((address_space(1))) uint32_t gu32;
typedef const __attribute__((address_space(1))) uint16_t gu16;
typedef const __attribute__((address_space(1))) double gf64;
typedef __attribute__((address_space(1))) double2 gc128;
// The op list, its angles and the model constants are read-only for the
// whole launch: constant address space, so that their wave-uniform loads are
// scalar loads (as generic pointers they became vector loads with a wait in
// front of every op).
typedef const __attribute__((address_space(4))) SecOp kSecOp;
typedef const __attribute__((address_space(4))) SecModel kSecModel;
typedef const __attribute__((address_space(4))) double2 kc128;
typedef const __attribute__((address_space(4))) uint32_t ku32;
typedef const __attribute__((address_space(4))) double kf64;

// The gate's codes of thread t, from the LDS copy of its table: one load
// per chunk (codes past the row end name zero slots in the table).
template <int RPT>
__device__ __forceinline__ Codes<RPT> load_codes(const uint16_t *cb, uint32_t t)
{
    constexpr int CW = cw_of(RPT), NCH = rp_of(RPT) / CW;
    Codes<RPT> c;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        const uint16_t *q = cb + ((size_t)ch * kT + t) * CW;
        if constexpr (CW == 8) {
            const uint4 v = *(const uint4 *)q;
            c.w[ch * 4 + 0] = v.x;
            c.w[ch * 4 + 1] = v.y;
            c.w[ch * 4 + 2] = v.z;
            c.w[ch * 4 + 3] = v.w;
        } else if constexpr (CW == 4) {
            const uint2 v = *(const uint2 *)q;
            c.w[ch * 2 + 0] = v.x;
            c.w[ch * 2 + 1] = v.y;
        } else {
            c.w[ch] = *(const uint32_t *)q;
        }
    }
    return c;
}

// The gate's codes of thread t straight from its table in global memory
// (the same chunks as load_codes: a wave's loads are contiguous).
template <int RPT>
__device__ __forceinline__ Codes<RPT> load_codes_g(const gu16 *__restrict__ src, uint32_t t)
{
    constexpr int CW = cw_of(RPT), NCH = rp_of(RPT) / CW;
    Codes<RPT> c;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        // CW / 2 adjacent dwords: one vector load
        const gu32 *q = (const gu32 *)(src + ((size_t)ch * kT + t) * CW);
#pragma unroll
        for (int k = 0; k < (CW + 1) / 2; ++k)
            c.w[ch * ((CW + 1) / 2) + k] = q[k];
    }
    return c;
}

// Asynchronous copy of a gate's code table (kT rp_of(RPT) 16-bit entries)
// from global memory into LDS, a dword per lane and round, without
// registers; complete for the issuing wave after its vmcnt wait.
template <int TT, int RPT>
__device__ __forceinline__ void fetch_codes(const gu16 *__restrict__ src, uint16_t *cb, int tid)
{
    constexpr int ROUNDS = kT * rp_of(RPT) / 2 / TT;
    // the wave's LDS base is uniform (a scalar register, no per-round
    // readfirstlane); the lane's source offset is 32-bit (scalar base +
    // vector offset addressing)
    const uint32_t wbase = __builtin_amdgcn_readfirstlane((uint32_t)(tid & ~63));
    const gu32 *__restrict__ s32 = (const gu32 *)src;
#pragma unroll
    for (int k = 0; k < ROUNDS; ++k) {
        const uint32_t d0 = (uint32_t)k * TT;
        __builtin_amdgcn_global_load_lds(
            (const __attribute__((address_space(1))) void *)(s32 + (d0 + (uint32_t)tid)),
            (__attribute__((address_space(3))) void *)(cb + 2 * (d0 + wbase)), 4, 0, 0);
    }
}

// One gate's exchange of vector x through the pair slots: every active
// element publishes its value to its slot, then every element calls use(j,
// partner, active, sign bit) with the partner read from its slot XOR 1 (the
// Jordan-Wigner sign (-1)^bit).  An inactive element's code names one of
// the kZero zero slots, so its "partner" is zero and every term with it
// vanishes whatever the sign: the reads and updates are branch-free and
// take no select.  The zero slot of the inactive lanes of a group of 16
// lanes is chosen by the host in a bank group that none of the group's
// active reads uses (the lanes of a 16-byte LDS access are served in such
// groups; all of the group's inactive lanes read the same slot, a
// broadcast).  (Inactive elements writing to zero slots too, to make the
// writes branch-free as well, cost 4 % of an evaluation in LDS traffic.)
// The codes are in registers: they are made opaque before each half, so that
// the decoded slot addresses are not kept across the barrier; mid() (the
// next gate's table fetch into the LDS the codes came from) is issued after
// the reads, before the closing barrier (every thread holds its codes since
// the publishing barrier; issued right after that barrier, the copies
// overlapped the reads and the gate took longer).
template <int RPT, int INF, typename G, typename F>
__device__ __forceinline__ void exchange(const double2 (&x)[RPT], Codes<RPT> cd, double2 *xch,
                                         uint32_t nz, G &&mid, F &&use)
{
#pragma unroll
    for (int k = 0; k < rp_of(RPT) / 2; ++k)
        asm volatile("" : "+v"(cd.w[k]));
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const uint32_t sl = cd.get(j) & 0x7FFFu;
        if (sl < nz)
            xch[sl] = x[j];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < rp_of(RPT) / 2; ++k)
        asm volatile("" : "+v"(cd.w[k]));
    // INF partner values in flight per thread: element j + INF - 1's read is
    // issued before element j is updated (the other waves hide the rest of
    // the LDS latency; the register tile keeps its registers)
    auto partner = [&](int j) __attribute__((always_inline)) {
        return xch[(cd.get(j) & 0x7FFFu) ^ 1u];
    };
    double2 pq[INF];
#pragma unroll
    for (int k = 0; k + 1 < INF && k < RPT; ++k)
        pq[k] = partner(k);
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const uint32_t c = cd.get(j);
        if (j + INF - 1 < RPT)
            pq[(j + INF - 1) % INF] = partner(j + INF - 1);
        if constexpr (INF > 1)
            __builtin_amdgcn_sched_barrier(0);
        use(j, pq[j % INF], ((c & 0x7FFFu) ^ 1u) < nz, (c >> 15) & 1u);
        __builtin_amdgcn_sched_barrier(0);
    }
    mid();
    __builtin_amdgcn_s_waitcnt(0);   // this wave's part of mid()'s copies has landed
    __syncthreads();
}

// Row pass.  Each workgroup takes rows blockIdx.x, blockIdx.x + gridDim.x, ...
// of the layout whose columns are indexed by spin `col`; thread t holds the
// row's elements t + j TT, j < RPT (TT = kT, the layout of the code tables).
//   S_FWD: v0 <- ops applied in order.
//   S_REV: v0 = chi <- ops un-applied in reverse order; the expectation
//          <chi| G |chi> of every op before its un-application goes to its
//          reduction slot (negated with SF_NEGATE).  The adjoint bracket
//          Im <lambda|G|psi> is (<chi2|G|chi2> - <chi1|G|chi1>) / 4 with
//          chi1, chi2 = lambda +- i psi, both of which evolve by the same
//          un-applied gates: two one-vector sweeps instead of one sweep
//          holding both psi and lambda.
//   S_HAM: v1 <- sum of the ops' generators applied to v0 (D if a DIAG op
//          is present), slot 0 <- Re <v0|v1>.
// Reductions: per-wave sums in LDS, then per workgroup one partial per slot
// at partial[(row0 + slot) * pstride + blockIdx.x] (fixed order).
// GEN: the diagonal has eps or V terms (D from the pattern tables, its phase
// by cis_neg); else D = U #(doubly occupied) and its phase comes from the
// op's table dph[op.tab][k] = exp(-i th U k), copied into LDS at the start.
template <int MODE, int TT, int RPT, bool GEN>
__global__ void __launch_bounds__(TT)
k_sec_rows(const SecOp *__restrict__ ops, int n_ops, int col, int n_red,
           const double2 *__restrict__ ang, const double2 *__restrict__ dph,
           const SecModel *__restrict__ M, double2 *__restrict__ v0, double2 *__restrict__ v1,
           double *__restrict__ partial, int row0, int pstride, int flags, int xch_elems)
{
    static_assert(TT == kT, "the code tables are laid out for kT threads");
    const kSecOp *__restrict__ kops = (const kSecOp *)ops;
    const kc128 *__restrict__ kang = (const kc128 *)ang;
    const kSecModel *__restrict__ kM = (const kSecModel *)M;
    constexpr int N = RPT;         // elements per thread
    constexpr int kWv = TT / 64;   // waves of the workgroup
    constexpr bool REV = MODE == S_REV;
    // partner reads in flight per thread in a gate's exchange (H: one, its
    // two register tiles leave no registers for more)
    constexpr int kInFlight = MODE == S_HAM ? 1 : 3;
    // gate codes: forward and reverse passes load the next gate's codes from
    // global memory into registers while a gate is applied; H (no registers
    // to spare) copies them into LDS (cbuf)
    constexpr bool RC = MODE != S_HAM;
    // column of thread u's element e
    auto elem = [](uint32_t u, int e) -> uint32_t { return u + (uint32_t)(e * TT); };
    extern __shared__ __align__(16) char smem[];
    double2 *xch = (double2 *)smem;   // pair slots below xch_elems, then kZero zero slots
    double *acc = (double *)(smem + (size_t)(xch_elems + kZero) * 16);   // kMaxRed x kWaves
    double2 *dloc = (double2 *)(acc + kMaxRed * kWaves);   // the pass's U-count phase table
    double2 *cis = dloc + kDiagTab;                                       // unit phases
    uint16_t *cbuf = (uint16_t *)(cis + (1u << kCisBits));                // the next gate's codes
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t n = (uint32_t)kM->n[col];
    const int nr = kM->n[1 - col];
    // the tables' pointers come from memory: global address space, so that
    // the loads take a scalar base and a 32-bit offset
    const gu32 *__restrict__ cpat = (const gu32 *)kM->pat[col];
    const gf64 *__restrict__ cbase = (const gf64 *)kM->base[col];
    const gu16 *__restrict__ gcode = (const gu16 *)kM->code;
    // row-uniform: scalar loads
    const ku32 *__restrict__ rpat = (const ku32 *)kM->pat[1 - col];
    const kf64 *__restrict__ rbase = (const kf64 *)kM->base[1 - col];
    for (int i = tid; i < kMaxRed * kWv; i += TT)
        acc[i] = 0.0;
    for (int i = tid; i < kZero; i += TT)   // read by inactive elements, never written
        xch[xch_elems + i] = make_double2(0.0, 0.0);
    if constexpr (MODE != S_HAM && GEN)
        build_cis(cis, tid, TT);
    // execution position of the pass's diagonal op (at most one; n_ops: none)
    int dexec = n_ops;
    for (int io = 0; io < n_ops; ++io)
        if (kops[io].kind == SOP_DIAG)
            dexec = REV ? n_ops - 1 - io : io;
    // U-only gate passes: the diagonal op's phase table in LDS (conjugated to
    // un-apply), looked up per element by the number of doubly occupied sites
    if constexpr (MODE != S_HAM && !GEN) {
        if (dexec < n_ops && tid < kDiagTab) {
            double2 e = dph[(size_t)kops[REV ? n_ops - 1 - dexec : dexec].tab * kDiagTab + tid];
            if constexpr (REV)
                e.y = -e.y;
            dloc[tid] = e;
        }
    }
    // cbuf holds the code table of op `ready` (-1: none); the first hopping
    // op in execution order now
    int ready = -1;
    for (int oi = 0; oi < n_ops && ready < 0; ++oi) {
        const int io = REV ? n_ops - 1 - oi : oi;
        if (kops[io].kind == SOP_HOP)
            ready = io;
    }
    Codes<RPT> pre;   // RC: the codes of op `ready`
    if (ready >= 0) {
        if constexpr (RC) {
            pre = load_codes_g<RPT>(gcode + kops[ready].tab, (uint32_t)tid);
        } else {
            fetch_codes<TT, RPT>(gcode + kops[ready].tab, cbuf, tid);
            __builtin_amdgcn_s_waitcnt(0);
        }
    }
    __syncthreads();
    double eacc = 0.0;

    for (int r = blockIdx.x; r < nr; r += gridDim.x) {
        uint32_t tr = (uint32_t)tid;   // per-row indices are not kept across rows
        asm volatile("" : "+v"(tr));
        const uint32_t rp = rpat[r];
        const double rb = rbase[r];
        gc128 *__restrict__ x0 = (gc128 *)(v0 + (size_t)r * (size_t)n);
        gc128 *__restrict__ x1 = (gc128 *)(v1 + (size_t)r * (size_t)n);
        // elements past the row end (the last register of some threads) hold
        // zero: every op leaves them zero and they add nothing to a sum
        double2 a[N], b[N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const uint32_t idx = elem(tr, j), ic = min(idx, n - 1);
            a[j] = make_double2(x0[ic].x, x0[ic].y);
            a[j] = idx < n ? a[j] : make_double2(0.0, 0.0);
            b[j] = make_double2(0.0, 0.0);
        }
        // this thread's part of the current reduction slot's sum (REV)
        double racc = 0.0;
        // op at execution position oi; IS_DIAG: the diagonal op, else a hop
        auto step = [&](int oi, auto diag_tag) __attribute__((always_inline)) {
            constexpr bool IS_DIAG = decltype(diag_tag)::value;
            const int io = REV ? n_ops - 1 - oi : oi;
            const kSecOp &op = kops[io];
            // the element indices recomputed per op, not kept live (with
            // their 64-bit table addresses) across the op loop
            uint32_t t = (uint32_t)tid;
            asm volatile("" : "+v"(t));
            if constexpr (IS_DIAG) {
                double th = 0.0;
                if constexpr (MODE != S_HAM)
                    th = kang[io].x;
                // every element's column pattern (U-only: its number of doubly
                // occupied sites) first, the loads in flight together
                uint32_t kc[N];
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    const uint32_t cp = cpat[min(elem(t, j), n - 1)];   // past the end: a zero element
                    kc[j] = GEN ? cp : __popc(rp & cp);
                }
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    {
                        const uint32_t k = kc[j];
                        const double d = GEN ? diag_d(kM, rp, rb, k, cbase[min(elem(t, j), n - 1)])
                                             : kM->U * (double)k;
                        if constexpr (MODE == S_HAM) {
                            fmac_ip(b[j].x, d, a[j].x);
                            fmac_ip(b[j].y, d, a[j].y);
                        } else {
                            // exp(-i th D) forward, exp(+i th D) to un-apply
                            double2 e;
                            if constexpr (GEN) {
                                e = cis_neg(REV ? -th * d : th * d, cis);
                            } else {
                                e = dloc[k];
                            }
                            if constexpr (REV)   // <chi|D|chi> term
                                racc += d * (a[j].x * a[j].x + a[j].y * a[j].y);
                            // a <- e a
                            const double tx = e.y * a[j].y, ty = e.y * a[j].x;
                            fma_ip(a[j].x, e.x, -tx);
                            fma_ip(a[j].y, e.x, ty);
                        }
                    }
                    // one element's phase at a time: fewer live temporaries
                    __builtin_amdgcn_sched_barrier(0);
                }
            } else {
                double cs = 0.0, sn = 0.0;
                if constexpr (MODE != S_HAM) {
                    cs = kang[io].x;                 // (cos, sin)(th t)
                    sn = REV ? -kang[io].y : kang[io].y;   // un-apply: sin -> -sin
                }
                const double mt = -op.t;
                Codes<RPT> cd;
                if constexpr (RC) {
                    if (ready != io)   // not prefetched (the op list's nxt links are broken)
                        pre = load_codes_g<RPT>(gcode + op.tab, t);
                    cd = pre;
                } else {
                    if (ready != io) {
                        fetch_codes<TT, RPT>(gcode + op.tab, cbuf, tid);
                        __builtin_amdgcn_s_waitcnt(0);
                        __syncthreads();
                    }
                    cd = load_codes<RPT>(cbuf, t);
                }
                // the next hop's codes: loaded into registers now (RC), or
                // copied into cbuf at the end of this one's exchange (every
                // thread has its codes in registers by then)
                ready = (r + (int)gridDim.x < nr || oi + 1 < n_ops) ? op.nxt[REV ? 1 : 0] : -1;
                const int nxt = ready;
                if constexpr (RC) {
                    if (nxt >= 0)
                        pre = load_codes_g<RPT>(gcode + kops[nxt].tab, t);
                }
                // w = sign (active) or 0 (inactive: cos factor 1, no partner term)
                exchange<RPT, kInFlight>(a, cd, xch, (uint32_t)xch_elems, [&]() {
                    if (!RC && nxt >= 0)
                        fetch_codes<TT, RPT>(gcode + kops[nxt].tab, cbuf, tid);
                }, [&](int j, double2 p, bool act, uint32_t sgn) {
                    // s (-t) and s sn by a flip of the sign bit (p = 0 when
                    // inactive: those terms then vanish without a select)
                    if constexpr (MODE == S_HAM) {   // phi += (-t) s psi_x'
                        const double m = flip_sign(mt, sgn);
                        fmac_ip(b[j].x, m, p.x);
                        fmac_ip(b[j].y, m, p.y);
                        pin(b[j]);
                    } else {
                        const double2 y = a[j];
                        if constexpr (REV) {   // <chi|h|chi> term: (-t) s Re(conj(chi_x) chi_x')
                            racc += flip_sign(mt, sgn) * (y.x * p.x + y.y * p.y);
                            pin(racc);
                        }
                        const double ss = flip_sign(sn, sgn);   // x <- cs x + i s sn x'
                        const double c = act ? cs : 1.0;
                        fma_ip(a[j].x, c, -ss * p.y);
                        fma_ip(a[j].y, c, ss * p.x);
                        pin(a[j]);
                    }
                });
            }
        };
        // REV: the thread's sum of a run of ops with one reduction slot into
        // that slot (one wave reduction per run, not per op)
        auto flush = [&](int red) __attribute__((always_inline)) {
            if constexpr (REV) {
                const double w = wave_sum(racc);
                if (lane == 0)
                    acc[red * kWv + wave] += w;
                racc = 0.0;
            }
        };
        // the hops at execution positions [o0, o1) (REV: in runs of equal
        // reduction slots)
        auto hops = [&](int o0, int o1) __attribute__((always_inline)) {
            if constexpr (REV) {
                for (int oi = o0; oi < o1;) {
                    const int red = kops[n_ops - 1 - oi].red;
                    do {
                        step(oi, std::false_type());
                        ++oi;
                    } while (oi < o1 && kops[n_ops - 1 - oi].red == red);
                    flush(red);
                }
            } else {
                for (int oi = o0; oi < o1; ++oi)
                    step(oi, std::false_type());
            }
        };
        // the hops before the diagonal, the diagonal, the hops after it: each
        // loop body is a single path, so the register tile keeps its
        // registers across ops (a loop over both kinds merges two versions
        // of the tile at the end of every op, and copies it)
        hops(0, dexec);
        if (dexec < n_ops) {
            step(dexec, std::true_type());
            flush(kops[REV ? n_ops - 1 - dexec : dexec].red);
        }
        hops(dexec + 1, n_ops);
        if constexpr (MODE == S_HAM) {
#pragma unroll
            for (int j = 0; j < N; ++j)
                eacc += a[j].x * b[j].x + a[j].y * b[j].y;
        }
        if (!(flags & SF_NO_STORE)) {
            // addresses recomputed here rather than kept from the loads
            uint32_t t = (uint32_t)tid;
            asm volatile("" : "+v"(t));
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const uint32_t idx = elem(t, j);
                if (idx < n) {
                    if constexpr (MODE != S_HAM) {
                        x0[idx].x = a[j].x;
                        x0[idx].y = a[j].y;
                    } else {
                        x1[idx].x = b[j].x;
                        x1[idx].y = b[j].y;
                    }
                }
            }
        }
    }
    if constexpr (MODE == S_HAM) {
        const double w = wave_sum(eacc);
        if (lane == 0)
            acc[wave] = w;
    }
    __syncthreads();
    if constexpr (MODE != S_FWD) {
        if (tid < n_red) {
            double s = 0.0;
            for (int w = 0; w < kWv; ++w)
                s += acc[tid * kWv + w];
            partial[(size_t)(row0 + tid) * pstride + blockIdx.x] = (flags & SF_NEGATE) ? -s : s;
        }
    }
}

// chi1 <- lambda + i psi in psi's place, chi2 <- lambda - i psi in lambda's.
__global__ void __launch_bounds__(256)
k_sec_mix(double2 *__restrict__ psi, double2 *__restrict__ lam, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const double2 p = psi[i], l = lam[i];
        psi[i] = make_double2(l.x - p.y, l.y + p.x);
        lam[i] = make_double2(l.x + p.y, l.y - p.x);
    }
}

// Per op of a sweep: HOP (cos, sin)(th_param t_b); DIAG (th_param, 0) and
// its phase table dph[op.tab][k] = exp(-i th U k), k = 0 .. kDiagTab - 1.
__global__ void __launch_bounds__(256)
k_sec_angles(const SecOp *__restrict__ ops, int n, const double *__restrict__ theta, double U,
             double2 *__restrict__ ang, double2 *__restrict__ dph)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const SecOp o = ops[i];
        if (o.param < 0)   // a term of H: no angle
            continue;
        if (o.kind == SOP_HOP) {
            double s, c;
            sincos(theta[o.param] * o.t, &s, &c);
            ang[i] = make_double2(c, s);
        } else {
            const double th = theta[o.param];
            ang[i] = make_double2(th, 0.0);
            for (int k = 0; k < kDiagTab; ++k) {
                double s, c;
                sincos(th * (U * (double)k), &s, &c);
                dph[(size_t)o.tab * kDiagTab + k] = make_double2(c, -s);
            }
        }
    }
}

// out[c nr + r] = in[r nc + c] (add: out += that), through 64 x 64 LDS tiles
// (1 KB row segments; 32 x 32 tiles reached 3.7 TB/s at 12870 x 12870, these
// 4.6 TB/s).
constexpr int kTrTile = 64, kTrThreads = 512;
__global__ void __launch_bounds__(kTrThreads)
k_sec_transpose(const double2 *__restrict__ in, double2 *__restrict__ out, int nr, int nc, int add)
{
    constexpr int RW = kTrThreads / kTrTile;   // tile rows per sweep of the threads
    __shared__ double2 tile[kTrTile][kTrTile + 1];
    const int c0 = blockIdx.x * kTrTile, r0 = blockIdx.y * kTrTile;
    const int tx = threadIdx.x % kTrTile, ty = threadIdx.x / kTrTile;
    for (int k = ty; k < kTrTile; k += RW) {
        const int r = r0 + k, c = c0 + tx;
        if (r < nr && c < nc)
            tile[k][tx] = in[(size_t)r * nc + c];
    }
    __syncthreads();
    for (int k = ty; k < kTrTile; k += RW) {
        const int c = c0 + k, r = r0 + tx;
        if (r < nr && c < nc) {
            double2 v = tile[tx][k];
            double2 *o = out + (size_t)c * nr + r;
            if (add) {
                const double2 w = *o;
                v.x += w.x;
                v.y += w.y;
            }
            *o = v;
        }
    }
}

// psi <- the basis state at position `at` (zeros elsewhere).
__global__ void __launch_bounds__(256) k_sec_basis(double2 *__restrict__ psi, size_t n, size_t at)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        psi[i] = make_double2(i == at ? 1.0 : 0.0, 0.0);
}

// out[o] = scale[o] * sum over partial rows rows[ptr[o] .. ptr[o+1]) of the
// nblk[row] entries each (the workgroups of the pass that wrote it), in a
// fixed order; o = 0 goes to E, o >= 1 to grad[o-1].
__global__ void __launch_bounds__(256)
k_sec_reduce(const double *__restrict__ partial, int pstride, const int32_t *__restrict__ nblk,
             const int32_t *__restrict__ ptr, const int32_t *__restrict__ rows,
             const double *__restrict__ scale, double *__restrict__ E, double *__restrict__ grad)
{
    __shared__ double sm[256];
    const int o = blockIdx.x, tid = threadIdx.x;
    double s = 0.0;
    for (int k = ptr[o]; k < ptr[o + 1]; ++k) {
        const double *p = partial + (size_t)rows[k] * pstride;
        for (int b = tid; b < nblk[rows[k]]; b += 256)
            s += p[b];
    }
    sm[tid] = s;
    for (int st = 128; st > 0; st >>= 1) {
        __syncthreads();
        if (tid < st)
            sm[tid] += sm[tid + st];
    }
    if (tid == 0) {
        const double v = scale[o] * sm[0];
        if (o == 0)
            E[0] = v;
        else
            grad[o - 1] = v;
    }
}

// ------------------------------------------------------------------ host --

struct RowPass {
    int col = 0;
    std::vector<SecOp> ops;
    std::vector<int> red_param;   // parameter of each reduction slot
};

// Sector tables of one model on one device.
struct Tables {
    int n[2] = {0, 0};
    int xch = 0;                  // first zero slot: above every gate's pair slots, a multiple of 16
    std::vector<int> tab[2];      // per bond: offset of its spin-s code table
    size_t b0_pos = 0;            // position of |b0> in layout A
    bool general = false;         // eps or V terms in the diagonal
    double U = 0.0;
    SecModel *d_model = nullptr;
    uint32_t *d_pat[2] = {nullptr, nullptr};
    double *d_base[2] = {nullptr, nullptr};
    uint16_t *d_code = nullptr;
    ~Tables()
    {
        (void)hipFree(d_model);
        for (int s = 0; s < 2; ++s) {
            (void)hipFree(d_pat[s]);
            (void)hipFree(d_base[s]);
        }
        (void)hipFree(d_code);
    }
};

struct Program {
    std::vector<RowPass> fwd;
    int final_col = 0;
    SecOp *d_ops = nullptr;       // forward passes' ops, then H ops (X spin + D, Y spin)
    int n_ops = 0;                // all of them (the angle table's entries)
    int n_diag = 0;               // diagonal ops of the sweep (phase tables)
    std::vector<int> op_off;      // per forward pass
    int ham_x_off = 0, ham_x_n = 0, ham_y_off = 0, ham_y_n = 0;
    // reduction: partial rows 0, 1 = the two energy parts, then each reverse
    // pass's slots (forward order of passes)
    std::vector<int> red_row0;    // per forward pass: its chi2 rows, then its chi1 rows
    int n_rows = 0;
    int32_t *d_ptr = nullptr, *d_rows = nullptr, *d_nblk = nullptr;
    double *d_scale = nullptr;
    int n_out = 0;
    ~Program()
    {
        (void)hipFree(d_ops);
        (void)hipFree(d_nblk);
        (void)hipFree(d_ptr);
        (void)hipFree(d_rows);
        (void)hipFree(d_scale);
    }
};

struct Entry {
    std::unique_ptr<Tables> tab;
    std::map<int, std::unique_ptr<Program>> progs;   // by layer count
};

std::mutex g_mu;
std::map<std::pair<uint64_t, int>, Entry> g_cache;   // (handle uid, device)

hubbard_status fail(hubbard_status s, const std::string &m) { return set_error(s, m); }

hipError_t upload(void **dst, const void *src, size_t bytes)
{
    hipError_t e = hipMalloc(dst, std::max<size_t>(bytes, 16));
    if (e == hipSuccess && bytes)
        e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    return e;
}

int popc(uint32_t x) { return __builtin_popcount(x); }

// LDS slots of a gate's pairs, chosen so that the exchange's LDS accesses
// are free of bank conflicts.  Pair q takes the slots 2p and 2p + 1 for some
// p, in either order (an element reads its partner at its own slot XOR 1),
// and p and the order are free.  On this GPU a wave's 16-byte LDS write is
// served 8 lanes per cycle (32 banks of 4 bytes: slots equal modulo 8
// conflict) and a 16-byte read 16 lanes per cycle (64 banks: modulo 16).
// An element e (thread e mod kT, register e / kT) writes its slot s and reads
// s XOR 1, so a pair with lower slot residue r (mod 16) puts r (mod 8) into
// e1's write group, r ^ 1 (mod 8) into e2's, r ^ 1 into e1's read group and r
// into e2's.  Greedy over the pairs in rank order: the residue that adds no
// conflict (else the fewest), then the least used class p mod 8 (the slots
// stay dense).  Returns the slots used (2 + 2 max p).
int pair_slots(const std::vector<std::array<int, 2>> &prs, int rpt, std::vector<int> &slot)
{
    const int groups = rpt * kT / 8;
    std::vector<uint8_t> w8((size_t)groups, 0);        // write residues (mod 8) per 8 lanes
    std::vector<uint16_t> r16((size_t)groups / 2, 0);  // read residues (mod 16) per 16 lanes
    auto g8 = [](int e) { return (e / kT) * (kT / 8) + (e % kT) / 8; };
    int count[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int top = -1;
    slot.assign(2 * prs.size(), 0);
    for (size_t q = 0; q < prs.size(); ++q) {
        const int a8 = g8(prs[q][0]), b8 = g8(prs[q][1]), a16 = a8 / 2, b16 = b8 / 2;
        int best = 0, best_score = 1 << 30;
        for (int r = 0; r < 16; ++r) {
            const int r2 = r ^ 1;
            const int miss = ((w8[a8] >> (r & 7)) & 1) + ((w8[b8] >> (r2 & 7)) & 1) +
                             ((r16[a16] >> r2) & 1) + ((r16[b16] >> r) & 1);
            const int score = miss * (1 << 20) + count[r >> 1];
            if (score < best_score) {
                best_score = score;
                best = r;
            }
        }
        const int cls = best >> 1, p = cls + 8 * count[cls]++;
        top = std::max(top, p);
        slot[2 * q] = 2 * p + (best & 1);
        slot[2 * q + 1] = 2 * p + 1 - (best & 1);
        w8[a8] |= (uint8_t)(1u << (best & 7));
        w8[b8] |= (uint8_t)(1u << ((best ^ 1) & 7));
        r16[a16] |= (uint16_t)(1u << (best ^ 1));
        r16[b16] |= (uint16_t)(1u << best);
    }
    return 2 * top + 2;
}

// LDS of a row workgroup: the pair and zero slots, the reduction slots, the
// U-count phase table, the unit phases, one gate's code table (of the longer
// row).
size_t lds_bytes(const Tables &T)
{
    const int rp = std::max(rp_of(rpt_of(T.n[0])), rp_of(rpt_of(T.n[1])));
    return (size_t)(T.xch + kZero) * 16 + kMaxRed * kWaves * 8 + kDiagTab * 16 +
           (1u << kCisBits) * 16 + (size_t)kT * rp * 2;
}

hubbard_status build_tables(const Model &m, Tables &T)
{
    const int ns = m.ns;
    const uint32_t smask = ns >= 32 ? 0xffffffffu : ((1u << ns) - 1u);
    const int ne[2] = {popc((uint32_t)m.neel & smask), popc((uint32_t)(m.neel >> ns) & smask)};
    std::vector<uint32_t> pat[2];
    std::vector<double> base[2];
    std::vector<int32_t> rank_of[2];
    for (int s = 0; s < 2; ++s) {
        rank_of[s].assign((size_t)1 << ns, -1);
        for (uint32_t p = 0; p <= smask; ++p) {
            if (popc(p) != ne[s])
                continue;
            rank_of[s][p] = (int32_t)pat[s].size();
            pat[s].push_back(p);
            double b = 0.0;
            for (int i = 0; i < ns; ++i)
                if ((p >> i) & 1u)
                    b += m.eps[i];
            for (int k = 0; k < m.nb; ++k)
                if (((p >> m.bi[k]) & 1u) && ((p >> m.bj[k]) & 1u))
                    b += m.V[k];
            base[s].push_back(b);
            if (p == smask)
                break;
        }
        T.n[s] = (int)pat[s].size();
    }
    if (T.n[0] > kMaxRows || T.n[1] > kMaxRows)
        return fail(HUBBARD_ERR_ARG, "sector rows longer than 13 x 1024");
    const uint32_t up0 = (uint32_t)m.neel & smask, dn0 = (uint32_t)(m.neel >> ns) & smask;
    T.b0_pos = (size_t)rank_of[1][dn0] * T.n[0] + rank_of[0][up0];
    // per bond and spin: pair slots and the Jordan-Wigner sign of the sites
    // strictly between the bond's ends, at the rank's entry of the
    // register-tile layout; every other entry (the bond's inactive elements
    // and the tile's padding) names a zero slot
    struct Gate {
        std::vector<std::array<int, 2>> prs;   // (lower, upper) rank, in rank order
        std::vector<uint32_t> sgn;
        std::vector<int> slot;                 // per pair: lower's, upper's slot
    };
    std::vector<Gate> gates[2];
    int used = 2;
    for (int s = 0; s < 2; ++s) {
        const int R = rpt_of(T.n[s]);
        gates[s].resize(m.nb);
        for (int k = 0; k < m.nb; ++k) {
            const int i = std::min(m.bi[k], m.bj[k]), j = std::max(m.bi[k], m.bj[k]);
            const uint32_t mask = (1u << i) | (1u << j);
            const uint32_t between = ((1u << j) - 1u) & ~((2u << i) - 1u);
            Gate &G = gates[s][k];
            for (int r = 0; r < T.n[s]; ++r) {
                const uint32_t p = pat[s][r];
                if (((p >> i) ^ (p >> j)) & 1u) {
                    const int r2 = rank_of[s][p ^ mask];
                    if (r2 > r) {
                        G.prs.push_back({r, r2});
                        G.sgn.push_back((uint32_t)(popc(p & between) & 1) << 15);
                    }
                }
            }
            used = std::max(used, pair_slots(G.prs, R, G.slot));
        }
    }
    T.xch = (used + 15) & ~15;
    if (T.xch + kZero > 0x7FFF || lds_bytes(T) > 160 * 1024)
        return fail(HUBBARD_ERR_ARG, "sector gate pairs do not fit the workgroup's LDS");
    std::vector<uint16_t> codes;
    for (int s = 0; s < 2; ++s) {
        T.tab[s].assign(m.nb, 0);
        const int R = rpt_of(T.n[s]);
        auto entry = [&](int r) { return (size_t)code_index(R, r % kT, r / kT); };
        for (int k = 0; k < m.nb; ++k) {
            const Gate &G = gates[s][k];
            T.tab[s][k] = (int)codes.size();
            const size_t at = codes.size();
            codes.resize(at + (size_t)kT * rp_of(R), (uint16_t)T.xch);
            std::vector<int> slot((size_t)R * kT, -1);   // per element (rank)
            for (size_t q = 0; q < G.prs.size(); ++q)
                for (int h = 0; h < 2; ++h) {
                    slot[G.prs[q][h]] = G.slot[2 * q + h];
                    codes[at + entry(G.prs[q][h])] = (uint16_t)(G.slot[2 * q + h] | G.sgn[q]);
                }
            // per group of 16 threads and register (the lanes one cycle of a
            // 16-byte LDS read serves): the zero slot its inactive elements
            // read, one per half of the group, in a bank group (slot mod 16)
            // that the group's other reads leave free
            for (int e0 = 0; e0 < R * kT; e0 += 16) {
                uint32_t taken = 0, u8[2] = {0, 0};
                for (int e = e0; e < e0 + 16; ++e)
                    if (slot[e] >= 0) {
                        const int q = (slot[e] ^ 1) & 15;
                        taken |= 1u << q;
                        u8[(e - e0) / 8] |= 1u << (q & 7);
                    }
                for (int h = 0; h < 2; ++h) {
                    int best = 0, best_miss = 1 << 30;
                    for (int q = 0; q < 16; ++q) {
                        const int miss = 4 * ((taken >> q) & 1) + ((u8[h] >> (q & 7)) & 1);
                        if (miss < best_miss) {
                            best_miss = miss;
                            best = q;
                        }
                    }
                    taken |= 1u << best;
                    // read slot T.xch + best (T.xch is a multiple of 16)
                    for (int e = e0 + 8 * h; e < e0 + 8 * h + 8; ++e)
                        if (slot[e] < 0)
                            codes[at + entry(e)] = (uint16_t)((T.xch + best) ^ 1);
                }
            }
        }
    }
    T.general = m.general;
    T.U = m.U;
    SecModel sm;
    std::memset(&sm, 0, sizeof(sm));
    sm.ns = ns;
    sm.U = m.U;
    sm.n[0] = T.n[0];
    sm.n[1] = T.n[1];
    for (int k = 0; k < m.nb; ++k)
        if (m.V[k] != 0.0) {
            sm.vi[sm.nvb] = m.bi[k];
            sm.vj[sm.nvb] = m.bj[k];
            sm.vV[sm.nvb] = m.V[k];
            ++sm.nvb;
        }
    hipError_t e = hipSuccess;
    for (int s = 0; s < 2 && e == hipSuccess; ++s) {
        e = upload((void **)&T.d_pat[s], pat[s].data(), pat[s].size() * 4);
        if (e == hipSuccess)
            e = upload((void **)&T.d_base[s], base[s].data(), base[s].size() * 8);
        sm.pat[s] = T.d_pat[s];
        sm.base[s] = T.d_base[s];
    }
    if (e == hipSuccess)
        e = upload((void **)&T.d_code, codes.data(), codes.size() * 2);
    sm.code = T.d_code;
    if (e == hipSuccess)
        e = upload((void **)&T.d_model, &sm, sizeof(sm));
    if (e != hipSuccess)
        return fail(HUBBARD_ERR_DEVICE, std::string("uploading sector tables: ") +
                                            hipGetErrorString(e));
    return HUBBARD_OK;
}

// Each op's nxt links: the next HOP op of the list in forward and in reverse
// order, wrapping around (-1: the list has none).
void link_hops(std::vector<SecOp> &v)
{
    const int n = (int)v.size();
    for (int i = 0; i < n; ++i) {
        v[i].nxt[0] = v[i].nxt[1] = -1;
        for (int k = 1; k <= n && v[i].nxt[0] < 0; ++k)
            if (v[(i + k) % n].kind == SOP_HOP)
                v[i].nxt[0] = (i + k) % n;
        for (int k = 1; k <= n && v[i].nxt[1] < 0; ++k)
            if (v[(i - k + n) % n].kind == SOP_HOP)
                v[i].nxt[1] = (i - k + n) % n;
    }
}

void add_red(RowPass &p, SecOp &o)
{
    for (size_t s = 0; s < p.red_param.size(); ++s)
        if (p.red_param[s] == o.param) {
            o.red = (int)s;
            return;
        }
    o.red = (int)p.red_param.size();
    p.red_param.push_back(o.param);
}

hubbard_status build_program(const Model &m, const Tables &T, int layers, Program &P)
{
    const int per = m.params_per_layer();
    auto hops = [&](int l, int spin, RowPass &p) {
        for (int s = 1; s < per; ++s)
            for (int k = 0; k < m.nb; ++k)
                if (m.slot[k] == s) {
                    SecOp o;
                    std::memset(&o, 0, sizeof(o));
                    o.kind = SOP_HOP;
                    o.param = l * per + s;
                    o.tab = T.tab[spin][k];
                    o.t = m.t[k];
                    add_red(p, o);
                    p.ops.push_back(o);
                }
    };
    int n_diag = 0;
    auto diag = [&](int l, RowPass &p) {
        SecOp o;
        std::memset(&o, 0, sizeof(o));
        o.kind = SOP_DIAG;
        o.param = l * per;
        o.tab = n_diag++;   // its phase table
        add_red(p, o);
        p.ops.push_back(o);
    };
    P.fwd.clear();
    if (layers > 0) {
        RowPass cur;
        cur.col = 0;
        for (int l = 0; l < layers; ++l) {
            diag(l, cur);
            hops(l, cur.col, cur);
            RowPass nxt;
            nxt.col = 1 - cur.col;
            hops(l, nxt.col, nxt);
            P.fwd.push_back(cur);
            cur = nxt;
        }
        P.fwd.push_back(cur);
    }
    for (RowPass &p : P.fwd) {
        if ((int)p.red_param.size() > kMaxRed)
            return fail(HUBBARD_ERR_ARG, "sector row pass with more than 16 parameters");
        if (std::count_if(p.ops.begin(), p.ops.end(),
                          [](const SecOp &o) { return o.kind == SOP_DIAG; }) > 1)
            return fail(HUBBARD_ERR_ARG, "sector row pass with two diagonal ops");
        link_hops(p.ops);
    }
    P.final_col = P.fwd.empty() ? 0 : P.fwd.back().col;
    P.n_diag = n_diag;
    // H: the final layout's spin hops and D, then the other spin's hops
    std::vector<SecOp> all;
    for (const RowPass &p : P.fwd) {
        P.op_off.push_back((int)all.size());
        all.insert(all.end(), p.ops.begin(), p.ops.end());
    }
    auto ham_ops = [&](int spin, bool with_d) {
        std::vector<SecOp> v;
        if (with_d) {
            SecOp o;
            std::memset(&o, 0, sizeof(o));
            o.kind = SOP_DIAG;
            o.param = -1;
            o.tab = -1;
            v.push_back(o);
        }
        for (int k = 0; k < m.nb; ++k) {
            SecOp o;
            std::memset(&o, 0, sizeof(o));
            o.kind = SOP_HOP;
            o.param = -1;
            o.tab = T.tab[spin][k];
            o.t = m.t[k];
            v.push_back(o);
        }
        return v;
    };
    std::vector<SecOp> hx = ham_ops(P.final_col, true), hy = ham_ops(1 - P.final_col, false);
    link_hops(hx);
    link_hops(hy);
    P.ham_x_off = (int)all.size();
    P.ham_x_n = (int)hx.size();
    all.insert(all.end(), hx.begin(), hx.end());
    P.ham_y_off = (int)all.size();
    P.ham_y_n = (int)hy.size();
    all.insert(all.end(), hy.begin(), hy.end());
    // reduction rows, and the workgroups of the pass that writes each
    auto grid_of = [&](int col) { return std::min(T.n[1 - col], kGrid); };
    P.n_rows = 2;
    std::vector<int32_t> nblk{grid_of(P.final_col), grid_of(1 - P.final_col)};
    std::vector<std::vector<int>> rows_of(1 + layers * per);
    rows_of[0] = {0, 1};
    for (const RowPass &p : P.fwd) {
        P.red_row0.push_back(P.n_rows);
        for (int half = 0; half < 2; ++half) {   // chi2, then chi1 (stored negated)
            for (size_t s = 0; s < p.red_param.size(); ++s) {
                rows_of[1 + p.red_param[s]].push_back(P.n_rows + (int)s);
                nblk.push_back(grid_of(p.col));
            }
            P.n_rows += (int)p.red_param.size();
        }
    }
    std::vector<int32_t> ptr{0}, rows;
    std::vector<double> scale;
    for (size_t o = 0; o < rows_of.size(); ++o) {
        rows.insert(rows.end(), rows_of[o].begin(), rows_of[o].end());
        ptr.push_back((int32_t)rows.size());
        // dE/dth_k = 2 Im <lambda_k|G_k|psi_k> = (<chi2|G_k|chi2> - <chi1|G_k|chi1>) / 2
        scale.push_back(o == 0 ? 1.0 : 0.5);
    }
    P.n_out = (int)rows_of.size();
    P.n_ops = (int)all.size();
    hipError_t e = upload((void **)&P.d_ops, all.data(), all.size() * sizeof(SecOp));
    if (e == hipSuccess)
        e = upload((void **)&P.d_ptr, ptr.data(), ptr.size() * 4);
    if (e == hipSuccess)
        e = upload((void **)&P.d_rows, rows.data(), rows.size() * 4);
    if (e == hipSuccess)
        e = upload((void **)&P.d_scale, scale.data(), scale.size() * 8);
    if (e == hipSuccess)
        e = upload((void **)&P.d_nblk, nblk.data(), nblk.size() * 4);
    if (e != hipSuccess)
        return fail(HUBBARD_ERR_DEVICE, std::string("uploading the sector program: ") +
                                            hipGetErrorString(e));
    return HUBBARD_OK;
}

// Tables and (layers >= 0) the program of a handle on the current device.
hubbard_status get(hubbard_t h, int layers, Tables **T, Program **P)
{
    const Model *m = handle_model(h);
    if (!m)
        return fail(HUBBARD_ERR_ARG, "null handle");
    if (m->ansatz != 0)
        return fail(HUBBARD_ERR_STATE, "the sector form needs the HVA circuit (the NP "
                                       "ansatz's on-site gates change N_up and N_dn)");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return fail(HUBBARD_ERR_DEVICE, "hipGetDevice failed");
    std::lock_guard<std::mutex> lk(g_mu);
    Entry &en = g_cache[std::make_pair(handle_uid(h), dev)];
    if (!en.tab) {
        std::unique_ptr<Tables> t(new Tables());
        hubbard_status st = build_tables(*m, *t);
        if (st != HUBBARD_OK)
            return st;
        en.tab = std::move(t);
    }
    *T = en.tab.get();
    if (P) {
        auto it = en.progs.find(layers);
        if (it == en.progs.end()) {
            std::unique_ptr<Program> p(new Program());
            hubbard_status st = build_program(*m, *en.tab, layers, *p);
            if (st != HUBBARD_OK)
                return st;
            it = en.progs.emplace(layers, std::move(p)).first;
        }
        *P = it->second.get();
    }
    return HUBBARD_OK;
}

size_t vec_elems(const Tables &T) { return (size_t)T.n[0] * (size_t)T.n[1]; }
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workgroup shape by row length: 1024 threads holding up to 13 elements of
// each vector.  (At 13 elements, H -- two vectors -- and the general
// diagonal's gate passes keep part of their tiles in scratch memory, about
// 100 bytes per thread; 512 threads playing two tile threads each spilled
// more.)
template <int MODE, bool GEN>
void launch_rows_g(const Tables &T, const SecOp *ops, int n_ops, int col, int n_red,
                   const double2 *ang, const double2 *dph, double2 *v0, double2 *v1,
                   double *partial, int row0, int flags, hipStream_t s)
{
    const int nr = T.n[1 - col], n = T.n[col];
    const int grid = std::min(nr, kGrid);
    const size_t lds = lds_bytes(T);
#define HV_SEC(TT, R)                                                                           \
    hipLaunchKernelGGL((k_sec_rows<MODE, TT, R, GEN>), dim3(grid), dim3(TT), lds, s, ops,       \
                       n_ops, col, n_red, ang, dph, T.d_model, v0, v1, partial, row0, kGrid,    \
                       flags, T.xch)
    switch (rpt_of(n)) {   // the register tile the code tables are laid out for
    case 1: HV_SEC(kT, 1); break;
    case 2: HV_SEC(kT, 2); break;
    case 4: HV_SEC(kT, 4); break;
    case 8: HV_SEC(kT, 8); break;
    default: HV_SEC(kT, 13); break;
    }
#undef HV_SEC
}

template <int MODE>
void launch_rows(const Tables &T, const SecOp *ops, int n_ops, int col, int n_red,
                 const double2 *ang, const double2 *dph, double2 *v0, double2 *v1,
                 double *partial, int row0, int flags, hipStream_t s)
{
    if (T.general)
        launch_rows_g<MODE, true>(T, ops, n_ops, col, n_red, ang, dph, v0, v1, partial, row0,
                                  flags, s);
    else
        launch_rows_g<MODE, false>(T, ops, n_ops, col, n_red, ang, dph, v0, v1, partial, row0,
                                   flags, s);
}

void transpose(const Tables &T, int from_col, const double2 *in, double2 *out, bool add,
               hipStream_t s)
{
    const int nr = T.n[1 - from_col], nc = T.n[from_col];
    hipLaunchKernelGGL(k_sec_transpose, dim3((nc + kTrTile - 1) / kTrTile, (nr + kTrTile - 1) / kTrTile),
                       dim3(kTrThreads), 0, s, in, out, nr, nc, add ? 1 : 0);
}

void set_attrs()
{
    static std::once_flag once;
    std::call_once(once, [] {
        const void *fns[] = {
#define HV_SEC_FNS(MODE, GEN)                                                                   \
    (const void *)k_sec_rows<MODE, kT, 1, GEN>, (const void *)k_sec_rows<MODE, kT, 2, GEN>,     \
        (const void *)k_sec_rows<MODE, kT, 4, GEN>, (const void *)k_sec_rows<MODE, kT, 8, GEN>, \
        (const void *)k_sec_rows<MODE, kT, 13, GEN>
            HV_SEC_FNS(S_FWD, false), HV_SEC_FNS(S_REV, false), HV_SEC_FNS(S_HAM, false),
            HV_SEC_FNS(S_FWD, true), HV_SEC_FNS(S_REV, true), HV_SEC_FNS(S_HAM, true)};
#undef HV_SEC_FNS
        for (const void *f : fns)
            (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    });
}

double2 *dph_of(const Program &P, double2 *ang)
{
    return (double2 *)((char *)ang + align256((size_t)P.n_ops * 16));
}

// Angles of every op, then the diagonal phase tables.
size_t ang_bytes(const Program &P)
{
    return align256((size_t)P.n_ops * 16) + align256((size_t)P.n_diag * kDiagTab * 16);
}

// ang[i] for every op of the program and dph (see k_sec_angles); dph follows ang.
void angles(const Tables &T, const Program &P, const double *theta, double2 *ang, hipStream_t s)
{
    const int blocks = std::max(1, std::min(64, (P.n_ops + 255) / 256));
    hipLaunchKernelGGL(k_sec_angles, dim3(blocks), dim3(256), 0, s, P.d_ops, P.n_ops, theta, T.U,
                       ang, dph_of(P, ang));
}

// Forward sweep: psi starts in layout A in `a`; `b` is the layout-B buffer.
// Returns the buffer holding the result (in layout P.final_col).
double2 *forward(const Tables &T, const Program &P, const double2 *ang, double2 *a, double2 *b,
                 hipStream_t s)
{
    double2 *cur = a;
    int col = 0;
    for (size_t i = 0; i < P.fwd.size(); ++i) {
        const RowPass &p = P.fwd[i];
        if (p.col != col) {
            double2 *dst = (cur == a) ? b : a;
            transpose(T, col, cur, dst, false, s);
            cur = dst;
            col = p.col;
        }
        launch_rows<S_FWD>(T, P.d_ops + P.op_off[i], (int)p.ops.size(), p.col, 0,
                           ang + P.op_off[i], dph_of(P, (double2 *)ang), cur, nullptr, nullptr,
                           0, 0, s);
    }
    return cur;
}

// phi_x <- H psi_x for psi_x in layout `col` (x): the col-spin hops and D in
// layout x, the other spin's hops in the transposed layout; psi_y, phi_y are
// scratch of the other layout.  Energy parts to partial rows 0 and 1.
void hamiltonian(const Tables &T, const Program &P, int col, const double2 *psi_x,
                 double2 *phi_x, double2 *psi_y, double2 *phi_y, double *partial, hipStream_t s,
                 const SecOp *ops_x, int n_x, const SecOp *ops_y, int n_y)
{
    launch_rows<S_HAM>(T, ops_x, n_x, col, 1, nullptr, nullptr, (double2 *)psi_x, phi_x,
                       partial, 0, 0, s);
    transpose(T, col, psi_x, psi_y, false, s);
    launch_rows<S_HAM>(T, ops_y, n_y, 1 - col, 1, nullptr, nullptr, psi_y, phi_y, partial, 1, 0,
                       s);
    transpose(T, 1 - col, phi_y, phi_x, true, s);
}

// out <- H in for sector vectors in layout A (the 0-layer program's H ops:
// up hops and D in layout A, down hops in layout B through in_b, out_b).
void apply_h(const Tables &T, const Program &P, const double2 *in, double2 *out, double2 *in_b,
             double2 *out_b, hipStream_t s)
{
    launch_rows<S_HAM>(T, P.d_ops + P.ham_x_off, P.ham_x_n, 0, 0, nullptr, nullptr,
                       (double2 *)in, out, nullptr, 0, 0, s);
    transpose(T, 0, in, in_b, false, s);
    launch_rows<S_HAM>(T, P.d_ops + P.ham_y_off, P.ham_y_n, 1, 0, nullptr, nullptr, in_b, out_b,
                       nullptr, 0, 0, s);
    transpose(T, 1, out_b, out, true, s);
}

hubbard_status check(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(HUBBARD_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return HUBBARD_OK;
}

}  // namespace sec

// Drop the sector tables and programs of a destroyed handle.
void sector_forget(uint64_t uid)
{
    std::lock_guard<std::mutex> lk(sec::g_mu);
    for (auto it = sec::g_cache.begin(); it != sec::g_cache.end();)
        it = it->first.first == uid ? sec::g_cache.erase(it) : std::next(it);
}

}  // namespace hv

using namespace hv;
using namespace hv::sec;

hubbard_status hubbard_sector_dim(hubbard_t h, int64_t *n_up, int64_t *n_dn)
{
    Tables *T = nullptr;
    hubbard_status st = get(h, -1, &T, nullptr);
    if (st != HUBBARD_OK)
        return st;
    if (n_up)
        *n_up = T->n[0];
    if (n_dn)
        *n_dn = T->n[1];
    return HUBBARD_OK;
}

hubbard_status hubbard_sector_workspace_size(hubbard_t h, int32_t n_layers, int32_t op,
                                             size_t *bytes)
{
    if (!bytes || n_layers < 0 || op < HUBBARD_SECTOR_ANSATZ || op > HUBBARD_SECTOR_LANCZOS)
        return set_error(HUBBARD_ERR_ARG, "bad arguments to hubbard_sector_workspace_size");
    Tables *T = nullptr;
    Program *P = nullptr;
    const bool h_only = op == HUBBARD_SECTOR_HAMILTONIAN || op == HUBBARD_SECTOR_LANCZOS;
    hubbard_status st = get(h, h_only ? 0 : n_layers, &T, &P);
    if (st != HUBBARD_OK)
        return st;
    const size_t v = align256(vec_elems(*T) * 16);
    if (op == HUBBARD_SECTOR_ANSATZ)
        *bytes = v + ang_bytes(*P);
    else if (op == HUBBARD_SECTOR_HAMILTONIAN)
        *bytes = 2 * v;
    else if (op == HUBBARD_SECTOR_LANCZOS)
        *bytes = 5 * v + lanczos_partial_bytes();
    else
        *bytes = 4 * v + align256((size_t)P->n_rows * kGrid * 8) + ang_bytes(*P);
    return HUBBARD_OK;
}

hubbard_status hubbard_sector_init_neel(hubbard_t h, void *psi_dev, void *stream)
{
    Tables *T = nullptr;
    hubbard_status st = get(h, -1, &T, nullptr);
    if (st != HUBBARD_OK)
        return st;
    if (!psi_dev)
        return set_error(HUBBARD_ERR_ARG, "null vector");
    hipLaunchKernelGGL(k_sec_basis, dim3(2048), dim3(256), 0, (hipStream_t)stream,
                       (double2 *)psi_dev, vec_elems(*T), T->b0_pos);
    return check("sector init");
}

hubbard_status sector_ansatz_apply(hubbard_t h, const double *theta_dev, int32_t n_layers,
                                   void *psi_dev, void *ws_dev, size_t ws_bytes, void *stream)
{
    if (n_layers < 0 || !psi_dev || (n_layers > 0 && !theta_dev))
        return set_error(HUBBARD_ERR_ARG, "bad arguments to sector_ansatz_apply");
    Tables *T = nullptr;
    Program *P = nullptr;
    hubbard_status st = get(h, n_layers, &T, &P);
    if (st != HUBBARD_OK)
        return st;
    const size_t v = align256(vec_elems(*T) * 16);
    if (!ws_dev || ws_bytes < v + ang_bytes(*P))
        return set_error(HUBBARD_ERR_SIZE, "workspace too small for sector_ansatz_apply");
    set_attrs();
    hipStream_t s = (hipStream_t)stream;
    double2 *ang = (double2 *)((char *)ws_dev + v);
    if (n_layers > 0)
        angles(*T, *P, theta_dev, ang, s);
    double2 *out = forward(*T, *P, ang, (double2 *)psi_dev, (double2 *)ws_dev, s);
    if (out != (double2 *)psi_dev)   // ended in layout B
        transpose(*T, 1, out, (double2 *)psi_dev, false, s);
    return check("sector ansatz");
}

hubbard_status sector_hamiltonian_apply(hubbard_t h, const void *psi_dev, void *out_dev,
                                        void *ws_dev, size_t ws_bytes, void *stream)
{
    if (!psi_dev || !out_dev || psi_dev == out_dev)
        return set_error(HUBBARD_ERR_ARG, "sector_hamiltonian_apply needs distinct vectors");
    Tables *T = nullptr;
    Program *P = nullptr;
    hubbard_status st = get(h, 0, &T, &P);
    if (st != HUBBARD_OK)
        return st;
    const size_t v = align256(vec_elems(*T) * 16);
    if (!ws_dev || ws_bytes < 2 * v)
        return set_error(HUBBARD_ERR_SIZE, "workspace too small for sector_hamiltonian_apply");
    set_attrs();
    char *w = (char *)ws_dev;
    apply_h(*T, *P, (const double2 *)psi_dev, (double2 *)out_dev, (double2 *)w,
            (double2 *)(w + v), (hipStream_t)stream);
    return check("sector H");
}

hubbard_status hubbard_sector_lanczos(hubbard_t h, const void *start_dev, int32_t max_iter,
                                      double tol, double *E0, int32_t *iters, double *residual,
                                      void *gs_dev, void *ws_dev, size_t ws_bytes, void *stream)
{
    if (!start_dev || max_iter < 1 || !(tol > 0.0) || !E0 || !ws_dev)
        return set_error(HUBBARD_ERR_ARG, "bad arguments to hubbard_sector_lanczos");
    Tables *T = nullptr;
    Program *P = nullptr;
    hubbard_status st = get(h, 0, &T, &P);
    if (st != HUBBARD_OK)
        return st;
    const size_t n = vec_elems(*T), v = align256(n * 16);
    const size_t need = 5 * v + lanczos_partial_bytes();
    if (ws_bytes < need)
        return set_error(HUBBARD_ERR_SIZE, "workspace too small for hubbard_sector_lanczos");
    const char *ws = (const char *)ws_dev;
    for (const void *p : {start_dev, (const void *)gs_dev}) {
        const char *q = (const char *)p;
        if (q && q < ws + need && ws < q + n * 16)
            return set_error(HUBBARD_ERR_ARG, "start or state vector overlaps the workspace");
    }
    set_attrs();
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws_dev;
    double2 *buf[3] = {(double2 *)w, (double2 *)(w + v), (double2 *)(w + 2 * v)};
    double2 *in_b = (double2 *)(w + 3 * v), *out_b = (double2 *)(w + 4 * v);
    const ApplyH apply = [&](const double2 *in, double2 *out) {
        apply_h(*T, *P, in, out, in_b, out_b, s);
        return check("sector H");
    };
    return lanczos_run(apply, n, (const double2 *)start_dev, max_iter, tol, E0, iters, residual,
                       (double2 *)gs_dev, buf, (double2 *)(w + 5 * v), s);
}

hubbard_status sector_energy_grad(hubbard_t h, const double *theta_dev, int32_t n_layers,
                                  double *E_dev, double *grad_dev, void *ws_dev, size_t ws_bytes,
                                  void *stream)
{
    if (n_layers < 0 || !E_dev || (n_layers > 0 && (!theta_dev || !grad_dev)))
        return set_error(HUBBARD_ERR_ARG, "bad arguments to sector_energy_grad");
    Tables *T = nullptr;
    Program *P = nullptr;
    hubbard_status st = get(h, n_layers, &T, &P);
    if (st != HUBBARD_OK)
        return st;
    const size_t v = align256(vec_elems(*T) * 16);
    const size_t pbytes = align256((size_t)P->n_rows * kGrid * 8);
    if (!ws_dev || ws_bytes < 4 * v + pbytes + ang_bytes(*P))
        return set_error(HUBBARD_ERR_SIZE, "workspace too small for sector_energy_grad");
    set_attrs();
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws_dev;
    double2 *psi[2] = {(double2 *)w, (double2 *)(w + v)};
    double2 *lam[2] = {(double2 *)(w + 2 * v), (double2 *)(w + 3 * v)};
    double *partial = (double *)(w + 4 * v);
    double2 *ang = (double2 *)(w + 4 * v + pbytes);
    if (n_layers > 0)
        angles(*T, *P, theta_dev, ang, s);
    hipLaunchKernelGGL(k_sec_basis, dim3(2048), dim3(256), 0, s, psi[0], vec_elems(*T),
                       T->b0_pos);
    double2 *end = forward(*T, *P, ang, psi[0], psi[1], s);
    int col = P->final_col;
    if (end != psi[col]) {   // cannot happen: layout A lives in psi[0], B in psi[1]
        return set_error(HUBBARD_ERR_STATE, "sector forward ended in the wrong buffer");
    }
    // lambda = H psi in the final layout; the partial rows 0 and 1 get E
    hamiltonian(*T, *P, col, psi[col], lam[col], psi[1 - col], lam[1 - col], partial, s,
                P->d_ops + P->ham_x_off, P->ham_x_n, P->d_ops + P->ham_y_off, P->ham_y_n);
    // reverse sweep on chi1 = lambda + i psi (psi's buffers) and chi2 =
    // lambda - i psi (lambda's): brackets from their expectations
    if (!P->fwd.empty())
        hipLaunchKernelGGL(k_sec_mix, dim3(2048), dim3(256), 0, s, psi[col], lam[col],
                           vec_elems(*T));
    for (int i = (int)P->fwd.size() - 1; i >= 0; --i) {
        const RowPass &p = P->fwd[i];
        if (p.col != col) {
            transpose(*T, col, psi[col], psi[p.col], false, s);
            transpose(*T, col, lam[col], lam[p.col], false, s);
            col = p.col;
        }
        const int nred = (int)p.red_param.size(), last = i == 0 ? SF_NO_STORE : 0;
        launch_rows<S_REV>(*T, P->d_ops + P->op_off[i], (int)p.ops.size(), p.col, nred,
                           ang + P->op_off[i], dph_of(*P, ang), lam[col], nullptr, partial,
                           P->red_row0[i], last, s);
        launch_rows<S_REV>(*T, P->d_ops + P->op_off[i], (int)p.ops.size(), p.col, nred,
                           ang + P->op_off[i], dph_of(*P, ang), psi[col], nullptr, partial,
                           P->red_row0[i] + nred, last | SF_NEGATE, s);
    }
    hipLaunchKernelGGL(k_sec_reduce, dim3(P->n_out), dim3(256), 0, s, partial, kGrid,
                       P->d_nblk, P->d_ptr, P->d_rows, P->d_scale, E_dev, grad_dev);
    return check("sector energy_grad");
}
