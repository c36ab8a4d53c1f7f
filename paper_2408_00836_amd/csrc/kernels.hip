// kernels.hip -- gfx950 kernels of the Hubbard state-vector engine.
//
// Every kernel streams the complex128 state vector through LDS in tiles of
// 2^k amplitudes.  The tile's index bits are the pass's chosen qubits; the
// other n-k bits (the tile id) are spread over the grid with a grid-stride
// loop.  Tile bits 0..c-1 are the low c bits of the amplitude index, so every
// global access is a run of 2^c contiguous 16-byte amplitudes.
//
// Operations (see hubvqe.hpp):
//   OP_HOP   exp(-i th (-t)(a+_p a_q + h.c.)) on the pairs x <-> x^(2^p+2^q)
//            with exactly one of p, q occupied.  On such a pair the term is
//            s * [[0,1],[1,0]] with the Jordan-Wigner sign
//            s = (-1)^popcount(x & between(p,q)), so the gate is the rotation
//            (cos(th t), i s sin(th t)) -- no other amplitude changes.
//   OP_DIAG  exp(-i th D_sub) with D_sub = U * #{doubly occupied sites in the
//            op's set} + sum eps over its qubits + sum V_b n_i n_j over its bonds.
// No MFMA: nothing here is a dense contraction; the bound is HBM bandwidth.
#include <hip/hip_runtime.h>

#include "hubvqe.hpp"

namespace hv {

__device__ __forceinline__ uint32_t insert_zero(uint32_t x, int pos)
{
    uint32_t lo = x & ((1u << pos) - 1u);
    return ((x >> pos) << (pos + 1)) | lo;
}

// Global index bits contributed by the tile id (deposit over the free bits).
__device__ __forceinline__ uint32_t tile_base(uint64_t tile, const DevPass &P)
{
    uint32_t g = 0;
    for (int f = 0; f < P.nfree; ++f)
        g |= (uint32_t)((tile >> f) & 1u) << P.free_pos[f];
    return g;
}

// Diagonal sub-term value D_sub(g) for the general model.
__device__ __forceinline__ double diag_value(const DevOp &op, uint32_t g, const DevModel *M,
                                             const DevVBond *vb)
{
    uint32_t up = g & op.umask;
    uint32_t dn = (uint32_t)((uint64_t)g >> M->ns) & op.umask;
    double d = M->U * (double)__popc(up & dn);
    if (M->general) {
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

// Per-WG set-up shared by all pass kernels: tile offset table, per-op
// rotation coefficients and (U-count models) diagonal phase tables.
// sign = +1 applies the gates, -1 un-applies them.
__device__ void pass_setup(const DevPass &P, const DevOp *ops, const double *theta,
                           const DevModel *M, double sign, char *smem, const SmemPlan &sp)
{
    const int T = blockDim.x, tid = threadIdx.x;
    uint32_t *offs = (uint32_t *)(smem + sp.offs);
    double2 *opc = (double2 *)(smem + sp.opc);
    double2 *dtab = (double2 *)(smem + sp.dtab);
    const int nhi = P.k - P.c;
    for (int i = tid; i < (1 << nhi); i += T) {
        uint32_t o = 0;
        for (int j = 0; j < nhi; ++j)
            if ((i >> j) & 1)
                o |= 1u << P.tile_pos[P.c + j];
        offs[i] = o;
    }
    for (int o = tid; o < P.n_ops; o += T) {
        const DevOp op = ops[P.op_begin + o];
        if (op.kind == OP_HOP && op.param >= 0) {
            double s, c;
            sincos(theta[op.param] * op.t, &s, &c);
            opc[o] = make_double2(c, sign * s);
        }
    }
    if (!M->general) {
        for (int o = 0; o < P.n_ops; ++o) {
            const DevOp op = ops[P.op_begin + o];
            if (op.kind != OP_DIAG || op.param < 0)
                continue;
            for (int mcount = tid; mcount < kDiagTab; mcount += T) {
                double s, c;
                sincos(theta[op.param] * (M->U * (double)mcount), &s, &c);
                dtab[op.dtab * kDiagTab + mcount] = make_double2(c, -sign * s);
            }
        }
    }
}

// exp(-i sign th D_sub) for amplitude index g.
__device__ __forceinline__ double2 diag_phase(const DevOp &op, uint32_t g, const DevModel *M,
                                              const DevVBond *vb, const double *theta,
                                              double sign, const double2 *dtab)
{
    if (!M->general) {
        uint32_t up = g & op.umask;
        uint32_t dn = (uint32_t)((uint64_t)g >> M->ns) & op.umask;
        return dtab[op.dtab * kDiagTab + __popc(up & dn)];
    }
    double s, c;
    sincos(theta[op.param] * diag_value(op, g, M, vb), &s, &c);
    return make_double2(c, -sign * s);
}

// ------------------------------------------------------------ forward pass --

__global__ void __launch_bounds__(256)
k_forward(DevPass P, const DevOp *__restrict__ ops, const DevVBond *__restrict__ vb,
          const double *__restrict__ theta, const DevModel *__restrict__ M,
          double2 *__restrict__ psi)
{
    extern __shared__ __align__(16) char smem[];
    const int T = blockDim.x, tid = threadIdx.x;
    const SmemPlan sp = smem_plan(P.k, P.c, 1, P.n_ops, P.n_diag, 0, T);
    double2 *tile = (double2 *)(smem + sp.tiles);
    const uint32_t *offs = (const uint32_t *)(smem + sp.offs);
    const double2 *opc = (const double2 *)(smem + sp.opc);
    const double2 *dtab = (const double2 *)(smem + sp.dtab);
    pass_setup(P, ops, theta, M, 1.0, smem, sp);
    __syncthreads();

    const int k = P.k, c = P.c;
    const uint32_t cmask = (1u << c) - 1u;
    const uint32_t tsize = 1u << k;
    const uint64_t ntiles = (uint64_t)1 << P.nfree;
    for (uint64_t tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        const uint32_t base = tile_base(tl, P);
        for (uint32_t l = tid; l < tsize; l += T)
            tile[l] = psi[(uint64_t)(base | offs[l >> c] | (l & cmask))];
        __syncthreads();
        for (int o = 0; o < P.n_ops; ++o) {
            const DevOp op = ops[P.op_begin + o];
            if (op.kind == OP_DIAG) {
                for (uint32_t l = tid; l < tsize; l += T) {
                    uint32_t g = base | offs[l >> c] | (l & cmask);
                    tile[l] = cmul(tile[l], diag_phase(op, g, M, vb, theta, 1.0, dtab));
                }
            } else {
                const double cs = opc[o].x, sn = opc[o].y;
                const uint32_t par0 = __popc((uint32_t)tl & op.bm_free) & 1u;
                const int lo = min(op.pl, op.ql), hi = max(op.pl, op.ql);
                const uint32_t flip = (1u << op.pl) | (1u << op.ql);
                for (uint32_t j = tid; j < (tsize >> 2); j += T) {
                    uint32_t x = insert_zero(insert_zero(j, lo), hi) | (1u << op.pl);
                    uint32_t y = x ^ flip;
                    uint32_t par = (__popc(x & op.bm_local) + par0) & 1u;
                    double ss = par ? -sn : sn;
                    double2 a = tile[x], b = tile[y];
                    tile[x] = make_double2(cs * a.x - ss * b.y, cs * a.y + ss * b.x);
                    tile[y] = make_double2(cs * b.x - ss * a.y, cs * b.y + ss * a.x);
                }
            }
            __syncthreads();
        }
        for (uint32_t l = tid; l < tsize; l += T)
            psi[(uint64_t)(base | offs[l >> c] | (l & cmask))] = tile[l];
        __syncthreads();
    }
}

// ------------------------------------------------------------ reverse pass --
// Un-applies the pass's ops (listed in un-application order; angle -th) to psi
// and lambda and
// accumulates, per op, Im <lambda| G |psi> into the op's reduction row:
//   HOP : (-t) s (conj(lam_x) psi_y + conj(lam_y) psi_x) over the pairs
//   DIAG: D_sub(b) conj(lam_b) psi_b
// (the generator commutes with its own gate, so evaluating before the
// un-application is exact).  Row sums land in partial[row * stride + block].

__device__ __forceinline__ double im_conj_mul(double2 a, double2 b)
{
    return a.x * b.y - a.y * b.x;   // Im(conj(a) b)
}

__device__ void block_reduce_rows(double *red, int n_red, double *partial, int red_base,
                                  int stride)
{
    const int T = blockDim.x, tid = threadIdx.x;
    for (int r = 0; r < n_red; ++r) {
        double *row = red + r * T;
        for (int s = T >> 1; s > 0; s >>= 1) {
            __syncthreads();
            if (tid < s)
                row[tid] += row[tid + s];
        }
        __syncthreads();
        if (tid == 0)
            partial[(size_t)(red_base + r) * stride + blockIdx.x] = row[0];
    }
}

__global__ void __launch_bounds__(256)
k_reverse(DevPass P, const DevOp *__restrict__ ops, const DevVBond *__restrict__ vb,
          const double *__restrict__ theta, const DevModel *__restrict__ M,
          double2 *__restrict__ psi, double2 *__restrict__ lam, double *__restrict__ partial,
          int stride)
{
    extern __shared__ __align__(16) char smem[];
    const int T = blockDim.x, tid = threadIdx.x;
    const SmemPlan sp = smem_plan(P.k, P.c, 2, P.n_ops, P.n_diag, P.n_red, T);
    double2 *tp = (double2 *)(smem + sp.tiles);
    double2 *tq = tp + (1u << P.k);
    const uint32_t *offs = (const uint32_t *)(smem + sp.offs);
    const double2 *opc = (const double2 *)(smem + sp.opc);
    const double2 *dtab = (const double2 *)(smem + sp.dtab);
    double *red = (double *)(smem + sp.red);
    pass_setup(P, ops, theta, M, -1.0, smem, sp);
    for (int r = 0; r < P.n_red; ++r)
        red[r * T + tid] = 0.0;
    __syncthreads();

    const int k = P.k, c = P.c;
    const uint32_t cmask = (1u << c) - 1u;
    const uint32_t tsize = 1u << k;
    const uint64_t ntiles = (uint64_t)1 << P.nfree;
    for (uint64_t tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        const uint32_t base = tile_base(tl, P);
        for (uint32_t l = tid; l < tsize; l += T) {
            uint64_t g = base | offs[l >> c] | (l & cmask);
            tp[l] = psi[g];
            tq[l] = lam[g];
        }
        __syncthreads();
        // the reverse plan stores each pass's ops in un-application order
        for (int o = 0; o < P.n_ops; ++o) {
            const DevOp op = ops[P.op_begin + o];
            double acc = 0.0;
            if (op.kind == OP_DIAG) {
                for (uint32_t l = tid; l < tsize; l += T) {
                    uint32_t g = base | offs[l >> c] | (l & cmask);
                    double2 a = tp[l], b = tq[l];
                    acc += diag_value(op, g, M, vb) * im_conj_mul(b, a);
                    double2 ph = diag_phase(op, g, M, vb, theta, -1.0, dtab);
                    tp[l] = cmul(a, ph);
                    tq[l] = cmul(b, ph);
                }
            } else {
                const double cs = opc[o].x, sn = opc[o].y;
                const uint32_t par0 = __popc((uint32_t)tl & op.bm_free) & 1u;
                const int lo = min(op.pl, op.ql), hi = max(op.pl, op.ql);
                const uint32_t flip = (1u << op.pl) | (1u << op.ql);
                for (uint32_t j = tid; j < (tsize >> 2); j += T) {
                    uint32_t x = insert_zero(insert_zero(j, lo), hi) | (1u << op.pl);
                    uint32_t y = x ^ flip;
                    uint32_t par = (__popc(x & op.bm_local) + par0) & 1u;
                    double ss = par ? -sn : sn;
                    double sg = par ? -1.0 : 1.0;
                    double2 a = tp[x], b = tp[y];
                    double2 la = tq[x], lb = tq[y];
                    acc += sg * (im_conj_mul(la, b) + im_conj_mul(lb, a));
                    tp[x] = make_double2(cs * a.x - ss * b.y, cs * a.y + ss * b.x);
                    tp[y] = make_double2(cs * b.x - ss * a.y, cs * b.y + ss * a.x);
                    tq[x] = make_double2(cs * la.x - ss * lb.y, cs * la.y + ss * lb.x);
                    tq[y] = make_double2(cs * lb.x - ss * la.y, cs * lb.y + ss * la.x);
                }
                acc *= -op.t;
            }
            if (op.red >= 0)
                red[op.red * T + tid] += acc;
            __syncthreads();
        }
        for (uint32_t l = tid; l < tsize; l += T) {
            uint64_t g = base | offs[l >> c] | (l & cmask);
            psi[g] = tp[l];
            lam[g] = tq[l];
        }
        __syncthreads();
    }
    block_reduce_rows(red, P.n_red, partial, P.red_base, stride);
}

// ---------------------------------------------------------------- H passes --
// phi <- D psi + sum of the pass's terms (first pass), phi += terms (others);
// the last pass also reduces Re <psi|phi> into its row 0.

__global__ void __launch_bounds__(256)
k_hamiltonian(DevPass P, const DevOp *__restrict__ ops, const DevVBond *__restrict__ vb,
              const DevModel *__restrict__ M, const double2 *__restrict__ psi,
              double2 *__restrict__ phi, double *__restrict__ partial, int stride)
{
    extern __shared__ __align__(16) char smem[];
    const int T = blockDim.x, tid = threadIdx.x;
    const SmemPlan sp = smem_plan(P.k, P.c, 2, P.n_ops, P.n_diag, P.n_red, T);
    double2 *tp = (double2 *)(smem + sp.tiles);
    double2 *tf = tp + (1u << P.k);
    double *red = (double *)(smem + sp.red);
    uint32_t *offs = (uint32_t *)(smem + sp.offs);
    {
        const int nhi = P.k - P.c;
        for (int i = tid; i < (1 << nhi); i += T) {
            uint32_t o = 0;
            for (int j = 0; j < nhi; ++j)
                if ((i >> j) & 1)
                    o |= 1u << P.tile_pos[P.c + j];
            offs[i] = o;
        }
    }
    double eacc = 0.0;
    __syncthreads();
    const int k = P.k, c = P.c;
    const uint32_t cmask = (1u << c) - 1u;
    const uint32_t tsize = 1u << k;
    const uint64_t ntiles = (uint64_t)1 << P.nfree;
    const bool first = (P.flags & PF_HAM_FIRST) != 0;
    const bool last = (P.flags & PF_HAM_LAST) != 0;
    for (uint64_t tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        const uint32_t base = tile_base(tl, P);
        for (uint32_t l = tid; l < tsize; l += T) {
            uint64_t g = base | offs[l >> c] | (l & cmask);
            tp[l] = psi[g];
            tf[l] = first ? make_double2(0.0, 0.0) : phi[g];
        }
        __syncthreads();
        for (int o = 0; o < P.n_ops; ++o) {
            const DevOp op = ops[P.op_begin + o];
            if (op.kind == OP_DIAG) {
                for (uint32_t l = tid; l < tsize; l += T) {
                    uint32_t g = base | offs[l >> c] | (l & cmask);
                    double d = diag_value(op, g, M, vb);
                    tf[l].x += d * tp[l].x;
                    tf[l].y += d * tp[l].y;
                }
            } else {
                const uint32_t par0 = __popc((uint32_t)tl & op.bm_free) & 1u;
                const int lo = min(op.pl, op.ql), hi = max(op.pl, op.ql);
                const uint32_t flip = (1u << op.pl) | (1u << op.ql);
                for (uint32_t j = tid; j < (tsize >> 2); j += T) {
                    uint32_t x = insert_zero(insert_zero(j, lo), hi) | (1u << op.pl);
                    uint32_t y = x ^ flip;
                    uint32_t par = (__popc(x & op.bm_local) + par0) & 1u;
                    double w = par ? op.t : -op.t;   // (-t) * s
                    tf[x].x += w * tp[y].x;
                    tf[x].y += w * tp[y].y;
                    tf[y].x += w * tp[x].x;
                    tf[y].y += w * tp[x].y;
                }
            }
            __syncthreads();
        }
        for (uint32_t l = tid; l < tsize; l += T) {
            uint64_t g = base | offs[l >> c] | (l & cmask);
            double2 f = tf[l];
            if (last)
                eacc += tp[l].x * f.x + tp[l].y * f.y;
            phi[g] = f;
        }
        __syncthreads();
    }
    if (P.n_red > 0) {
        red[tid] = eacc;
        block_reduce_rows(red, 1, partial, P.red_base, stride);
    }
}

// ------------------------------------------------------- expectation pass --
// Read-only energy: sum over its terms of <psi|term|psi>, and D if present:
//   DIAG: D(b) |psi_b|^2;  HOP: 2 (-t) s Re(conj(psi_x) psi_y) per pair.

__global__ void __launch_bounds__(256)
k_expect(DevPass P, const DevOp *__restrict__ ops, const DevVBond *__restrict__ vb,
         const DevModel *__restrict__ M, const double2 *__restrict__ psi,
         double *__restrict__ partial, int stride)
{
    extern __shared__ __align__(16) char smem[];
    const int T = blockDim.x, tid = threadIdx.x;
    const SmemPlan sp = smem_plan(P.k, P.c, 1, P.n_ops, P.n_diag, 1, T);
    double2 *tp = (double2 *)(smem + sp.tiles);
    double *red = (double *)(smem + sp.red);
    uint32_t *offs = (uint32_t *)(smem + sp.offs);
    {
        const int nhi = P.k - P.c;
        for (int i = tid; i < (1 << nhi); i += T) {
            uint32_t o = 0;
            for (int j = 0; j < nhi; ++j)
                if ((i >> j) & 1)
                    o |= 1u << P.tile_pos[P.c + j];
            offs[i] = o;
        }
    }
    double eacc = 0.0;
    __syncthreads();
    const int k = P.k, c = P.c;
    const uint32_t cmask = (1u << c) - 1u;
    const uint32_t tsize = 1u << k;
    const uint64_t ntiles = (uint64_t)1 << P.nfree;
    for (uint64_t tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        const uint32_t base = tile_base(tl, P);
        for (uint32_t l = tid; l < tsize; l += T)
            tp[l] = psi[(uint64_t)(base | offs[l >> c] | (l & cmask))];
        __syncthreads();
        for (int o = 0; o < P.n_ops; ++o) {
            const DevOp op = ops[P.op_begin + o];
            if (op.kind == OP_DIAG) {
                for (uint32_t l = tid; l < tsize; l += T) {
                    uint32_t g = base | offs[l >> c] | (l & cmask);
                    double2 a = tp[l];
                    eacc += diag_value(op, g, M, vb) * (a.x * a.x + a.y * a.y);
                }
            } else {
                const uint32_t par0 = __popc((uint32_t)tl & op.bm_free) & 1u;
                const int lo = min(op.pl, op.ql), hi = max(op.pl, op.ql);
                const uint32_t flip = (1u << op.pl) | (1u << op.ql);
                double acc = 0.0;
                for (uint32_t j = tid; j < (tsize >> 2); j += T) {
                    uint32_t x = insert_zero(insert_zero(j, lo), hi) | (1u << op.pl);
                    uint32_t y = x ^ flip;
                    uint32_t par = (__popc(x & op.bm_local) + par0) & 1u;
                    double2 a = tp[x], b = tp[y];
                    double re = a.x * b.x + a.y * b.y;
                    acc += par ? -re : re;
                }
                eacc += -2.0 * op.t * acc;
            }
        }
        __syncthreads();
    }
    red[tid] = eacc;
    block_reduce_rows(red, 1, partial, P.red_base, stride);
}

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
