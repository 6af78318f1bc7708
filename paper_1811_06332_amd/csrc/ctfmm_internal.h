// Internal declarations shared by the kernels and the host side of libctfmm.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "generated/ctfmm_gen.h"

namespace ctfmm {

constexpr int PMAX = GEN_PMAX;
constexpr int NIND = GEN_NIND;    // (PMAX+1)^2 independent traceless components
constexpr int NFULL = GEN_NFULL;  // C(PMAX+3,3) full components
constexpr int NOFF = 343;         // offset slots v in [-3,3]^3, slot = (vx+3) + 7 (vy+3) + 49 (vz+3)

// Device copies of the generated operator tables (one allocation).
struct DevTables {
    const int8_t* ind;        // [NIND][3]
    const int8_t* full;       // [NFULL][3]
    const double* inv_mfact;  // [NFULL] 1/(nx! ny! nz!)
    const int16_t* exp_start; // [NFULL+1]
    const uint8_t* exp_slot;
    const int32_t* exp_coef;
    const int16_t* p2m_start; // [NIND+1]
    const double* p2m_coef;
    const int8_t* p2m_exp;    // [terms][4]
    const double* m2m_t;      // [8][NIND j][NIND n] (transposed)
    const double* l2l_t;      // [8][NIND j][NIND n] (transposed)
    const int32_t* c_start;   // [NIND n][NIND j]
    const uint8_t* c_count;   // [NIND n][NIND j]
    const uint8_t* c_slot;
    const double* c_coef;
    const int16_t* det_start;  // [NIND+1] detracer rows: independent n <- full f
    const int16_t* det_full;
    const double* det_coef;
};

// row stride of the expansion buffers: (p+1)^2 rounded up to a multiple of 4
__host__ __device__ constexpr int ldm_of(int p) { return ((p + 1) * (p + 1) + 3) & ~3; }

// Morton interleave of 10-bit coordinates (x in bit 0 of each triple).
__host__ __device__ inline uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__host__ __device__ inline uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030C30C3u;
    v = (v | (v >> 4)) & 0x0300F00Fu;
    v = (v | (v >> 8)) & 0x030000FFu;
    v = (v | (v >> 16)) & 0x3ffu;
    return v;
}
__host__ __device__ inline uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

// Geometry of the uniform octree.
struct Box {
    double lo[3];
    double side;
    int depth;
};

// ---- adaptive octree ----
constexpr int AMAX = 21;  // deepest level: 3 x 21-bit Morton keys

// Morton interleave of 21-bit coordinates into 63-bit keys (x in bit 0)
__host__ __device__ inline uint64_t spread21(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}
__host__ __device__ inline uint32_t compact21(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return (uint32_t)v;
}

// ---- expansion-order network (ctfmm_mlp.hip) ----
constexpr int MLP_NIN = 12, MLP_NH = 64, MLP_NOUT = 9;  // outputs: orders 2..10
constexpr int MLP_NPARAM = MLP_NH * MLP_NIN + MLP_NH + MLP_NH * MLP_NH + MLP_NH + MLP_NOUT * MLP_NH + MLP_NOUT;
constexpr int NCLASS = 15;  // occupied |v|^2 classes of the ws=1 offsets

// root cube of one adaptive tree
struct ABox {
    double lo[3];
    double side;
};

// Node arrays of the adaptive tree (structure of arrays, levels contiguous).
struct ATree {
    uint64_t* key;   // Morton prefix at the node's level (3 * level bits)
    int32_t* pb;     // first sorted particle
    int32_t* pe;     // one past the last
    int32_t* par;    // parent node, -1 for the root
    int32_t* info;   // level | (leaf << 8)
    int32_t* child;  // [8] child per octant (x = bit 0), -1 = empty
    int32_t* nb;     // [27] same-level neighbour at offset d = (dx+1)+3(dy+1)+9(dz+1),
                     // else the coarser leaf covering that cell, else -1
    int32_t* sys;    // system (tree of the forest) the node belongs to
    double4* geo;    // (centre x, y, z, side) of the node's cube
};

// Systems of a forest: particles of system s are forest positions
// [goff[s], goff[s+1]) and global indices gbase[s] + (i - goff[s]).
struct ASys {
    int nsys;
    const int32_t* goff;
    const int32_t* gbase;
};

// M2L over tables: tile t has TT target rows tgt[TT t ..] (-1 = none) of
// octant tiles[t].x, and for offset i of that octant the source rows
// src[(189 t + i) TT ..] (-1 = none); kslot[o][i] = slot of its operator.
// The offsets a tile runs are all 189, or (ivlist) the ivcnt[t] listed in
// ivlist[189 t ..]; with ivord, list entry j of tile t runs at order
// ivord[189 t + j] (<= the kernel order P), using the operators of that
// order at Kpk + order * kord_stride (each order's set in the order-P chunk
// layout, of which the first nup[order] chunks are non-zero; the launcher
// fills nup); the FP32 kernel (launch_m2l_rb) instead takes the order-P set
// and truncates it per offset in registers.
struct AdaptM2L {
    const int4* tiles;
    const int32_t* tgt;
    const int32_t* src;
    const int16_t* kslot;
    int tile_base;
    const int16_t* ivlist = nullptr;
    const int32_t* ivcnt = nullptr;
    const int8_t* ivord = nullptr;
    size_t kord_stride = 0;
    int nup[11] = {};
    bool acc = false;
    // the offsets of a tile split over nchunk workgroups (balanced, in list
    // order); chunk c writes the first (p+1)^2 entries of its targets' rows
    // into L + c * chunk_stride (zeros if it has no offsets); other entries
    // of a slot are left as they were.  acc: the output is partial-sum slots
    // (needed for nchunk > 1)
    int nchunk = 1;
    size_t chunk_stride = 0;
};

// P2M of one cell by one wavefront, two phases.  (1) Full monomial moments
// S_f = sum_a q_a u_a^f, u = (z - x)/h, |f| <= P, with the power tables of up
// to 64 particles at a time in LDS and lanes over f.  (2) The detracer:
// M~_n = sum_f DET[n][f] S_f for the independent n (Eq. P2M with Eq.
// Detracer).  Particles [b, e) of P; writes the ldm_of(P) entries of Mc.
// DIP: the particles also carry point dipoles d_a (Pd, xyz), each a pure
// dipole (rank-1 moment -d_a) moved from x_a to z by Eq. M2M (Appendix B.1):
// S_f += -(1/h) sum_i d_{a,i} f_i u_a^(f - e_i).
// CH: particles whose power tables are staged at a time (the LDS held per
// wavefront; small for trees with few particles per leaf).
template <int PP, bool DIP = false, int CH = 64>
__device__ inline void p2m_cell(double zx, double zy, double zz, double h, int b, int e,
                                const double4* __restrict__ P, const DevTables& T, double* __restrict__ Mc,
                                const double4* __restrict__ Pd = nullptr) {
    static_assert(CH >= 1 && CH <= 64, "one wavefront stages at most 64 particles");
    const int lane = threadIdx.x;
    constexpr int nc = (PP + 1) * (PP + 1);
    constexpr int nf = (PP + 1) * (PP + 2) * (PP + 3) / 6;
    constexpr int ldm = ldm_of(PP);
    __shared__ double pw[CH][3][PP + 1];
    __shared__ double qs[CH];
    __shared__ double ds[DIP ? CH : 1][3];
    __shared__ double S[nf];
    constexpr int FPL = (nf + 63) / 64;  // full components per lane
    double acc[FPL];
    int fa[FPL], fb[FPL], fc[FPL];
#pragma unroll
    for (int k = 0; k < FPL; ++k) {
        acc[k] = 0.0;
        const int f = lane + 64 * k;
        fa[k] = f < nf ? T.full[3 * f] : 0;
        fb[k] = f < nf ? T.full[3 * f + 1] : 0;
        fc[k] = f < nf ? T.full[3 * f + 2] : 0;
    }
    for (int s0 = b; s0 < e; s0 += CH) {
        const int cnt = min(CH, e - s0);
        if (lane < cnt) {
            const double4 pt = P[s0 + lane];
            const double u[3] = {(zx - pt.x) / h, (zy - pt.y) / h, (zz - pt.z) / h};
#pragma unroll
            for (int dim = 0; dim < 3; ++dim) {
                double v = 1.0;
#pragma unroll
                for (int k = 0; k <= PP; ++k) {
                    pw[lane][dim][k] = v;
                    v *= u[dim];
                }
            }
            qs[lane] = pt.w;
            if (DIP) {
                const double4 d = Pd[s0 + lane];
                ds[DIP ? lane : 0][0] = -d.x / h;
                ds[DIP ? lane : 0][1] = -d.y / h;
                ds[DIP ? lane : 0][2] = -d.z / h;
            }
        }
        __syncthreads();
        for (int i = 0; i < cnt; ++i) {
            const double q = qs[i];
#pragma unroll
            for (int k = 0; k < FPL; ++k) {
                const double X = pw[i][0][fa[k]], Y = pw[i][1][fb[k]], Z = pw[i][2][fc[k]];
                acc[k] += q * X * Y * Z;
                if (DIP) {
                    const int j = DIP ? i : 0;
                    acc[k] += ds[j][0] * fa[k] * pw[i][0][max(fa[k] - 1, 0)] * Y * Z +
                              ds[j][1] * fb[k] * X * pw[i][1][max(fb[k] - 1, 0)] * Z +
                              ds[j][2] * fc[k] * X * Y * pw[i][2][max(fc[k] - 1, 0)];
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < FPL; ++k)
        if (lane + 64 * k < nf) S[lane + 64 * k] = acc[k];
    __syncthreads();
    for (int n = lane; n < ldm; n += 64) {
        double v = 0.0;
        // unrolled so that several of the independent table loads are in
        // flight (the sum keeps its order)
        if (n < nc) {
            const int t1 = T.det_start[n + 1];
#pragma unroll 8
            for (int t = T.det_start[n]; t < t1; ++t) v += T.det_coef[t] * S[T.det_full[t]];
        }
        Mc[n] = v;  // padding is kept zero
    }
}

// one source: phi += q/r, grad -= q (x_b - x_a)/r^3; a pair at distance 0
// (the particle itself, or a coincident one) contributes nothing (no branch:
// the reciprocal distance is selected to 0)
// 1/sqrt(x) for x > 0: the hardware estimate y0, refined by the second-order
// expansion of (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ... with e = 1 - x y0^2.
// Measured over 2^22 values spread across 2^+-40: the estimate is within
// 2^-24.2 relative, so the neglected e^3 term is far below double rounding,
// and the result within 1.25 ulp.  x = 0 gives a NaN, selected away by the caller.
__device__ inline double rsqrt_pos(double x) {
    const double y0 = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y0, y0, 1.0);
    return fma(y0 * e, fma(e, 0.375, 0.5), y0);
}

// Eq. PhiAB for one pair: potential and gradient at (xb, yb, zb) of the
// charge src.w at src.xyz; coincident points (the particle itself) add nothing.
__device__ inline void pair_add_a(double xb, double yb, double zb, double4 src, double& f, double& gx, double& gy,
                                  double& gz) {
    const double dx = xb - src.x, dy = yb - src.y, dz = zb - src.z;
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const double y = r2 > 0.0 ? rsqrt_pos(r2) : 0.0;  // a select: both sides are computed
    const double qy = src.w * y;
    f += qy;
    const double ir3 = qy * y * y;
    gx = fma(-ir3, dx, gx);
    gy = fma(-ir3, dy, gy);
    gz = fma(-ir3, dz, gz);
}

// ---- launchers (ctfmm_kernels.hip); every one enqueues on `s` ----
void launch_keys(hipStream_t s, int n, const double* xyz, Box box, uint32_t* keys, int32_t* idx, int* err);
void launch_gather(hipStream_t s, int n, const int32_t* idx, const double* xyz, const double* q, double4* P);
// point dipoles in sorted order (x, y, z, 0)
void launch_gather_dip(hipStream_t s, int n, const int32_t* idx, const double* dip, double4* Pd);
void launch_leaf_start(hipStream_t s, int nleaves, const uint32_t* keys, int n, int32_t* start);
// Pd (may be null): point dipoles in sorted order
void launch_p2m(hipStream_t s, int p, Box box, const int32_t* start, const double4* P, const DevTables& T, double* M,
                const double4* Pd = nullptr);
void launch_m2m(hipStream_t s, int p, int parent_level, const double* Mchild, double* Mparent, const DevTables& T);
void launch_offset_dtensors(hipStream_t s, int p, double* Dv);
void launch_build_k(hipStream_t s, int p, const double* Dv, const DevTables& T, double* Kt);
void launch_l2l(hipStream_t s, int p, int parent_level, const double* Lparent, double* Lchild, const DevTables& T);
void launch_l2p(hipStream_t s, int p, int n, Box box, const int32_t* start, const uint32_t* keys, const double4* P,
                const double* L, double4* F);
void launch_p2p(hipStream_t s, int n, Box box, const uint32_t* keys, const int32_t* start, const double4* P,
                const int32_t* idx, const double4* F, double* phi, double* grad, const double4* Pd = nullptr);
// the same without dipoles, one wavefront per leaf
void launch_p2p_leaves(hipStream_t s, Box box, const int32_t* start, const double4* P, const int32_t* idx,
                       const double4* F, double* phi, double* grad);
// M2L operand precision (ctfmm_precision values)
enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16X3 = 2 };
size_t m2l_packed_bytes(int p, int prec);
size_t m2l_lds_bytes(int p, int prec);
// K_v fragments of order p in the M2L precision; pmask < p packs the
// order-pmask operators in the same layout
void launch_pack_k(hipStream_t s, int p, int prec, const double* Kt, unsigned char* Kpk, int pmask);
void launch_to_f32(hipStream_t s, int p, long long ncell, const double* M, float* M32);
// the k-quad-major FP32 rows read by launch_m2l_rb
void launch_to_f32_kq(hipStream_t s, int p, long long ncell, const double* M, float* M32);
// FP32 (Kq given): with Lpar (the parent level's local expansions) the
// kernel also adds the L2L from the parents and writes L once
hipError_t launch_m2l(hipStream_t s, int p, int prec, int level, const void* Msrc, double* L,
                      const unsigned char* Kpk, const int16_t* offlist, const unsigned char* zero_row,
                      const float* Kq = nullptr, const double* Lpar = nullptr, const double* l2l_t = nullptr);
// FP32 operators with the chunks of a lane four at a time side by side:
// Kq[slot][chunk / 4][lane][chunk % 4] (chunks past the last are zero)
size_t m2l_quad_bytes(int p);
void launch_quad_k(hipStream_t s, int p, const unsigned char* Kpk, float* Kq);
// M2L of ntiles tiles of tt targets (32, 64 or 128) of the adaptive tree (any
// precision; rows are node indices)
hipError_t launch_m2l_tables(hipStream_t s, int p, int prec, int tt, int ntiles, const AdaptM2L& ad, const void* Msrc,
                             double* L, const unsigned char* Kpk, const unsigned char* zero_row);
// FP32 adaptive M2L with fixed orders (no ivlist, ord or ld_in) from k-quad-major rows
hipError_t launch_m2l_rb(hipStream_t s, int p, int tt, int ntiles, const AdaptM2L& ad, const float* M32k, double* L,
                         const unsigned char* Kpk, const unsigned char* zero_row);
size_t m2l_tile_lds_bytes(int p, int prec, int tt);
// row stride of the FP32 multipole copy: (p+1)^2 rounded up to a multiple of 32
__host__ __device__ constexpr int s32_of(int p) { return (((p + 1) * (p + 1) + 31) / 32) * 32; }
void launch_unscale_copy(hipStream_t s, int p, int level, int which, double side, const double* X, double* out);

// ---- adaptive tree launchers (ctfmm_adaptive.hip) ----
void launch_bbox(hipStream_t s, int n, const double* xyz, double* part, int nparts, double* out);
void launch_bbox_systems(hipStream_t s, const ASys& sy, const double* xyz, ABox* boxes);
void launch_low32(hipStream_t s, int n, const uint64_t* kc, uint32_t* k32s);
// composite: keys = system index << 32 | top 32 key bits (else the 63-bit keys)
void launch_keys64(hipStream_t s, int n, const ASys& sy, const double* xyz, const ABox* boxes, uint64_t* keys,
                   uint32_t* k32, int32_t* idx, int* err, bool composite = false);
void launch_gather_keyed(hipStream_t s, int n, const ASys& sy, const int32_t* idx, const double* xyz, const double* q,
                         const ABox* boxes, double4* P, uint64_t* keys);
void launch_deep_check(hipStream_t s, int n, const ASys& sy, const uint32_t* k32s, int leaf_max, int* flag);
void launch_roots(hipStream_t s, const ASys& sy, const ATree& t);
void launch_split(hipStream_t s, int level, int first, int count, int leaf_max, const uint64_t* keys, const ATree& t,
                  int32_t* flag, int32_t* cstart);
// also writes the next level's node count to host[0] (and *deep to host[1]
// when deep is given), host being device-accessible pinned memory (or null)
void launch_emit(hipStream_t s, int level, int first, int count, int next_first, const int32_t* flag,
                 const int32_t* incl, const int32_t* cstart, const ATree& t, int* host, const int32_t* deep);
void launch_nb(hipStream_t s, int first, int count, const ATree& t);
void launch_leaf_of(hipStream_t s, int nn, const ATree& t, int32_t* leaf_of);
void launch_lists(hipStream_t s, bool fill, int nn, const ATree& t, int32_t* ucnt, int32_t* wcnt, int32_t* xcnt,
                  int32_t* ufcnt, const int32_t* uoff, const int32_t* woff, const int32_t* xoff, int32_t* ulist,
                  int32_t* wlist, int32_t* xlist, int32_t* wfill, int32_t* ufill);
void launch_add_i32(hipStream_t s, int n, const int32_t* a, const int32_t* b, int32_t* out);
// segments [beg[g], end[g]) of in sorted ascending into out (one wavefront per segment)
void launch_rank_sort(hipStream_t s, int nseg, const int32_t* beg, const int32_t* end, const int32_t* in,
                      int32_t* out);
void launch_lvloct(hipStream_t s, int nn, const ATree& t, uint32_t* k, int32_t* v);
void launch_buckets(hipStream_t s, int nn, const uint32_t* sk, int32_t* bstart, int32_t* bend);
void launch_tile_keys(hipStream_t s, int ntiles, const int4* tiles, const int32_t* sorted, const ATree& t,
                      uint64_t* key, int32_t* idx);
void launch_gather_int4(hipStream_t s, int n, const int32_t* idx, const int4* in, int4* out);
void launch_m2l_tables(hipStream_t s, int tt, int ntiles, const int4* tiles, const int32_t* sorted, const ATree& t,
                       const int16_t* qu_list, int32_t* tgt_tab, int32_t* src_tab, int32_t* vcount);
void launch_node_geo(hipStream_t s, int nn, const ABox* boxes, const ATree& t);
void launch_p2m_nodes(hipStream_t s, int p, int first, int count, const ABox* boxes, const ATree& t, const double4* P,
                      const DevTables& T, double* M);
void launch_m2m_nodes(hipStream_t s, int p, int first, int count, const ATree& t, double* M, const DevTables& T);
void launch_l2l_nodes(hipStream_t s, int p, int first, int count, const ATree& t, double* L, const DevTables& T);
void launch_p2l(hipStream_t s, int p, int nn, const ABox* boxes, const ATree& t, const int32_t* xoff, const int32_t* xlist,
                const double4* P, const DevTables& T, double* L);
void launch_m2p_coef(hipStream_t s, int p, int first, int count, const double* M, const DevTables& T, double* Cm);
size_t m2p_coef_ld(int p);  // row stride of the W-list coefficient rows
// the W lists (wlists: added into Fn, before) and L2P, whose far field plus
// the near field Fn goes to phi and grad in input order (or with to_F to F)
void launch_far_adaptive(hipStream_t s, int p, int n, int nn, bool wlists, const ABox* boxes, const ATree& t,
                         const int32_t* leaf_of, const double4* P, const double* L, const double* Cm,
                         const int32_t* woff, const int32_t* wlist, double4* F, double4* Fn, const int32_t* idx,
                         bool to_F, double* phi, double* grad);
void launch_p2p_near(hipStream_t s, int n, int nn, const ATree& t, const double4* P, const int32_t* uoff,
                     const int32_t* ulist, double4* Fn);
// the W-list multipole evaluations alone, added into F
void launch_wlist_adaptive(hipStream_t s, int p, int nn, const ABox* boxes, const ATree& t, const double4* P,
                           const double* Cm, const int32_t* woff, const int32_t* wlist, double4* F);
void launch_scatter_out(hipStream_t s, int n, const int32_t* idx, const double4* F, double* phi, double* grad);

// ---- dual-tree traversal (ctfmm_dual.hip) ----
// centres and enclosing radii per node (mode: ctfmm_centre; sum: [nn]
// charge sums, used for modes 1 and 2); err bit 2 = a non-positive charge in
// the AP variant
void launch_dual_centres(hipStream_t s, int n, int nn, const std::vector<int>& lev_first,
                         const std::vector<int>& lev_count, const ATree& t, const ABox* boxes,
                         const int32_t* leaf_of, const double4* P, int mode, double4* sum, double4* zr, int* err);
void launch_dual_p2m(hipStream_t s, int p, int nn, const ATree& t, const double4* zr, const double4* P,
                     const DevTables& T, double* M);
void launch_dual_m2m(hipStream_t s, int p, int first, int count, const ATree& t, const double4* zr,
                     const DevTables& T, double* M);
void launch_dual_l2l(hipStream_t s, int p, int first, int count, const ATree& t, const double4* zr,
                     const DevTables& T, double* L);
// cnt: [nr + 1] frontier sizes, then the M2L and direct-pair entry counts
void launch_dual_init(hipStream_t s, int nr, int* cnt, int2* front);
void launch_dual_round(hipStream_t s, int r, int nr, const int2* fin, int2* fout, int cap_f, uint64_t* mk, int cap_m,
                       uint64_t* pk, int cap_p, int sh, int* cnt, const ATree& t, const double4* zr, double theta);
void launch_dual_csr(hipStream_t s, int nn, const uint64_t* keys, const int* nkeys, int cap, int sh, int32_t* off,
                     int32_t* src);
void launch_dual_m2l(hipStream_t s, int p, bool ap, int nn, const ATree& t, const double4* zr, const int32_t* off,
                     const int32_t* src, const double* M, double* L);
void launch_dual_l2p(hipStream_t s, int p, bool ap, int n, const ATree& t, const int32_t* leaf_of, const double4* zr,
                     const double4* P, const double* L, const double4* Fn, const int32_t* idx, double* phi,
                     double* grad);

// ---- expansion orders per pair (ctfmm_adaptive.hip, ctfmm_mlp.hip) ----
// order of every (tile, offset): the largest its pairs ask for (-1 = no pair),
// into tq[189 tile + i]; ocnt[o][189 tile + i] = its pairs if that order is o
void launch_m2l_orders(hipStream_t s, int tt, int ntiles, const int4* tiles, const int32_t* src_tab,
                       const int16_t* kslot, const int8_t* ordn, int8_t* tq, int32_t* ocnt);
// the active offsets of every tile (an order in tq, or with tq null a source
// in vcount) in offset order, with their orders (tq, or p)
void launch_active_offsets(hipStream_t s, int ntiles, int p, const int8_t* tq, const int32_t* vcount,
                           int16_t* ivlist, int8_t* ivord, int32_t* ivcnt);
void launch_fill0(hipStream_t s, long long n, double* a);
void launch_widen(hipStream_t s, long long n, const float* in, double* out);
void launch_narrow(hipStream_t s, long long n, const double* in, float* out);
void launch_mlp_forward32(hipStream_t s, long long n, const float* x, const float* prm, float* y);
void launch_mlp_forward16(hipStream_t s, long long n, const float* x, const float* prm, const float* norm, float* y);
void launch_mlp_backward(hipStream_t s, long long n, const float* x, const float* t, const float* prm, float* act,
                         float* err, float* grad, float* loss);
size_t mlp_backward_part_floats(long long n);
// the allocation-free backward pass: scratch in a device array (address
// looked up per device by mlp_noalloc_setup, once, at context creation)
long long mlp_noalloc_max();
hipError_t mlp_noalloc_setup(int device);
hipError_t launch_mlp_backward_noalloc(hipStream_t s, int device, long long n, const float* x, const float* t,
                                       const float* prm, float* grad, float* loss);
void launch_adam(hipStream_t s, int step, float lr, float* prm, const float* g, float* m, float* v);
void launch_mlp_labels(hipStream_t s, long long n, const double* M, long long mstride, const int32_t* sel,
                       const int32_t* vslot, const double* Kt, float* x, float* y);
void launch_mlp_pick(hipStream_t s, long long n, unsigned long long seed, int first, int count, int32_t* sel,
                     int32_t* vs);
void launch_gather_rows(hipStream_t s, long long n, const int32_t* sel, const double* M, int ldm, double* out);
void launch_mlp_node_features(hipStream_t s, int first, int count, const double* M, int ldm, float* x);
void launch_mlp_decide(hipStream_t s, int first, int count, const float* y, float thr, int8_t* ord);
void launch_order_table(hipStream_t s, int count, const int32_t* tab, int8_t* ord);
void launch_order_hash(hipStream_t s, int count, const ATree& t, unsigned long long seed, int pmin, int p,
                       int8_t* ord);

void launch_sum_chunks(hipStream_t s, int nslots, size_t stride, const double* part, double* L, int nc, int ldm,
                       long long row0);

}  // namespace ctfmm
