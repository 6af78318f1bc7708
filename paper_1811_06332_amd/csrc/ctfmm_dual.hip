// Dual-tree FMM of libctfmm (gfx950): the driver of Appendix C on the
// adaptive octree of ctfmm_adaptive.hip.
//
//   centres   every node's expansion centre z (its geometric centre, or the
//             charge-weighted mean of its particles) and enclosing radius r
//             (the largest distance from z to one of its particles);
//   upward    P2M at the leaves about z (Eq. P2M), then M2M to the parents
//             with the shift z_child - z_parent (Eq. M2M) level by level,
//             as three one-axis binomial shifts of the full components and
//             the detracer;
//   traversal from the pair (root, root), in rounds: a round takes every
//             pair of its frontier and either accepts it (theta |z_B - z_A|
//             > r_A + r_B: two directed M2L entries), sums it directly (two
//             leaves), or opens the node of larger radius (never a leaf) and
//             puts its children's pairs into the next frontier; a node paired
//             with itself gives its children's self pairs and each two
//             children once.  The entries are appended with one atomic per
//             workgroup and chunk of pairs and sorted afterwards, so the
//             lists (and every sum over them) do not depend on the order of
//             the appends;
//   M2L       per target node, its sources in ascending order, one lane per
//             source: the traceless gradient of 1/r at the pair's offset and
//             the contraction of Eq. M2L, both straight-line generated code;
//             the lanes' sums are added by a butterfly (the same total on
//             every lane);
//   downward  L2L from each parent to its children (Eq. L2L, three one-axis
//             Taylor shifts of the full components), L2P at the
//             leaves (Eq. L2P); the direct part by the leaf-pair kernel of
//             the adaptive tree.
// Scaled expansions per node: M~_n = M_n / h^|n| and L~_n = L_n h^(|n|+1)
// with h the node's cube side.  The AP variant (Sec. 4: centre of mass,
// positive charges) leaves the dipole out of every M2L and computes the
// gradient only.
#include <math.h>

#include <vector>

#include "ctfmm_internal.h"

namespace ctfmm {

namespace {

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

__device__ inline bool leaf_d(int info) { return (info >> 8) & 1; }

__device__ inline int rank_d(int k) {
    int r = 0;
    while ((r + 1) * (r + 1) <= k) ++r;
    return r;
}

// |v| with the squares and sums rounded one by one, x + y first: the MAC is
// decided on the same floating-point values as a plain C evaluation
__device__ inline double norm_plain(double x, double y, double z) {
#pragma clang fp contract(off)
    const double xx = x * x, yy = y * y, zz = z * z;
    return sqrt((xx + yy) + zz);
}

// the cube centre of a node (level, Morton prefix key), with the products
// and sums rounded one by one as in a plain C evaluation
__device__ inline void cube_centre(const ABox& box, uint64_t key, int level, double* z) {
#pragma clang fp contract(off)
    const double h = box.side / (double)(1ll << level);
#pragma unroll
    for (int d = 0; d < 3; ++d) z[d] = box.lo[d] + ((double)compact21(key >> d) + 0.5) * h;
}

}  // namespace

// ------------------------------------------------------------------ centres and radii

// charge and charge moment (q, q x, q y, q z) of every leaf, one wavefront
// per leaf; AP (mode 2) flags a non-positive charge (bit 2 of err)
__global__ __launch_bounds__(64) void k_dual_leafsum(ATree t, const double4* __restrict__ P, int mode,
                                                     double4* __restrict__ sum, int* __restrict__ err) {
    const int g = blockIdx.x;
    if (!leaf_d(t.info[g])) return;
    const int b = t.pb[g], e = t.pe[g];
    double w = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    bool bad = false;
    for (int s = b + (int)threadIdx.x; s < e; s += 64) {
        const double4 pt = P[s];
        w += pt.w;
        sx += pt.w * pt.x;
        sy += pt.w * pt.y;
        sz += pt.w * pt.z;
        bad |= !(pt.w > 0.0);
    }
    if (mode == 2 && bad) atomicOr(err, 2);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        w += __shfl_xor(w, m);
        sx += __shfl_xor(sx, m);
        sy += __shfl_xor(sy, m);
        sz += __shfl_xor(sz, m);
    }
    if (threadIdx.x == 0) sum[g] = make_double4(sx, sy, sz, w);
}

// the non-leaf nodes of [first, first+count): the sums of their children
// in octant order
__global__ void k_dual_upsum(int first, int count, ATree t, double4* __restrict__ sum) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int g = first + i;
    if (leaf_d(t.info[g])) return;
    double4 a = make_double4(0.0, 0.0, 0.0, 0.0);
    for (int o = 0; o < 8; ++o) {
        const int c = t.child[8 * g + o];
        if (c < 0) continue;
        const double4 v = sum[c];
        a.x += v.x;
        a.y += v.y;
        a.z += v.z;
        a.w += v.w;
    }
    sum[g] = a;
}

// centre of every node (mode 0: the cube centre; else the charge-weighted
// mean where the total charge is positive, else the cube centre); radius 0
__global__ void k_dual_zr(int nn, ATree t, const ABox* __restrict__ boxes, int mode, const double4* __restrict__ sum,
                          double4* __restrict__ zr) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nn) return;
    double z[3];
    cube_centre(boxes[t.sys[g]], t.key[g], t.info[g] & 0xff, z);
    if (mode != 0) {
        const double4 v = sum[g];
        if (v.w > 0.0) {
            z[0] = v.x / v.w;
            z[1] = v.y / v.w;
            z[2] = v.z / v.w;
        }
    }
    zr[g] = make_double4(z[0], z[1], z[2], 0.0);
}

// enclosing radii: every particle takes its distance to the centre of each
// node that holds it (level by level from its leaf up); the lanes of a
// wavefront that share a node take the largest of theirs and one of them
// raises the node's radius by an atomic maximum on the bit pattern (radii
// are non-negative, so the bit patterns order like the values)
__global__ __launch_bounds__(256) void k_dual_radius(int n, int maxlev, ATree t, const int32_t* __restrict__ leaf_of,
                                                     const double4* __restrict__ P, double4* __restrict__ zr) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = s < n;
    int cur = live ? leaf_of[s] : -1;
    const double4 pt = live ? P[s] : make_double4(0.0, 0.0, 0.0, 0.0);
    int lev = cur >= 0 ? (t.info[cur] & 0xff) : -1;
    for (int l = maxlev; l >= 0; --l) {
        const int node = lev == l ? cur : -1;
        double d = 0.0;
        if (node >= 0) {
            const double4 z = zr[node];
            d = norm_plain(pt.x - z.x, pt.y - z.y, pt.z - z.z);
            cur = t.par[node];
            lev = cur >= 0 ? l - 1 : -1;
        }
        // one atomic per distinct node among the wavefront's lanes
        uint64_t todo = __ballot(node >= 0);
        while (todo) {
            const int leader = __ffsll((long long)todo) - 1;
            const int ln = __shfl(node, leader);
            const bool mine = node == ln && node >= 0;
            double v = mine ? d : 0.0;
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m));
            if ((int)(threadIdx.x & 63) == leader)
                atomicMax((unsigned long long*)&zr[ln].w, (unsigned long long)__double_as_longlong(v));
            todo &= ~__ballot(mine);
        }
    }
}

void launch_dual_centres(hipStream_t s, int n, int nn, const std::vector<int>& lev_first,
                         const std::vector<int>& lev_count, const ATree& t, const ABox* boxes,
                         const int32_t* leaf_of, const double4* P, int mode, double4* sum, double4* zr, int* err) {
    if (nn <= 0) return;
    const int maxlev = (int)lev_first.size() - 1;
    if (mode != 0) {
        hipLaunchKernelGGL(k_dual_leafsum, dim3(nn), dim3(64), 0, s, t, P, mode, sum, err);
        for (int l = maxlev - 1; l >= 0; --l)
            hipLaunchKernelGGL(k_dual_upsum, dim3(cdiv(lev_count[l], 256)), dim3(256), 0, s, lev_first[l],
                               lev_count[l], t, sum);
    }
    hipLaunchKernelGGL(k_dual_zr, dim3(cdiv(nn, 256)), dim3(256), 0, s, nn, t, boxes, mode, sum, zr);
    hipLaunchKernelGGL(k_dual_radius, dim3(cdiv(n, 256)), dim3(256), 0, s, n, maxlev, t, leaf_of, P, zr);
}

// ------------------------------------------------------------------ P2M, M2M, L2L about arbitrary centres

// P2M of every leaf about its centre, one wavefront per node
template <int PP>
__global__ __launch_bounds__(64) void k_dual_p2m(ATree t, const double4* __restrict__ zr,
                                                 const double4* __restrict__ P, DevTables T, double* __restrict__ M) {
    const int g = blockIdx.x;
    if (!leaf_d(t.info[g])) return;
    const double4 z = zr[g];
    p2m_cell<PP>(z.x, z.y, z.z, t.geo[g].w, t.pb[g], t.pe[g], P, T, M + (size_t)g * ldm_of(PP));
}

// position of the full component (a, b, c) (rank-major, a then b descending)
__device__ inline int fidx(int a, int b, int c) {
    const int n = a + b + c;
    return n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + (n - a - b);
}

// full traceless components X[f], |f| <= P, of the independent ones x
// (scaled by 2^-|f| if halve), one wavefront
template <int P>
__device__ inline void expand_full(const double* __restrict__ x, bool halve, const DevTables& T, double* X) {
    constexpr int nf = (P + 1) * (P + 2) * (P + 3) / 6;
    for (int f = threadIdx.x; f < nf; f += 64) {
        double v = 0.0;
        const int t1 = T.exp_start[f + 1];
        for (int t = T.exp_start[f]; t < t1; ++t) v += (double)T.exp_coef[t] * x[T.exp_slot[t]];
        X[f] = halve ? ldexp(v, -(T.full[3 * f] + T.full[3 * f + 1] + T.full[3 * f + 2])) : v;
    }
}

// Y[n] = sum_t w(n_d, t) X[n with n_d replaced] along axis d, for every
// full n with |n| <= P.  M2M (shift of the moments, Eq. M2M): the binomial
// sum over t <= n_d of C(n_d, t) s^(n_d - t) X[.., t, ..]; L2L (Taylor
// shift, Eq. L2L): the sum over t <= P - |n| of s^t / t! X[.., n_d + t, ..].
template <int P, bool TAYLOR>
__device__ inline void shift_axis(int d, double s, const double* X, double* Y, bool add, const DevTables& T) {
    constexpr int nf = (P + 1) * (P + 2) * (P + 3) / 6;
    for (int f = threadIdx.x; f < nf; f += 64) {
        int e[3] = {T.full[3 * f], T.full[3 * f + 1], T.full[3 * f + 2]};
        const int nd = e[d], rank = e[0] + e[1] + e[2];
        double v = 0.0;
        if (TAYLOR) {
            double w = 1.0;
            for (int t = 0; t <= P - rank; ++t) {
                e[d] = nd + t;
                v += w * X[fidx(e[0], e[1], e[2])];
                w *= s / (double)(t + 1);
            }
        } else {
            double w = 1.0;  // C(nd, t) s^(nd - t), from t = nd down
            for (int t = nd; t >= 0; --t) {
                e[d] = t;
                v += w * X[fidx(e[0], e[1], e[2])];
                w *= s * (double)t / (double)(nd - t + 1);
            }
        }
        Y[f] = add ? Y[f] + v : v;
    }
}

// M~(parent) = the detracer of the sum over its children, in octant order,
// of the child's multipole (full components, rho = 1/2 applied) moved by
// d = z_child - z_parent (Eq. M2M): three one-axis binomial shifts with
// s = -d/h_P, then M~_n = sum DET[n][f] S_f (Eq. Detracer, as in P2M).
// One workgroup per non-leaf node of [first, first+count); the eight
// children are shifted side by side (a missing child contributes zeros).
constexpr int M2M_B = 256;
template <int P>
__global__ __launch_bounds__(M2M_B) void k_dual_m2m(int first, ATree t, const double4* __restrict__ zr, DevTables T,
                                                    double* __restrict__ M) {
    constexpr int nc = (P + 1) * (P + 1);
    constexpr int nf = (P + 1) * (P + 2) * (P + 3) / 6;
    constexpr int ldm = ldm_of(P);
    const int g = first + blockIdx.x;
    if (leaf_d(t.info[g])) return;
    __shared__ double X[8][nf], Y[8][nf];
    __shared__ int8_t E[nf][3];
    __shared__ double sd[8][3];
    __shared__ int cid[8];
    const int tid = threadIdx.x;
    for (int f = tid; f < nf; f += M2M_B)
        for (int d = 0; d < 3; ++d) E[f][d] = T.full[3 * f + d];
    if (tid < 8) {
        const int c = t.child[8 * g + tid];
        cid[tid] = c;
        const double4 zp = zr[g];
        const double ih = 1.0 / t.geo[g].w;
        const double4 zc = c >= 0 ? zr[c] : zp;
        sd[tid][0] = -(zc.x - zp.x) * ih;
        sd[tid][1] = -(zc.y - zp.y) * ih;
        sd[tid][2] = -(zc.z - zp.z) * ih;
    }
    __syncthreads();
    for (int it = tid; it < 8 * nf; it += M2M_B) {
        const int ch = it / nf, f = it % nf;
        const int c = cid[ch];
        double v = 0.0;
        if (c >= 0) {
            const double* x = M + (size_t)c * ldm;
            const int t1 = T.exp_start[f + 1];
            for (int q = T.exp_start[f]; q < t1; ++q) v += (double)T.exp_coef[q] * x[T.exp_slot[q]];
            v = ldexp(v, -(E[f][0] + E[f][1] + E[f][2]));
        }
        X[ch][f] = v;
    }
    // three one-axis shifts: X -> Y (x), Y -> X (y), X -> Y (z)
    for (int d = 0; d < 3; ++d) {
        __syncthreads();
        double(*src)[nf] = (d == 1) ? Y : X;
        double(*dst)[nf] = (d == 1) ? X : Y;
        for (int it = tid; it < 8 * nf; it += M2M_B) {
            const int ch = it / nf, f = it % nf;
            int e[3] = {E[f][0], E[f][1], E[f][2]};
            const int nd = e[d];
            const double sv = sd[ch][d];
            double v = 0.0, w = 1.0;  // C(nd, t) s^(nd - t), from t = nd down
            for (int tt = nd; tt >= 0; --tt) {
                e[d] = tt;
                v += w * src[ch][fidx(e[0], e[1], e[2])];
                w *= sv * (double)tt / (double)(nd - tt + 1);
            }
            dst[ch][f] = v;
        }
    }
    __syncthreads();
    for (int n = tid; n < ldm; n += M2M_B) {
        double v = 0.0;
        if (n < nc) {
            const int t1 = T.det_start[n + 1];
            for (int q = T.det_start[n]; q < t1; ++q) {
                const int f = T.det_full[q];
                double sf = 0.0;
#pragma unroll
                for (int ch = 0; ch < 8; ++ch) sf += Y[ch][f];
                v += T.det_coef[q] * sf;
            }
        }
        M[(size_t)g * ldm + n] = v;  // padding stays zero
    }
}

// L~(child) += rho^(|n|+1) [Taylor shift of the parent's expansion by
// d = z_child - z_parent (Eq. L2L)]_n, rho = 1/2: the parent's full
// components, three one-axis Taylor shifts with s = d/h_P, truncated at
// rank P.  One wavefront per node of [first, first+count) (level >= 1).
template <int P>
__global__ __launch_bounds__(64) void k_dual_l2l(int first, ATree t, const double4* __restrict__ zr, DevTables T,
                                                 double* __restrict__ L) {
    constexpr int nc = (P + 1) * (P + 1);
    constexpr int nf = (P + 1) * (P + 2) * (P + 3) / 6;
    constexpr int ldm = ldm_of(P);
    const int g = first + blockIdx.x;
    const int par = t.par[g];
    __shared__ double X[nf], Y[nf];
    const int lane = threadIdx.x;
    const double4 zp = zr[par], zc = zr[g];
    const double ih = 1.0 / t.geo[par].w;
    expand_full<P>(L + (size_t)par * ldm, false, T, X);
    __syncthreads();
    shift_axis<P, true>(0, (zc.x - zp.x) * ih, X, Y, false, T);
    __syncthreads();
    shift_axis<P, true>(1, (zc.y - zp.y) * ih, Y, X, false, T);
    __syncthreads();
    shift_axis<P, true>(2, (zc.z - zp.z) * ih, X, Y, false, T);
    __syncthreads();
    for (int n = lane; n < nc; n += 64) {
        const int a = T.ind[3 * n], b = T.ind[3 * n + 1], c = T.ind[3 * n + 2];
        L[(size_t)g * ldm + n] += ldexp(Y[fidx(a, b, c)], -(a + b + c + 1));
    }
}

void launch_dual_p2m(hipStream_t s, int p, int nn, const ATree& t, const double4* zr, const double4* P,
                     const DevTables& T, double* M) {
    if (nn <= 0) return;
    switch (p) {
#define CASE(PP) case PP: hipLaunchKernelGGL(k_dual_p2m<PP>, dim3(nn), dim3(64), 0, s, t, zr, P, T, M); break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

void launch_dual_m2m(hipStream_t s, int p, int first, int count, const ATree& t, const double4* zr,
                     const DevTables& T, double* M) {
    if (count <= 0) return;
    switch (p) {
#define CASE(PP) case PP: hipLaunchKernelGGL(k_dual_m2m<PP>, dim3(count), dim3(M2M_B), 0, s, first, t, zr, T, M); break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

void launch_dual_l2l(hipStream_t s, int p, int first, int count, const ATree& t, const double4* zr,
                     const DevTables& T, double* L) {
    if (count <= 0) return;
    switch (p) {
#define CASE(PP) case PP: hipLaunchKernelGGL(k_dual_l2l<PP>, dim3(count), dim3(64), 0, s, first, t, zr, T, L); break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

// ------------------------------------------------------------------ traversal

// cnt[r]: pairs of round r's frontier (cnt[0] = 1: the root with itself);
// cnt[nr + 1]: directed M2L entries; cnt[nr + 2]: ordered direct leaf pairs
__global__ void k_dual_init(int nr, int* __restrict__ cnt, int2* __restrict__ front) {
    for (int k = threadIdx.x; k < nr + 3; k += blockDim.x) cnt[k] = k == 0 ? 1 : 0;
    if (threadIdx.x == 0) front[0] = make_int2(0, 0);
}

// One round.  Entries past a buffer's capacity are counted but not written
// (the host then grows the buffers and runs the traversal again).  M2L
// entries are keys (target << sh) | source, direct pairs (leaf << sh) |
// partner.  A workgroup takes DW_B * DW_I pairs at a time, DW_I consecutive
// ones per thread, and reserves its room in each output with one atomic.
constexpr int DW_B = 256, DW_I = 16;

struct PairStep {
    int kind;   // 0 none, 1 M2L, 2 direct, 3 open node o against other, 4 split a self pair
    int a, b, o, other, nch;
};

__device__ inline PairStep pair_step(int i, int nin, const int2* __restrict__ fin, const ATree& t,
                                     const double4* __restrict__ zr, double theta) {
    PairStep q{0, 0, 0, 0, 0, 0};
    if (i >= nin) return q;
    const int2 pr = fin[i];
    q.a = pr.x;
    q.b = pr.y;
    const bool la = leaf_d(t.info[q.a]), lb = leaf_d(t.info[q.b]);
    if (q.a == q.b) {
        q.kind = la ? 2 : 4;
        q.o = q.a;
    } else {
        const double4 A = zr[q.a], B = zr[q.b];
        const double dist = norm_plain(B.x - A.x, B.y - A.y, B.z - A.z);
        if (theta * dist > A.w + B.w) {
            q.kind = 1;
        } else if (la && lb) {
            q.kind = 2;
        } else {
            const bool open_a = !la && (lb || A.w >= B.w);
            q.kind = 3;
            q.o = open_a ? q.a : q.b;
            q.other = open_a ? q.b : q.a;
        }
    }
    if (q.kind >= 3)
        for (int k = 0; k < 8; ++k) q.nch += t.child[8 * q.o + k] >= 0;
    return q;
}

__global__ __launch_bounds__(DW_B) void k_dual_round(int r, int nr, const int2* __restrict__ fin,
                                                     int2* __restrict__ fout, int cap_f, uint64_t* __restrict__ mk,
                                                     int cap_m, uint64_t* __restrict__ pk, int cap_p, int sh,
                                                     int* __restrict__ cnt, ATree t, const double4* __restrict__ zr,
                                                     double theta) {
    const int nin = min(cnt[r], cap_f);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    __shared__ int wtot[3][DW_B / 64];
    __shared__ int bbase[3];
    for (long long c0 = (long long)blockIdx.x * DW_B * DW_I; c0 < nin; c0 += (long long)gridDim.x * DW_B * DW_I) {
        const int i0 = (int)c0 + tid * DW_I;
        int tf = 0, tm = 0, tp = 0;
#pragma unroll 4
        for (int k = 0; k < DW_I; ++k) {
            const PairStep q = pair_step(i0 + k, nin, fin, t, zr, theta);
            tf += q.kind == 3 ? q.nch : (q.kind == 4 ? q.nch * (q.nch + 1) / 2 : 0);
            tm += q.kind == 1 ? 2 : 0;
            tp += q.kind == 2 ? (q.a == q.b ? 1 : 2) : 0;
        }
        // exclusive positions of this thread's entries within the workgroup
        int v[3] = {tf, tm, tp};
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            int incl = v[x];
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int o = __shfl_up(incl, d);
                if (lane >= d) incl += o;
            }
            if (lane == 63) wtot[x][wv] = incl;
            v[x] = incl - v[x];
        }
        __syncthreads();
        if (tid < 3) {
            int tot = 0;
            for (int w = 0; w < DW_B / 64; ++w) tot += wtot[tid][w];
            const int ctr = tid == 0 ? r + 1 : nr + tid;
            bbase[tid] = tot > 0 ? atomicAdd(&cnt[ctr], tot) : 0;
        }
        __syncthreads();
        int pf = bbase[0] + v[0], pm = bbase[1] + v[1], pp = bbase[2] + v[2];
        for (int w = 0; w < wv; ++w) {
            pf += wtot[0][w];
            pm += wtot[1][w];
            pp += wtot[2][w];
        }
        for (int k = 0; k < DW_I; ++k) {
            const PairStep q = pair_step(i0 + k, nin, fin, t, zr, theta);
            if (q.kind == 1) {
                if (pm + 1 < cap_m) {
                    mk[pm] = ((uint64_t)q.b << sh) | (uint64_t)q.a;      // A -> B
                    mk[pm + 1] = ((uint64_t)q.a << sh) | (uint64_t)q.b;  // B -> A
                }
                pm += 2;
            } else if (q.kind == 2) {
                if (pp < cap_p) pk[pp] = ((uint64_t)q.a << sh) | (uint64_t)q.b;
                if (q.a != q.b && pp + 1 < cap_p) pk[pp + 1] = ((uint64_t)q.b << sh) | (uint64_t)q.a;
                pp += q.a == q.b ? 1 : 2;
            } else if (q.kind == 3) {
                for (int k2 = 0; k2 < 8; ++k2) {
                    const int c = t.child[8 * q.o + k2];
                    if (c < 0) continue;
                    if (pf < cap_f) fout[pf] = q.o == q.a ? make_int2(c, q.other) : make_int2(q.other, c);
                    ++pf;
                }
            } else if (q.kind == 4) {
                for (int x = 0; x < 8; ++x) {
                    const int cx = t.child[8 * q.o + x];
                    if (cx < 0) continue;
                    for (int y = x; y < 8; ++y) {
                        const int cy = t.child[8 * q.o + y];
                        if (cy < 0) continue;
                        if (pf < cap_f) fout[pf] = make_int2(cx, cy);
                        ++pf;
                    }
                }
            }
        }
        __syncthreads();  // wtot and bbase are rewritten by the next chunk
    }
}

void launch_dual_init(hipStream_t s, int nr, int* cnt, int2* front) {
    hipLaunchKernelGGL(k_dual_init, dim3(1), dim3(64), 0, s, nr, cnt, front);
}

void launch_dual_round(hipStream_t s, int r, int nr, const int2* fin, int2* fout, int cap_f, uint64_t* mk, int cap_m,
                       uint64_t* pk, int cap_p, int sh, int* cnt, const ATree& t, const double4* zr, double theta) {
    // enough workgroups for the largest frontiers; smaller rounds exit early
    hipLaunchKernelGGL(k_dual_round, dim3(1024), dim3(DW_B), 0, s, r, nr, fin, fout, cap_f, mk, cap_m, pk, cap_p, sh,
                       cnt, t, zr, theta);
}

// off[g] = first sorted key with (key >> sh) >= g, g in [0, nn]; src[i] = the
// low sh bits of key i
__global__ void k_dual_csr(int nn, const uint64_t* __restrict__ keys, const int* __restrict__ nkeys_p, int cap,
                           int sh, int32_t* __restrict__ off, int32_t* __restrict__ src) {
    const int nk = min(*nkeys_p, cap);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= nn) {
        const uint64_t target = (uint64_t)i << sh;
        int lo = 0, hi = nk;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (keys[mid] < target) lo = mid + 1; else hi = mid;
        }
        off[i] = lo;
    }
    const uint64_t mask = (sh >= 64) ? ~0ull : ((1ull << sh) - 1);
    for (int k = i; k < nk; k += gridDim.x * blockDim.x) src[k] = (int32_t)(keys[k] & mask);
}

void launch_dual_csr(hipStream_t s, int nn, const uint64_t* keys, const int* nkeys, int cap, int sh, int32_t* off,
                     int32_t* src) {
    hipLaunchKernelGGL(k_dual_csr, dim3(cdiv(nn + 1, 256)), dim3(256), 0, s, nn, keys, nkeys, cap, sh, off, src);
}

// ------------------------------------------------------------------ M2L

// Outputs of ranks R0..R1 of every target node g (one wavefront each): its
// sources off[g]..off[g+1] go to the lanes in turn; each lane forms
// D(u), u = (z_T - z_S)/h_T, and adds the contraction of Eq. M2L with the
// source multipole scaled by rho^|j|, rho = h_S/h_T.  Every node's outputs
// are written (zero without sources).
template <int P, int R0, int R1, bool AP>
__global__ __launch_bounds__(64) void k_dual_m2l(ATree t, const double4* __restrict__ zr, const int32_t* __restrict__ off,
                                                 const int32_t* __restrict__ src, const double* __restrict__ M,
                                                 double* __restrict__ L) {
    constexpr int NL = (R1 + 1) * (R1 + 1) - R0 * R0;
    constexpr int ldm = ldm_of(P);
    constexpr int nc = (P + 1) * (P + 1);
    const int g = blockIdx.x;
    const int lane = threadIdx.x;
    const int b = off[g], e = off[g + 1];
    const double4 zt = zr[g];
    const double iht = 1.0 / t.geo[g].w;
    double acc[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) acc[k] = 0.0;
    for (int i = b + lane; i < e; i += 64) {
        const int s = src[i];
        const double4 zs = zr[s];
        const double rho = t.geo[s].w * iht;
        double rp[P + 1];
        rp[0] = 1.0;
#pragma unroll
        for (int k = 1; k <= P; ++k) rp[k] = rp[k - 1] * rho;
        double D[nc];
        gen_dtensor<P>((zt.x - zs.x) * iht, (zt.y - zs.y) * iht, (zt.z - zs.z) * iht, D);
        gen_m2l_pair<P, R0, R1, AP>(D, M + (size_t)s * ldm, rp, acc);
    }
    double* Lg = L + (size_t)g * ldm;
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        double v = acc[k];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
        if ((k & 63) == lane) Lg[R0 * R0 + k] = v;
    }
    if (R1 == P && lane < ldm - nc) Lg[nc + lane] = 0.0;  // padding
}

template <int P, bool AP>
void dual_m2l_passes(hipStream_t s, int nn, const ATree& t, const double4* zr, const int32_t* off, const int32_t* src,
                     const double* M, double* L) {
    // output ranks per pass, so that D and the pass's sums stay in registers
    // (narrower passes lower the register count but recompute D more often,
    // which measured slower)
#define PASS(A, B) hipLaunchKernelGGL((k_dual_m2l<P, A, B, AP>), dim3(nn), dim3(64), 0, s, t, zr, off, src, M, L)
    if constexpr (P <= 6) {
        PASS(0, P);
    } else if constexpr (P == 7) {
        PASS(0, 3); PASS(4, 7);
    } else if constexpr (P == 8) {
        PASS(0, 3); PASS(4, 5); PASS(6, 8);
    } else if constexpr (P == 9) {
        PASS(0, 2); PASS(3, 5); PASS(6, 7); PASS(8, 9);
    } else {
        PASS(0, 2); PASS(3, 4); PASS(5, 6); PASS(7, 8); PASS(9, 10);
    }
#undef PASS
}

void launch_dual_m2l(hipStream_t s, int p, bool ap, int nn, const ATree& t, const double4* zr, const int32_t* off,
                     const int32_t* src, const double* M, double* L) {
    if (nn <= 0) return;
    switch (p) {
#define CASE(PP)                                                                   \
    case PP:                                                                       \
        if (ap) dual_m2l_passes<PP, true>(s, nn, t, zr, off, src, M, L);           \
        else dual_m2l_passes<PP, false>(s, nn, t, zr, off, src, M, L);             \
        break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

// ------------------------------------------------------------------ L2P

// the far field of sorted particle s from its leaf's local expansion (Eq.
// L2P, nested Horner over the full polynomial coefficients) plus its near
// field Fn[s], written in input order; AP: the gradient only (phi is not
// written; the Horner scheme still carries the potential, which the
// gradient's recurrences use)
template <int P, bool AP>
__global__ __launch_bounds__(256) void k_dual_l2p(int n, ATree t, const int32_t* __restrict__ leaf_of,
                                                  const double4* __restrict__ zr, const double4* __restrict__ Pt,
                                                  const double* __restrict__ L, const double4* __restrict__ Fn,
                                                  const int32_t* __restrict__ idx, double* __restrict__ phi,
                                                  double* __restrict__ grad) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int B = leaf_of[s];
    const double4 pt = Pt[s];
    const double4 z = zr[B];
    const double h = t.geo[B].w;
    const double ih = 1.0 / h;
    double lf = 0.0, lx = 0.0, ly = 0.0, lz = 0.0;
    // (always taken: without the branch the compiler schedules the
    // polynomial's coefficient loads ahead and the kernel spills)
    if (h > 0.0)
        gen_l2p_hg<P>((pt.x - z.x) * ih, (pt.y - z.y) * ih, (pt.z - z.z) * ih, L + (size_t)B * ldm_of(P), lf, lx,
                      ly, lz);
    const double ih2 = ih * ih;
    const double4 nf = Fn[s];
    const size_t o = (size_t)idx[s];
    if (!AP && phi) phi[o] = lf * ih + nf.x;
    if (grad) {
        grad[3 * o] = lx * ih2 + nf.y;
        grad[3 * o + 1] = ly * ih2 + nf.z;
        grad[3 * o + 2] = lz * ih2 + nf.w;
    }
}

void launch_dual_l2p(hipStream_t s, int p, bool ap, int n, const ATree& t, const int32_t* leaf_of, const double4* zr,
                     const double4* P, const double* L, const double4* Fn, const int32_t* idx, double* phi,
                     double* grad) {
    if (n <= 0) return;
    const dim3 grid(cdiv(n, 256)), blk(256);
    switch (p) {
#define CASE(PP)                                                                                                   \
    case PP:                                                                                                       \
        if (ap) hipLaunchKernelGGL((k_dual_l2p<PP, true>), grid, blk, 0, s, n, t, leaf_of, zr, P, L, Fn, idx, phi, \
                                   grad);                                                                          \
        else hipLaunchKernelGGL((k_dual_l2p<PP, false>), grid, blk, 0, s, n, t, leaf_of, zr, P, L, Fn, idx, phi,   \
                                grad);                                                                             \
        break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

}  // namespace ctfmm
