// Dual-tree FMM of libctfmm (gfx950): the driver of Appendix C on the
// adaptive octree of ctfmm_adaptive.hip.
//
//   centres   every node's expansion centre z (its geometric centre, or the
//             charge-weighted mean of its particles) and enclosing radius r
//             (the largest distance from z to one of its particles);
//   upward    P2M at the leaves about z (Eq. P2M), then M2M to the parents
//             with the shift z_child - z_parent (Eq. M2M) level by level;
//   traversal from the pair (root, root), in rounds: a round takes every
//             pair of its frontier and either accepts it (theta |z_B - z_A|
//             > r_A + r_B: two directed M2L entries), sums it directly (two
//             leaves), or opens the node of larger radius (never a leaf) and
//             puts its children's pairs into the next frontier; a node paired
//             with itself gives its children's self pairs and each two
//             children once.  The entries are appended with one atomic per
//             wavefront and sorted afterwards, so the lists (and every sum
//             over them) do not depend on the order of the appends;
//   M2L       per target node, its sources in ascending order, one lane per
//             source: the traceless gradient of 1/r at the pair's offset and
//             the contraction of Eq. M2L, both straight-line generated code;
//             the lanes' sums are added by a butterfly (the same total on
//             every lane);
//   downward  L2L from each parent to its children (Eq. L2L), L2P at the
//             leaves (Eq. L2P); the direct part by the leaf-pair kernel of
//             the adaptive tree.
// Scaled expansions per node: M~_n = M_n / h^|n| and L~_n = L_n h^(|n|+1)
// with h the node's cube side.  The AP variant (Sec. 4: centre of mass,
// positive charges) leaves the dipole out of every M2L and computes the
// gradient only.
#include <math.h>

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

// wavefront-wide exclusive position of this lane's cnt entries in a buffer
// whose fill counter is *ctr (one atomic per wavefront); every lane calls it
__device__ inline int wave_append(int* ctr, int cnt) {
    const int lane = threadIdx.x & 63;
    int incl = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(incl, d);
        if (lane >= d) incl += o;
    }
    const int tot = __shfl(incl, 63);
    int base = 0;
    if (lane == 63 && tot > 0) base = atomicAdd(ctr, tot);
    base = __shfl(base, 63);
    return base + incl - cnt;
}

}  // namespace

// ------------------------------------------------------------------ centres and radii

// One workgroup per node.  mode 0: geometric centre; 1 and 2: the
// charge-weighted mean where the node's total charge is positive (else the
// geometric centre); 2 (AP) also flags a non-positive charge (bit 2 of err).
constexpr int DC_B = 256;
__global__ __launch_bounds__(DC_B) void k_dual_centres(ATree t, const ABox* __restrict__ boxes,
                                                       const double4* __restrict__ P, int mode,
                                                       double4* __restrict__ zr, int* __restrict__ err) {
    const int g = blockIdx.x;
    const int b = t.pb[g], e = t.pe[g];
    __shared__ double red[4][DC_B];
    __shared__ double zc[3];
    const int tid = threadIdx.x;
    if (tid == 0) cube_centre(boxes[t.sys[g]], t.key[g], t.info[g] & 0xff, zc);
    if (mode != 0) {
        double w = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
        bool bad = false;
        for (int s = b + tid; s < e; s += DC_B) {
            const double4 pt = P[s];
            w += pt.w;
            sx += pt.w * pt.x;
            sy += pt.w * pt.y;
            sz += pt.w * pt.z;
            bad |= !(pt.w > 0.0);
        }
        if (mode == 2 && bad) atomicOr(err, 2);
        red[0][tid] = w;
        red[1][tid] = sx;
        red[2][tid] = sy;
        red[3][tid] = sz;
        __syncthreads();
        for (int h = DC_B / 2; h > 0; h >>= 1) {
            if (tid < h)
#pragma unroll
                for (int k = 0; k < 4; ++k) red[k][tid] += red[k][tid + h];
            __syncthreads();
        }
        if (tid == 0 && red[0][0] > 0.0) {
            zc[0] = red[1][0] / red[0][0];
            zc[1] = red[2][0] / red[0][0];
            zc[2] = red[3][0] / red[0][0];
        }
    }
    __syncthreads();
    const double zx = zc[0], zy = zc[1], zz = zc[2];
    double r = 0.0;
    for (int s = b + tid; s < e; s += DC_B) {
        const double4 pt = P[s];
        r = fmax(r, norm_plain(pt.x - zx, pt.y - zy, pt.z - zz));
    }
    __syncthreads();  // red is reused
    red[0][tid] = r;
    __syncthreads();
    for (int h = DC_B / 2; h > 0; h >>= 1) {
        if (tid < h) red[0][tid] = fmax(red[0][tid], red[0][tid + h]);
        __syncthreads();
    }
    if (tid == 0) zr[g] = make_double4(zx, zy, zz, red[0][0]);
}

void launch_dual_centres(hipStream_t s, int nn, const ATree& t, const ABox* boxes, const double4* P, int mode,
                         double4* zr, int* err) {
    if (nn <= 0) return;
    hipLaunchKernelGGL(k_dual_centres, dim3(nn), dim3(DC_B), 0, s, t, boxes, P, mode, zr, err);
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

// the monomials (d/h)^f of the full components f, |f| <= P, into mono
template <int P>
__device__ inline void monomials(double dx, double dy, double dz, const DevTables& T, double* mono) {
    constexpr int nf = (P + 1) * (P + 2) * (P + 3) / 6;
    for (int f = threadIdx.x; f < nf; f += 64) {
        const int a = T.full[3 * f], b = T.full[3 * f + 1], c = T.full[3 * f + 2];
        double v = 1.0;
        for (int k = 0; k < a; ++k) v *= dx;
        for (int k = 0; k < b; ++k) v *= dy;
        for (int k = 0; k < c; ++k) v *= dz;
        mono[f] = v;
    }
}

// M~(parent) = sum over its children, in octant order, of the shift of
// Eq. M2M with d = z_child - z_parent and rho = 1/2:
//   M~_n += sum_t COEF[t] (d/h_P)^MONO[t] rho^|J[t]| M~child_J[t]
// One wavefront per non-leaf node of [first, first+count); lanes over n.
template <int P>
__global__ __launch_bounds__(64) void k_dual_m2m(int first, ATree t, const double4* __restrict__ zr, DevTables T,
                                                 double* __restrict__ M) {
    constexpr int nc = (P + 1) * (P + 1);
    constexpr int nf = (P + 1) * (P + 2) * (P + 3) / 6;
    constexpr int ldm = ldm_of(P);
    const int g = first + blockIdx.x;
    if (leaf_d(t.info[g])) return;
    __shared__ double mono[nf];
    __shared__ double mc[nc];
    const int lane = threadIdx.x;
    const double4 zp = zr[g];
    const double ih = 1.0 / t.geo[g].w;
    double acc[2] = {0.0, 0.0};
    for (int o = 0; o < 8; ++o) {
        const int c = t.child[8 * g + o];
        if (c < 0) continue;
        __syncthreads();  // the previous child's tables are read
        const double4 zc = zr[c];
        monomials<P>((zc.x - zp.x) * ih, (zc.y - zp.y) * ih, (zc.z - zp.z) * ih, T, mono);
        for (int j = lane; j < nc; j += 64) mc[j] = ldexp(M[(size_t)c * ldm + j], -rank_d(j));
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int n = lane + 64 * k;
            if (n >= nc) break;
            double v = 0.0;
            const int t1 = T.m2mg_start[n + 1];
            for (int q = T.m2mg_start[n]; q < t1; ++q) v += T.m2mg_coef[q] * mono[T.m2mg_mono[q]] * mc[T.m2mg_j[q]];
            acc[k] += v;
        }
    }
    for (int k = 0; k < 2; ++k) {
        const int n = lane + 64 * k;
        if (n < ldm) M[(size_t)g * ldm + n] = n < nc ? acc[k] : 0.0;
    }
}

// L~(child) += rho^(|n|+1) sum_t COEF[t] (d/h_P)^MONO[t] L~parent_J[t]
// (Eq. L2L), d = z_child - z_parent, rho = 1/2, terms with rank(J) > P left
// out.  One wavefront per node of [first, first+count) (level >= 1).
template <int P>
__global__ __launch_bounds__(64) void k_dual_l2l(int first, ATree t, const double4* __restrict__ zr, DevTables T,
                                                 double* __restrict__ L) {
    constexpr int nc = (P + 1) * (P + 1);
    constexpr int nf = (P + 1) * (P + 2) * (P + 3) / 6;
    constexpr int ldm = ldm_of(P);
    const int g = first + blockIdx.x;
    const int par = t.par[g];
    __shared__ double mono[nf];
    __shared__ double lp[nc];
    const int lane = threadIdx.x;
    const double4 zp = zr[par], zc = zr[g];
    const double ih = 1.0 / t.geo[par].w;
    monomials<P>((zc.x - zp.x) * ih, (zc.y - zp.y) * ih, (zc.z - zp.z) * ih, T, mono);
    for (int j = lane; j < nc; j += 64) lp[j] = L[(size_t)par * ldm + j];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int n = lane + 64 * k;
        if (n >= nc) break;
        double v = 0.0;
        const int t1 = T.l2lg_start[n + 1];
        for (int q = T.l2lg_start[n]; q < t1; ++q) {
            const int j = T.l2lg_j[q];
            if (j >= nc) break;  // terms are ordered by J
            v += T.l2lg_coef[q] * mono[T.l2lg_mono[q]] * lp[j];
        }
        L[(size_t)g * ldm + n] += ldexp(v, -(rank_d(n) + 1));
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
#define CASE(PP) case PP: hipLaunchKernelGGL(k_dual_m2m<PP>, dim3(count), dim3(64), 0, s, first, t, zr, T, M); break;
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
// partner.
constexpr int DW_B = 256;
__global__ __launch_bounds__(DW_B) void k_dual_round(int r, int nr, const int2* __restrict__ fin,
                                                     int2* __restrict__ fout, int cap_f, uint64_t* __restrict__ mk,
                                                     int cap_m, uint64_t* __restrict__ pk, int cap_p, int sh,
                                                     int* __restrict__ cnt, ATree t, const double4* __restrict__ zr,
                                                     double theta) {
    const int nin = min(cnt[r], cap_f);
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * DW_B + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * DW_B) >> 6;
    for (int i0 = wave * 64; i0 < nin; i0 += nwaves * 64) {
        const int i = i0 + lane;
        int kind = 0;  // 0 none, 1 M2L, 2 direct, 3 open node o against other
        int a = 0, b = 0, o = 0, other = 0, nch = 0;
        int ch[8];
        if (i < nin) {
            const int2 pr = fin[i];
            a = pr.x;
            b = pr.y;
            const bool la = leaf_d(t.info[a]), lb = leaf_d(t.info[b]);
            if (a == b) {
                kind = la ? 2 : 4;
                o = a;
            } else {
                const double4 A = zr[a], B = zr[b];
                const double dist = norm_plain(B.x - A.x, B.y - A.y, B.z - A.z);
                if (theta * dist > A.w + B.w) {
                    kind = 1;
                } else if (la && lb) {
                    kind = 2;
                } else {
                    const bool open_a = !la && (lb || A.w >= B.w);
                    kind = 3;
                    o = open_a ? a : b;
                    other = open_a ? b : a;
                }
            }
            if (kind >= 3)
                for (int k = 0; k < 8; ++k) {
                    const int c = t.child[8 * o + k];
                    if (c >= 0) ch[nch++] = c;
                }
        }
        const int nf = kind == 3 ? nch : (kind == 4 ? nch * (nch + 1) / 2 : 0);
        const int nm = kind == 1 ? 2 : 0;
        const int np = kind == 2 ? (a == b ? 1 : 2) : 0;
        const int bf = wave_append(&cnt[r + 1], nf);
        const int bm = wave_append(&cnt[nr + 1], nm);
        const int bp = wave_append(&cnt[nr + 2], np);
        if (kind == 1 && bm + 1 < cap_m) {
            mk[bm] = ((uint64_t)b << sh) | (uint64_t)a;  // A -> B
            mk[bm + 1] = ((uint64_t)a << sh) | (uint64_t)b;  // B -> A
        }
        if (kind == 2) {
            if (bp < cap_p) pk[bp] = ((uint64_t)a << sh) | (uint64_t)b;
            if (np == 2 && bp + 1 < cap_p) pk[bp + 1] = ((uint64_t)b << sh) | (uint64_t)a;
        }
        if (kind == 3) {
            for (int k = 0; k < nch; ++k)
                if (bf + k < cap_f) fout[bf + k] = o == a ? make_int2(ch[k], other) : make_int2(other, ch[k]);
        }
        if (kind == 4) {
            int w = bf;
            for (int x = 0; x < nch; ++x)
                for (int y = x; y < nch; ++y, ++w)
                    if (w < cap_f) fout[w] = make_int2(ch[x], ch[y]);
        }
    }
}

void launch_dual_init(hipStream_t s, int nr, int* cnt, int2* front) {
    hipLaunchKernelGGL(k_dual_init, dim3(1), dim3(64), 0, s, nr, cnt, front);
}

void launch_dual_round(hipStream_t s, int r, int nr, const int2* fin, int2* fout, int cap_f, uint64_t* mk, int cap_m,
                       uint64_t* pk, int cap_p, int sh, int* cnt, const ATree& t, const double4* zr, double theta) {
    // enough wavefronts for the largest frontiers; smaller rounds exit early
    hipLaunchKernelGGL(k_dual_round, dim3(2048), dim3(DW_B), 0, s, r, nr, fin, fout, cap_f, mk, cap_m, pk, cap_p, sh,
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
// L2P) plus its near field Fn[s], written in input order; AP: the gradient
// only (the potential's terms are dead code and phi is not written)
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
    gen_l2p<P>((pt.x - z.x) * ih, (pt.y - z.y) * ih, (pt.z - z.z) * ih, L + (size_t)B * ldm_of(P), lf, lx, ly, lz);
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
