// Device kernels of libctfmm (gfx950): tree keys, P2M, M2M, per-offset M2L
// operator matrices, M2L, L2L, L2P and the P2P near field.
//
// Expansions are stored in scaled form on a Morton-ordered uniform octree:
// level l holds 8^l cells, cell m at M[(m * ldm) + k] with nc = (p+1)^2
// independent traceless components k (ordered by rank, then n_z, then n_x
// descending) and rows padded to ldm = nc rounded up to a multiple of 4.  With h the cell side, M~_k = M_k / h^|k| and
// L~_k = L_k h^(|k|+1); then the M2L operator of an integer offset v is the
// same at every level (grad^n r^-1 is homogeneous of degree -n-1) and the
// M2M/L2L shifts are constant per octant.
#include <math.h>
#include <algorithm>

#include "ctfmm_internal.h"

namespace ctfmm {

static inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// rank of independent slot k (rank n occupies slots n^2 .. (n+1)^2 - 1)
__device__ inline int rank_of(int k) {
    int r = 0;
    while ((r + 1) * (r + 1) <= k) ++r;
    return r;
}

// ------------------------------------------------------------------ tree

// leaf coordinate floor((x - lo)/side * 2^d), clamped to [0, 2^d - 1]
__device__ inline uint32_t leaf_coord(double x, double lo, double side, int d) {
    const double s = floor((x - lo) / side * (double)(1 << d));
    const int n1 = 1 << d;
    if (!(s >= 0.0)) return 0u;
    if (s > (double)(n1 - 1)) return (uint32_t)(n1 - 1);
    return (uint32_t)s;
}

__global__ void k_keys(int n, const double* __restrict__ xyz, Box box, uint32_t* __restrict__ keys,
                       int32_t* __restrict__ idx, int* __restrict__ err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = xyz[3 * (size_t)i], y = xyz[3 * (size_t)i + 1], z = xyz[3 * (size_t)i + 2];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) atomicOr(err, 1);
    const uint32_t ix = leaf_coord(x, box.lo[0], box.side, box.depth);
    const uint32_t iy = leaf_coord(y, box.lo[1], box.side, box.depth);
    const uint32_t iz = leaf_coord(z, box.lo[2], box.side, box.depth);
    keys[i] = morton3(ix, iy, iz);
    idx[i] = i;
}

void launch_keys(hipStream_t s, int n, const double* xyz, Box box, uint32_t* keys, int32_t* idx, int* err) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_keys, dim3(cdiv(n, 256)), dim3(256), 0, s, n, xyz, box, keys, idx, err);
}

__global__ void k_gather(int n, const int32_t* __restrict__ idx, const double* __restrict__ xyz,
                         const double* __restrict__ q, double4* __restrict__ P) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const size_t i = (size_t)idx[s];
    P[s] = make_double4(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], q[i]);
}

void launch_gather(hipStream_t s, int n, const int32_t* idx, const double* xyz, const double* q, double4* P) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather, dim3(cdiv(n, 256)), dim3(256), 0, s, n, idx, xyz, q, P);
}

__global__ void k_gather_dip(int n, const int32_t* __restrict__ idx, const double* __restrict__ dip,
                             double4* __restrict__ Pd) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const size_t i = (size_t)idx[s];
    Pd[s] = make_double4(dip[3 * i], dip[3 * i + 1], dip[3 * i + 2], 0.0);
}

void launch_gather_dip(hipStream_t s, int n, const int32_t* idx, const double* dip, double4* Pd) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_dip, dim3(cdiv(n, 256)), dim3(256), 0, s, n, idx, dip, Pd);
}

// start[c] = first sorted position whose key is >= c (c = 0..nleaves)
__global__ void k_leaf_start(int nleaves, const uint32_t* __restrict__ keys, int n, int32_t* __restrict__ start) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nleaves) return;
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        if (keys[mid] < (uint32_t)c) lo = mid + 1; else hi = mid;
    }
    start[c] = lo;
}

void launch_leaf_start(hipStream_t s, int nleaves, const uint32_t* keys, int n, int32_t* start) {
    hipLaunchKernelGGL(k_leaf_start, dim3(cdiv(nleaves + 1, 256)), dim3(256), 0, s, nleaves, keys, n, start);
}

// ------------------------------------------------------------------ P2M

// One wavefront per leaf (the P2M of p2m_cell, ctfmm_internal.h).
template <int PP, bool DIP>
__global__ __launch_bounds__(64) void k_p2m(Box box, const int32_t* __restrict__ start,
                                            const double4* __restrict__ P, DevTables T, double* __restrict__ M,
                                            const double4* __restrict__ Pd) {
    const uint32_t c = blockIdx.x;
    const double h = box.side / (double)(1 << box.depth);
    const double zx = box.lo[0] + ((double)compact3(c) + 0.5) * h;
    const double zy = box.lo[1] + ((double)compact3(c >> 1) + 0.5) * h;
    const double zz = box.lo[2] + ((double)compact3(c >> 2) + 0.5) * h;
    // uniform leaves hold few particles: 16 are staged at a time
    p2m_cell<PP, DIP, 16>(zx, zy, zz, h, start[c], start[c + 1], P, T, M + (size_t)c * ldm_of(PP), Pd);
}

// the independent components of ranks N .. N1 from their moments S (rank by
// rank, each rank's (N+1)(N+2)/2 sums in turn)
template <int N, int N1>
__device__ __forceinline__ void p2m_lane_store(const double* S, double* __restrict__ Mc) {
    if constexpr (N <= N1) {
        double out[2 * N + 1];
        gen_det_rank<N>(S, out);
#pragma unroll
        for (int k = 0; k < 2 * N + 1; ++k) Mc[N * N + k] = out[k];
        p2m_lane_store<N + 1, N1>(S + (N + 1) * (N + 2) / 2, Mc);
    }
}

// P2M of the uniform tree without dipoles, one thread per leaf (leaves hold
// few particles): for a group of ranks N0..N1 at a time, the full monomial
// moments S_f = sum_a q_a u_a^f, u = (z - x)/h, |f| = N, are summed in
// registers over one pass through the leaf's particles, and each rank's are
// mapped to its independent components by the generated detracer rows
// (Eq. P2M with Eq. Detracer).  A group holds at most 66 sums (rank 10 alone),
// so p = 10 takes five passes over the particles instead of eleven.  The
// padding of each row is written as zero.
__host__ __device__ constexpr int p2m_nf(int n) { return (n + 1) * (n + 2) / 2; }
__host__ __device__ constexpr int p2m_group_end(int n0, int p) {
    int n1 = n0, tot = p2m_nf(n0);
    while (n1 < p && tot + p2m_nf(n1 + 1) <= 66) tot += p2m_nf(++n1);
    return n1;
}
template <int P, int N0>
__device__ __forceinline__ void p2m_lane_rank(double zx, double zy, double zz, double h, int b, int e,
                                              const double4* __restrict__ Pt, double* __restrict__ Mc) {
    if constexpr (N0 <= P) {
        constexpr int N1 = p2m_group_end(N0, P);
        constexpr int NS = (N1 + 1) * (N1 + 2) * (N1 + 3) / 6 - N0 * (N0 + 1) * (N0 + 2) / 6;
        double S[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) S[k] = 0.0;
        for (int i = b; i < e; ++i) {
            const double4 pt = Pt[i];
            const double ux = (zx - pt.x) / h, uy = (zy - pt.y) / h, uz = (zz - pt.z) / h;
            double px[N1 + 1], py[N1 + 1], pz[N1 + 1];
            px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
            for (int k = 1; k <= N1; ++k) {
                px[k] = px[k - 1] * ux;
                py[k] = py[k - 1] * uy;
                pz[k] = pz[k - 1] * uz;
            }
            // per rank, full-slot order: x exponent, then y exponent, descending
            int f = 0;
#pragma unroll
            for (int N = N0; N <= N1; ++N)
#pragma unroll
                for (int a = N; a >= 0; --a) {
                    const double t = pt.w * px[a];
#pragma unroll
                    for (int c = N - a; c >= 0; --c) {
                        S[f] = fma(t * py[c], pz[N - a - c], S[f]);
                        ++f;
                    }
                }
        }
        p2m_lane_store<N0, N1>(S, Mc);
        p2m_lane_rank<P, N1 + 1>(zx, zy, zz, h, b, e, Pt, Mc);
    }
}
template <int PP>
__global__ __launch_bounds__(256) void k_p2m_lane(Box box, const int32_t* __restrict__ start,
                                                  const double4* __restrict__ P, double* __restrict__ M) {
    const long long nleaves = 1ll << (3 * box.depth);
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nleaves) return;
    const double h = box.side / (double)(1 << box.depth);
    const double zx = box.lo[0] + ((double)compact3((uint32_t)c) + 0.5) * h;
    const double zy = box.lo[1] + ((double)compact3((uint32_t)c >> 1) + 0.5) * h;
    const double zz = box.lo[2] + ((double)compact3((uint32_t)c >> 2) + 0.5) * h;
    double* Mc = M + (size_t)c * ldm_of(PP);
    p2m_lane_rank<PP, 0>(zx, zy, zz, h, start[c], start[c + 1], P, Mc);
#pragma unroll
    for (int k = (PP + 1) * (PP + 1); k < ldm_of(PP); ++k) Mc[k] = 0.0;
}

void launch_p2m(hipStream_t s, int p, Box box, const int32_t* start, const double4* P, const DevTables& T, double* M,
                const double4* Pd) {
    const long long nleaves = 1ll << (3 * box.depth);
    const unsigned nb = (unsigned)cdiv(nleaves, 256);
    switch (p) {
#define CASE(PP)                                                                                                   \
    case PP:                                                                                                       \
        if (Pd)                                                                                                    \
            hipLaunchKernelGGL((k_p2m<PP, true>), dim3((unsigned)nleaves), dim3(64), 0, s, box, start, P, T, M, Pd);  \
        else                                                                                                       \
            hipLaunchKernelGGL((k_p2m_lane<PP>), dim3(nb), dim3(256), 0, s, box, start, P, M);                      \
        break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

// ------------------------------------------------------------------ M2M

constexpr int SHIFT_NP = 16;  // parents per workgroup in M2M/L2L
static_assert(ldm_of(PMAX) <= 128, "one thread per component in M2M");

// parent M~ = sum over the 8 children o of A_o M~_child (Eq. M2M in scaled
// form).  A_o[n][j] vanishes for rank(j) > rank(n) (the shift is exact and
// rank-lowering), so row n only reads the first (rank(n)+1)^2 columns.  One
// thread per component n; the children of one octant at a time are staged
// in LDS, component-major (15.5 KB at p = 10, so several workgroups share a
// CU), and each matrix element is loaded once per SHIFT_NP parents.
__global__ __launch_bounds__(128) void k_m2m(int p, long long nparents, const double* __restrict__ Mc,
                                             double* __restrict__ Mp, const double* __restrict__ m2m_t) {
    const long long P0 = (long long)blockIdx.x * SHIFT_NP;
    const int nc = (p + 1) * (p + 1);
    const int ldm = ldm_of(p);
    __shared__ double ch[NIND][SHIFT_NP];
    const int np = (int)min((long long)SHIFT_NP, nparents - P0);
    const int n = threadIdx.x;
    const int jmax = n < nc ? (rank_of(n) + 1) * (rank_of(n) + 1) : 0;
    double acc[SHIFT_NP];
#pragma unroll
    for (int pp = 0; pp < SHIFT_NP; ++pp) acc[pp] = 0.0;
    for (int o = 0; o < 8; ++o) {
        __syncthreads();  // the previous octant's reads are done
        for (int t = threadIdx.x; t < SHIFT_NP * nc; t += 128) {
            const int pp = t / nc, j = t % nc;
            ch[j][pp] = pp < np ? Mc[((size_t)(P0 + pp) * 8 + o) * ldm + j] : 0.0;
        }
        __syncthreads();
        const double* A = m2m_t + (size_t)o * NIND * NIND + n;
#pragma unroll 4
        for (int j = 0; j < jmax; ++j) {
            const double a = A[(size_t)j * NIND];
#pragma unroll
            for (int pp = 0; pp < SHIFT_NP; ++pp) acc[pp] += a * ch[j][pp];
        }
    }
    if (n < ldm)
        for (int pp = 0; pp < np; ++pp) Mp[(size_t)(P0 + pp) * ldm + n] = acc[pp];  // padding stays zero
}

void launch_m2m(hipStream_t s, int p, int parent_level, const double* Mchild, double* Mparent, const DevTables& T) {
    const long long np = 1ll << (3 * parent_level);
    hipLaunchKernelGGL(k_m2m, dim3((unsigned)((np + SHIFT_NP - 1) / SHIFT_NP)), dim3(128), 0, s, p, np, Mchild,
                       Mparent, T.m2m_t);
}

// ------------------------------------------------------------------ M2L operators

template <int P>
__global__ void k_offset_dtensors(double* __restrict__ Dv) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= NOFF) return;
    const int vx = v % 7 - 3, vy = (v / 7) % 7 - 3, vz = v / 49 - 3;
    double D[(P + 1) * (P + 1)];
    const bool far = abs(vx) > 1 || abs(vy) > 1 || abs(vz) > 1;
    if (far) gen_dtensor<P>((double)vx, (double)vy, (double)vz, D);
    for (int i = 0; i < (P + 1) * (P + 1); ++i) Dv[(size_t)v * NIND + i] = far ? D[i] : 0.0;
}

void launch_offset_dtensors(hipStream_t s, int p, double* Dv) {
    switch (p) {
#define CASE(PP) case PP: hipLaunchKernelGGL(k_offset_dtensors<PP>, dim3(cdiv(NOFF, 64)), dim3(64), 0, s, Dv); break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

// Kt[v][j][n] = K_v[n][j] = sum_i c[n,j,i] D_i(v)   (Eq. M2L, independent components)
__global__ void k_build_k(int p, const double* __restrict__ Dv, DevTables T, double* __restrict__ Kt) {
    const int nc = (p + 1) * (p + 1);
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (long long)NOFF * nc * nc) return;
    const int n = (int)(gid % nc);
    const int j = (int)((gid / nc) % nc);
    const int v = (int)(gid / ((long long)nc * nc));
    double k = 0.0;
    if (rank_of(n) + rank_of(j) <= p) {
        const int b = T.c_start[n * NIND + j], cnt = T.c_count[n * NIND + j];
        const double* D = Dv + (size_t)v * NIND;
        for (int t = b; t < b + cnt; ++t) k += T.c_coef[t] * D[T.c_slot[t]];
    }
    Kt[((size_t)v * nc + j) * nc + n] = k;
}

void launch_build_k(hipStream_t s, int p, const double* Dv, const DevTables& T, double* Kt) {
    const long long nc = (p + 1) * (p + 1);
    const long long tot = NOFF * nc * nc;
    hipLaunchKernelGGL(k_build_k, dim3(cdiv(tot, 256)), dim3(256), 0, s, p, Dv, T, Kt);
}

// ------------------------------------------------------------------ L2L

// child L~_o += B_o L~_parent (Eq. L2L in scaled form).  B_o[n][j] vanishes
// for rank(j) < rank(n), so row n needs only the columns from rank(n)^2 on.
// One thread per (octant, component) and SHIFT_NP parents per workgroup; each
// matrix element is loaded once per SHIFT_NP parents.
__global__ __launch_bounds__(256) void k_l2l(int p, long long nparents, const double* __restrict__ Lp,
                                             double* __restrict__ Lc, const double* __restrict__ l2l_t) {
    const long long P0 = (long long)blockIdx.x * SHIFT_NP;
    const int nc = (p + 1) * (p + 1);
    const int ldm = ldm_of(p);
    __shared__ __attribute__((aligned(16))) double lp[NIND][SHIFT_NP];  // component-major
    const int np = (int)min((long long)SHIFT_NP, nparents - P0);
    for (int t = threadIdx.x; t < SHIFT_NP * nc; t += 256) {
        const int pp = t / nc, k = t % nc;
        lp[k][pp] = pp < np ? Lp[(size_t)(P0 + pp) * ldm + k] : 0.0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 8 * nc; t += 256) {
        const int o = t / nc, n = t % nc;
        const double* B = l2l_t + (size_t)o * NIND * NIND + n;
        double acc[SHIFT_NP];
#pragma unroll
        for (int pp = 0; pp < SHIFT_NP; ++pp) acc[pp] = 0.0;
        // Every lane of the wave starts at the smallest rank(n)^2 among its
        // lanes, so that all read the same LDS row (a broadcast); the extra
        // terms have B_o[n][j] = 0 exactly and leave the sums unchanged.
        const int t0 = t & ~63, t1 = min(t0 + 63, 8 * nc - 1);
        const int r0 = t0 / nc == t1 / nc ? rank_of(t0 % nc) : 0;
        const int js = __builtin_amdgcn_readfirstlane(r0 * r0);
#pragma unroll 4
        for (int j = js; j < nc; ++j) {
            const double bcoef = B[(size_t)j * NIND];
#pragma unroll
            for (int pp = 0; pp < SHIFT_NP; ++pp) acc[pp] += bcoef * lp[j][pp];
        }
        for (int pp = 0; pp < np; ++pp) Lc[((size_t)(P0 + pp) * 8 + o) * ldm + n] += acc[pp];
    }
}

void launch_l2l(hipStream_t s, int p, int parent_level, const double* Lparent, double* Lchild, const DevTables& T) {
    const long long np = 1ll << (3 * parent_level);
    hipLaunchKernelGGL(k_l2l, dim3((unsigned)((np + SHIFT_NP - 1) / SHIFT_NP)), dim3(256), 0, s, p, np, Lparent,
                       Lchild, T.l2l_t);
}

// ------------------------------------------------------------------ L2P + P2P

// position of (a,b,c) in full storage: rank-major, a descending, b descending
__host__ __device__ constexpr int full_slot(int a, int b, int c) {
    const int n = a + b + c;
    return n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + (n - a - b);
}

// 1/sqrt(r2) in FP64 (the math library's reciprocal square root)
__device__ inline double rsqrt64(double r2) { return rsqrt(r2); }

__device__ inline void pair_add(double xb, double yb, double zb, double4 src, double& f, double& gx, double& gy,
                                double& gz) {
    const double dx = xb - src.x, dy = yb - src.y, dz = zb - src.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) return;  // coincident pair: contributes nothing
    const double ir = rsqrt64(r2);
    f += src.w * ir;
    const double ir3 = src.w * ir * ir * ir;
    gx -= ir3 * dx;
    gy -= ir3 * dy;
    gz -= ir3 * dz;
}

// hardware dispatches workgroups round-robin over the 8 XCDs (each with its
// own L2); give every XCD a contiguous range of the work instead (XCD x,
// which receives workgroups x, x + 8, ..., takes nb/8 items, one more when
// x < nb % 8)
__device__ inline long long xcd_remap(long long b, long long nb) {
    const long long x = b % 8, per = nb / 8, rem = nb % 8;
    return x * per + (x < rem ? x : rem) + b / 8;
}

// Workgroup barrier that orders LDS only: global loads in flight stay in
// flight across it (a full barrier also waits for them).
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// L2P of the uniform tree (Eq. L2P).  A persistent workgroup of L2P_THR
// threads takes groups of L2P_LB consecutive leaves (g, g + gridDim.x, ...).
// Per group it writes each leaf's local expansion as the NF coefficients
// C_n = L_n / n! of a plain polynomial in r = (x - z)/h, in LDS: the
// independent components scaled into their slots, then the others by the
// trace condition, pass by pass over n_z (each pass reads slots of the passes
// before it); then every particle of the group (one thread each, sorted
// order) evaluates the polynomial and its gradient by nested Horner, one FMA
// per coefficient and level.  The next group's coefficient rows, leaf range
// and first particle per thread are loaded while the current one is worked
// on; the construction tables sit in LDS for the whole launch.  F[s] = far
// field.
constexpr int L2P_LB = 32, L2P_THR = 256;
template <int P>
__global__ __launch_bounds__(L2P_THR) __attribute__((amdgpu_waves_per_eu(2))) void k_l2p(
    long long nleaves, Box box, const int32_t* __restrict__ start, const uint32_t* __restrict__ keys,
    const double4* __restrict__ Pt, const double* __restrict__ L, double4* __restrict__ F) {
    using T = GenL2PFull<P>;
    constexpr int ldm = ldm_of(P), NF = T::NF, NI = T::NI, NU = (L2P_LB * NI + L2P_THR - 1) / L2P_THR;
    constexpr int ND = T::dep_off(T::NPASS) > 0 ? T::dep_off(T::NPASS) : 1;
    __shared__ __attribute__((aligned(16))) double Cs[L2P_LB * NF];
    __shared__ double tIW[NI], tDA[ND], tDB[ND];
    __shared__ unsigned tDD[ND];
    __shared__ unsigned short tIS[NI];
    const long long ngroups = (nleaves + L2P_LB - 1) / L2P_LB;
    long long g = blockIdx.x;
    if (g >= ngroups) return;
    for (int i = threadIdx.x; i < NI; i += L2P_THR) {
        tIS[i] = T::is()[i];
        tIW[i] = T::iw()[i];
    }
    for (int i = threadIdx.x; i < T::dep_off(T::NPASS); i += L2P_THR) {
        tDD[i] = T::dd()[i];
        tDA[i] = T::da()[i];
        tDB[i] = T::db()[i];
    }
    const int tid0 = (int)threadIdx.x;
    const double h = box.side / (double)(1 << box.depth);
    const double ih = 1.0 / h;
    double lr[NU];
    int st0, st1;
    // coefficient rows (NI per leaf, row stride ldm) and leaf range of group gg
#define L2P_LOAD_GROUP(gg)                                                          \
    {                                                                               \
        const long long cc = (gg) * L2P_LB;                                         \
        const int nn = (int)min((long long)L2P_LB, nleaves - cc);                   \
        const double* Lg = L + (size_t)cc * ldm;                                    \
        _Pragma("unroll") for (int u = 0; u < NU; ++u) {                            \
            const int i = tid + u * L2P_THR;                                        \
            const int lf = i / NI, j = i - lf * NI;                                 \
            lr[u] = i < nn * NI ? Lg[(size_t)lf * ldm + j] : 0.0;                   \
        }                                                                           \
        st0 = start[cc];                                                            \
        st1 = start[cc + nn];                                                       \
    }
    {
        const int tid = tid0;
        L2P_LOAD_GROUP(g);
    }
    __syncthreads();
    uint32_t pkey = 0;
    double4 ppt = make_double4(0.0, 0.0, 0.0, 0.0);
    if (st0 + tid0 < st1) {
        pkey = keys[st0 + tid0];
        ppt = Pt[st0 + tid0];
    }
    for (; g < ngroups; g += gridDim.x) {
        const long long c0 = g * L2P_LB;
        const int nl = (int)min((long long)L2P_LB, nleaves - c0);
        const int s0 = st0, s1 = st1;
        // recomputed per group: values derived from the thread index alone are
        // not kept live across the loop (they would not fit in registers)
        int tid = tid0;
        __asm__ volatile("" : "+v"(tid));
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int i = tid + u * L2P_THR;
            if (i < nl * NI) {
                const int lf = i / NI, j = i - lf * NI;
                Cs[lf * NF + tIS[j]] = tIW[j] * lr[u];
            }
        }
        const bool more = g + gridDim.x < ngroups;
        if (more) L2P_LOAD_GROUP(g + gridDim.x);
        lds_barrier();
#pragma unroll
        for (int k = 0; k < T::NPASS; ++k) {
            const int e0 = T::dep_off(k), cnt = T::dep_off(k + 1) - e0;
#pragma unroll
            for (int u = 0; u < (L2P_LB * cnt + L2P_THR - 1) / L2P_THR; ++u) {
                const int i = tid + u * L2P_THR;
                if (i < nl * cnt) {
                    const int lf = i / cnt, e = e0 + i - lf * cnt;
                    const unsigned d = tDD[e];
                    double* C = Cs + lf * NF;
                    C[d & 1023u] = fma(tDA[e], C[(d >> 10) & 1023u], tDB[e] * C[d >> 20]);
                }
            }
            lds_barrier();
        }
        for (int s = s0 + tid; s < s1; s += L2P_THR) {
            const bool first = s == s0 + tid;
            const uint32_t key = first ? pkey : keys[s];
            const double4 pt = first ? ppt : Pt[s];
            const double zx = box.lo[0] + ((double)compact3(key) + 0.5) * h;
            const double zy = box.lo[1] + ((double)compact3(key >> 1) + 0.5) * h;
            const double zz = box.lo[2] + ((double)compact3(key >> 2) + 0.5) * h;
            lds_cdouble* Cp = (lds_cdouble*)(Cs + (size_t)(key - (uint32_t)c0) * NF);
            double f, gx, gy, gz;
            T::eval((pt.x - zx) * ih, (pt.y - zy) * ih, (pt.z - zz) * ih, Cp, f, gx, gy, gz);
            F[s] = make_double4(f * ih, gx * ih * ih, gy * ih * ih, gz * ih * ih);
        }
        if (more && st0 + tid < st1) {
            pkey = keys[st0 + tid];
            ppt = Pt[st0 + tid];
        }
        lds_barrier();
    }
#undef L2P_LOAD_GROUP
}

// One point dipole d at x_s on the target x: potential d.r/|r|^3, r = x - x_s,
// and its gradient d/|r|^3 - 3 (d.r) r/|r|^5 (the limit of two opposite
// charges, Appendix B.1); nothing for coincident points.
__device__ inline void pair_add_dip(double x, double y, double z, const double4 src, const double4 d, double& f,
                                    double& gx, double& gy, double& gz) {
    const double dx = x - src.x, dy = y - src.y, dz = z - src.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) return;
    const double ir = 1.0 / sqrt(r2);
    const double ir3 = ir * ir * ir, ir5 = ir3 * ir * ir;
    const double pr = d.x * dx + d.y * dy + d.z * dz;
    f += pr * ir3;
    gx += d.x * ir3 - 3.0 * pr * dx * ir5;
    gy += d.y * ir3 - 3.0 * pr * dy * ir5;
    gz += d.z * ir3 - 3.0 * pr * dz * ir5;
}

// P2P: one thread per (sorted) target; sources are the particles of the 27
// adjacent-or-equal leaves, self excluded (Appendix C near field), with their
// point dipoles Pd if given.  Adds the far field F[s] if given and writes the
// outputs in input order.
__global__ __launch_bounds__(256) void k_p2p(int n, Box box, const uint32_t* __restrict__ keys,
                                             const int32_t* __restrict__ start, const double4* __restrict__ Pt,
                                             const int32_t* __restrict__ idx, const double4* __restrict__ F,
                                             double* __restrict__ phi, double* __restrict__ grad,
                                             const double4* __restrict__ Pd) {
    const long long s = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int n1 = 1 << box.depth;
    const uint32_t key = keys[s];
    const int ix = compact3(key), iy = compact3(key >> 1), iz = compact3(key >> 2);
    const double4 pt = Pt[s];
    double f = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    if (F) {
        const double4 fv = F[s];
        f = fv.x; gx = fv.y; gy = fv.z; gz = fv.w;
    }
    for (int dz = -1; dz <= 1; ++dz) {
        const int cz = iz + dz;
        if (cz < 0 || cz >= n1) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            const int cy = iy + dy;
            if (cy < 0 || cy >= n1) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                const int cx = ix + dx;
                if (cx < 0 || cx >= n1) continue;
                const uint32_t cn = morton3(cx, cy, cz);
                const int sb = start[cn], se = start[cn + 1];
                for (int s2 = sb; s2 < se; ++s2) {
                    if (s2 == s) continue;
                    const double4 src = Pt[s2];
                    pair_add(pt.x, pt.y, pt.z, src, f, gx, gy, gz);
                    if (Pd) pair_add_dip(pt.x, pt.y, pt.z, src, Pd[s2], f, gx, gy, gz);
                }
            }
        }
    }
    const size_t o = (size_t)idx[s];
    if (phi) phi[o] = f;
    if (grad) {
        grad[3 * o] = gx;
        grad[3 * o + 1] = gy;
        grad[3 * o + 2] = gz;
    }
}

// P2P of the uniform tree, one wavefront per leaf, after the adaptive tree's
// k_p2p_leaf: the sources of the 27 adjacent-or-equal leaves (Appendix C near
// field) are staged in LDS, 64 KS at a time; the leaf's targets go to the
// lanes in chunks of ntc, the sources of each stage to G = 64/ntc groups
// (source j to group j mod G), whose sums are added in group order.  The far
// field F (if given) is added and the outputs written in input order.
constexpr int UP_KS = 3;
__global__ __launch_bounds__(64) void k_p2p_uleaf(Box box, const int32_t* __restrict__ start,
                                                  const double4* __restrict__ Pt, const int32_t* __restrict__ idx,
                                                  const double4* __restrict__ F, double* __restrict__ phi,
                                                  double* __restrict__ grad) {
    constexpr int KS = UP_KS;
    __shared__ double4 S[64 * KS];
    double4* red = S;  // the group sums, once the sources are no longer read
    __shared__ int epb[27], epre[28];
    const uint32_t c = (uint32_t)xcd_remap(blockIdx.x, gridDim.x);
    const int b = start[c], e = start[c + 1];
    if (b == e) return;
    const int lane = threadIdx.x;
    const int n1 = 1 << box.depth;
    const int ix = compact3(c), iy = compact3(c >> 1), iz = compact3(c >> 2);
    // lane k < 27: the neighbour at offset (k mod 3, k/3 mod 3, k/9) - 1
    int sz = 0;
    if (lane < 27) {
        const int cx = ix + lane % 3 - 1, cy = iy + (lane / 3) % 3 - 1, cz = iz + lane / 9 - 1;
        int pb = 0;
        if (cx >= 0 && cx < n1 && cy >= 0 && cy < n1 && cz >= 0 && cz < n1) {
            const uint32_t cn = morton3(cx, cy, cz);
            pb = start[cn];
            sz = start[cn + 1] - pb;
        }
        epb[lane] = pb;
    }
    int incl = sz;  // inclusive scan over the lanes
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(incl, d);
        if (lane >= d) incl += o;
    }
    if (lane < 27) epre[lane + 1] = incl;
    if (lane == 0) epre[0] = 0;
    __syncthreads();
    const int tot = epre[27];
    for (int t0 = b; t0 < e;) {
        int ntc = min(64, e - t0);
        if ((64 / ntc) * ntc * 8 < 64 * 7) ntc = 1 << (31 - __builtin_clz(ntc));
        const int G = 64 / ntc;
        const int g = lane / ntc, tl = lane % ntc;
        const bool active = g < G;
        const int s = t0 + tl;
        const double4 pt = Pt[s];
        double f = 0.0, gx = 0.0, gy = 0.0, gz = 0.0, f2 = 0.0, gx2 = 0.0, gy2 = 0.0, gz2 = 0.0;
        for (int base = 0; base < tot; base += 64 * KS) {
#pragma unroll
            for (int k = 0; k < KS; ++k) {
                const int j = base + lane + 64 * k;
                if (j < tot) {
                    int lo = 0, hi = 27;  // entry with epre[lo] <= j < epre[lo + 1]
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (epre[mid] <= j) lo = mid; else hi = mid;
                    }
                    S[lane + 64 * k] = Pt[epb[lo] + j - epre[lo]];
                }
            }
            __syncthreads();
            const int cnt = min(64 * KS, tot - base);
            if (active) {
                // two independent accumulator chains; the next two sources
                // are read ahead (indices clamped into the array, values past
                // cnt unused)
                constexpr int LIM = 64 * KS - 1;
                int jj = g;
                double4 a0 = S[min(jj, LIM)], a1 = S[min(jj + G, LIM)];
                for (; jj + G < cnt; jj += 2 * G) {
                    const double4 c0 = a0, c1 = a1;
                    a0 = S[min(jj + 2 * G, LIM)];
                    a1 = S[min(jj + 3 * G, LIM)];
                    pair_add_a(pt.x, pt.y, pt.z, c0, f, gx, gy, gz);
                    pair_add_a(pt.x, pt.y, pt.z, c1, f2, gx2, gy2, gz2);
                }
                if (jj < cnt) pair_add_a(pt.x, pt.y, pt.z, a0, f, gx, gy, gz);
            }
            __syncthreads();
        }
        red[lane] = make_double4(f + f2, gx + gx2, gy + gy2, gz + gz2);
        __syncthreads();
        if (g == 0) {
            double4 r = F ? F[s] : make_double4(0.0, 0.0, 0.0, 0.0);
            for (int gg = 0; gg < G; ++gg) {
                const double4 v = red[tl + ntc * gg];
                r.x += v.x;
                r.y += v.y;
                r.z += v.z;
                r.w += v.w;
            }
            const size_t o = (size_t)idx[s];
            if (phi) phi[o] = r.x;
            if (grad) {
                grad[3 * o] = r.y;
                grad[3 * o + 1] = r.z;
                grad[3 * o + 2] = r.w;
            }
        }
        __syncthreads();
        t0 += ntc;
    }
}

void launch_p2p_leaves(hipStream_t s, Box box, const int32_t* start, const double4* P, const int32_t* idx,
                       const double4* F, double* phi, double* grad) {
    const long long nleaves = 1ll << (3 * box.depth);
    hipLaunchKernelGGL(k_p2p_uleaf, dim3((unsigned)nleaves), dim3(64), 0, s, box, start, P, idx, F, phi, grad);
}

void launch_l2p(hipStream_t s, int p, int n, Box box, const int32_t* start, const uint32_t* keys, const double4* P,
                const double* L, double4* F) {
    if (n <= 0) return;
    const long long nleaves = 1ll << (3 * box.depth);
    const long long ngroups = (nleaves + L2P_LB - 1) / L2P_LB;
    int dev = 0, ncu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    // persistent: as many workgroups as fit on the device at once
    auto grid_of = [&](const void* k) {
        int per = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, L2P_THR, 0) != hipSuccess || per < 1) per = 1;
        return dim3((unsigned)std::min<long long>(ngroups, (long long)std::max(ncu, 1) * per));
    };
    const dim3 blk(L2P_THR);
    switch (p) {
#define CASE(PP)                                                                                         \
    case PP:                                                                                             \
        hipLaunchKernelGGL(k_l2p<PP>, grid_of((const void*)k_l2p<PP>), blk, 0, s, nleaves, box, start, keys, P, L, F); \
        break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

void launch_p2p(hipStream_t s, int n, Box box, const uint32_t* keys, const int32_t* start, const double4* P,
                const int32_t* idx, const double4* F, double* phi, double* grad, const double4* Pd) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_p2p, dim3(cdiv(n, 256)), dim3(256), 0, s, n, box, keys, start, P, idx, F, phi, grad, Pd);
}

// ------------------------------------------------------------------ debug copy-out

__global__ void k_unscale_copy(int p, int level, int which, double h, const double* __restrict__ X,
                               double* __restrict__ out) {
    const int nc = (p + 1) * (p + 1);
    const long long n1 = 1ll << level;
    const long long tot = n1 * n1 * n1 * nc;
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= tot) return;
    const int k = (int)(gid % nc);
    const long long cell = gid / nc;
    const uint32_t ix = (uint32_t)(cell % n1), iy = (uint32_t)((cell / n1) % n1), iz = (uint32_t)(cell / (n1 * n1));
    const uint32_t m = morton3(ix, iy, iz);
    double v = X[(size_t)m * ldm_of(p) + k];
    const int r = rank_of(k);
    double hp = 1.0;
    for (int t = 0; t < r; ++t) hp *= h;
    out[gid] = which == 0 ? v * hp : v / (hp * h);
}

void launch_unscale_copy(hipStream_t s, int p, int level, int which, double side, const double* X, double* out) {
    const long long nc = (p + 1) * (p + 1);
    const long long tot = (1ll << (3 * level)) * nc;
    const double h = side / (double)(1 << level);
    hipLaunchKernelGGL(k_unscale_copy, dim3(cdiv(tot, 256)), dim3(256), 0, s, p, level, which, h, X, out);
}

// ================================================================== tiled MFMA M2L
//
// Work unit: one target octant o and a block of up to 64 Morton-consecutive
// parent cells (a 4x4x4 cube of parents).  Its targets (parent*8 + o) share
// the same 189 offsets v of the ws=1 list, so for each v the whole tile is
// one small GEMM  L~[:, tile] += K_v * M~[:, tile + v].  K_v is stored as
// MFMA A-fragments of its non-zero blocks only (rows of rank a need columns
// of rank <= p - a).  Per offset, K_v and the 64 source rows are copied into
// LDS with direct global->LDS loads (no VGPR round trip), double-buffered so
// the copies for offset v+1 overlap the matrix-core work of offset v.  Wave
// w owns targets 16w..16w+15 and every row tile.
//
// Precisions (operand type -> accumulator):
//   F64    : FP64 16x16x4 MFMA, FP64 accumulation
//   F32    : operands rounded to FP32, FP32 16x16x4 MFMA, FP32 accumulation
//   BF16X3 : operands split x = x0 + x1 + x2 into BF16 pieces (24 significant
//            bits), the six products with piece-index sum <= 2 on BF16
//            16x16x32 MFMA, FP32 accumulation
// The local expansions are written back in FP64.

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

__host__ __device__ constexpr int rank_ce(int k) {
    int r = 0;
    while ((r + 1) * (r + 1) <= k) ++r;
    return r;
}

constexpr int LDS_LIMIT = 163840;
constexpr int STATIC_LDS = 2048;  // the tile kernel's static LDS (target coordinates, offset tables), rounded up

}  // namespace

template <int P, int PREC, int TT = 64>
struct Tile {
    static constexpr int NC = (P + 1) * (P + 1);
    static constexpr int LDM = (NC + 3) & ~3;                 // FP64 expansion row stride
    static constexpr int S32 = ((NC + 31) / 32) * 32;          // FP32 copy row stride
    static constexpr int KW = PREC == PREC_BF16X3 ? 32 : 4;    // k extent of one MFMA
    static constexpr int R = (NC + 15) / 16;                   // 16-row tiles
    static constexpr int nch(int r) {
        const int m = P - rank_ce(16 * r) + 1;
        return (m * m + KW - 1) / KW;
    }
    static constexpr int cb(int r) {
        int s = 0;
        for (int i = 0; i < r; ++i) s += nch(i);
        return s;
    }
    static constexpr int NCH = cb(R);
    static constexpr int NB = nch(0);
    // Chunk c of row tile r holds rows 16r.. and columns KW c..; its lowest
    // total rank is rank(16r) + rank(KW c), so the order-q operator (Eq. M2L
    // truncated at |n| + |m| <= q) is zero in it unless that sum is <= q.
    // Chunks are stored sorted by that rank (then r, then c): the chunks of
    // the order-q operator are then a prefix, nup(q) long, of every offset's
    // fragments, whatever q <= P.
    static constexpr int minord(int r, int c) { return rank_ce(16 * r) + rank_ce(KW * c); }
    // largest total rank of the chunk's entries (its padding is zero anyway)
    static constexpr int maxord(int r, int c) {
        return rank_ce(16 * r + 15 < NC ? 16 * r + 15 : NC - 1) + rank_ce(KW * c + KW - 1 < NC ? KW * c + KW - 1 : NC - 1);
    }
    struct PosTab {
        int v[R][NB > 0 ? NB : 1];
        int nup[P + 1];
    };
    static constexpr PosTab make_pos() {
        PosTab t{};
        int k = 0;
        for (int m = 0; m <= P; ++m) {
            for (int r = 0; r < R; ++r)
                for (int c = 0; c < nch(r); ++c)
                    if (minord(r, c) == m) t.v[r][c] = k++;
            t.nup[m] = k;
        }
        return t;
    }
    static constexpr PosTab PT = make_pos();
    static constexpr int pos(int r, int c) { return PT.v[r][c]; }
    // bytes of one packed A-fragment chunk (64 lanes)
    static constexpr int CHB = PREC == PREC_F64 ? 512 : PREC == PREC_F32 ? 256 : 3 * 64 * 16;
    static constexpr int KBYTES = NCH * CHB;
    // one source row: FP64 rows of LDM doubles, or FP32 rows of S32 floats;
    // in LDS the rows of one offset are contiguous (no padding), so that one
    // global->LDS copy instruction can fill parts of several rows
    static constexpr int BROW = PREC == PREC_F64 ? LDM * 8 : S32 * 4;
    static constexpr int RU = BROW / 16;       // 16-byte units of a row
    // Rows whose unit count is a multiple of 8 would put the 16 targets of a
    // B-fragment read on the same LDS banks; their units are rotated by the
    // row slot instead (LDS unit (u + s) mod RU of slot s holds unit u).
    static constexpr bool ROT = RU % 8 == 0;
    static constexpr int BBYTES = TT * BROW;   // the source rows of one offset for TT targets
    static constexpr int KBUF = (2 * KBYTES + 2 * BBYTES + STATIC_LDS <= LDS_LIMIT) ? 2 : 1;
    static constexpr int LDS = KBUF * KBYTES + 2 * BBYTES;
};

__device__ inline uint16_t bf16_rne(float x) {
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_to_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// K_v as MFMA A-fragments: Kpk[v slot][chunk position][...], lane -> (row
// 16r + lane%16, k 16-lane group); with pmask < P the order-pmask operator
// (entries of rank(row) + rank(col) > pmask are zero), in the same layout.
template <int P, int PREC>
__global__ void k_pack_k(const double* __restrict__ Kt, unsigned char* __restrict__ Kpk, int pmask) {
    using S = Tile<P, PREC>;
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (long long)NOFF * S::NCH * 64) return;
    const int lane = (int)(gid % 64);
    const int ch = (int)((gid / 64) % S::NCH);
    const int v = (int)(gid / (64ll * S::NCH));
    // the (row tile, chunk) stored at position ch (the order of Tile::make_pos)
    int r = 0, c = 0;
    {
        int k = 0;
        bool found = false;
        for (int m = 0; m <= P && !found; ++m)
            for (int rr = 0; rr < S::R && !found; ++rr)
                for (int cc = 0; cc < S::nch(rr) && !found; ++cc)
                    if (S::minord(rr, cc) == m) {
                        if (k == ch) {
                            r = rr;
                            c = cc;
                            found = true;
                        }
                        ++k;
                    }
    }
    const int row = 16 * r + (lane % 16);
    auto kval = [&](int col) -> double {
        if (row >= S::NC || col >= S::NC || rank_ce(row) + rank_ce(col) > pmask) return 0.0;
        return Kt[((size_t)v * S::NC + col) * S::NC + row];
    };
    unsigned char* dst = Kpk + ((size_t)v * S::NCH + ch) * S::CHB;
    if (PREC == PREC_F64) {
        reinterpret_cast<double*>(dst)[lane] = kval(4 * c + lane / 16);
    } else if (PREC == PREC_F32) {
        reinterpret_cast<float*>(dst)[lane] = (float)kval(4 * c + lane / 16);
    } else {
        // [piece][lane][8 bf16]
        for (int e = 0; e < 8; ++e) {
            const double x = kval(32 * c + 8 * (lane / 16) + e);
            const uint16_t h0 = bf16_rne((float)x);
            const double r1 = x - (double)bf16_to_f(h0);
            const uint16_t h1 = bf16_rne((float)r1);
            const double r2 = r1 - (double)bf16_to_f(h1);
            const uint16_t h2 = bf16_rne((float)r2);
            uint16_t* d16 = reinterpret_cast<uint16_t*>(dst);
            d16[(0 * 64 + lane) * 8 + e] = h0;
            d16[(1 * 64 + lane) * 8 + e] = h1;
            d16[(2 * 64 + lane) * 8 + e] = h2;
        }
    }
}

// FP32 copy of one level's multipoles, rows of S32 floats, zero padded
__global__ void k_to_f32(long long ncell, int nc, int ldm, int s32, const double* __restrict__ M,
                         float* __restrict__ M32) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= ncell * s32) return;
    const long long cell = gid / s32;
    const int k = (int)(gid % s32);
    M32[gid] = k < nc ? (float)M[cell * ldm + k] : 0.0f;
}

__device__ inline void lds_copy16(const void* g, void* lds) {
    __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}

// Targets of a tile whose chunk has no offsets: their local expansions (in
// the chunk's slot) are written as zeros.
__device__ inline void m2l_zero_tile(double* __restrict__ L, const AdaptM2L& ad, long long work, int chunk, int tt,
                                     int ldm) {
    L += (size_t)chunk * ad.chunk_stride;
    for (int x = threadIdx.x; x < tt; x += blockDim.x) {
        const long long t = ad.tgt[(size_t)tt * work + x];
        if (t < 0) continue;
        for (int k = 0; k < ldm; ++k) L[(size_t)t * ldm + k] = 0.0;
    }
}

// ADAPT = true: the work unit is a tile of the adaptive tree (AdaptM2L):
// targets, sources and the octant come from the tables instead of the
// uniform grid, and rows are node indices; the tile's offsets are all 189 or
// the active ones listed for it.  ORD (adaptive only): list entry j runs at
// order q_j = ivord[j] <= P, with the order-q_j operators (Eq. M2L truncated
// at |n| + |m| <= q_j, stored in the order-P chunk layout, of which only the
// first nup[q_j] chunks can be non-zero: only those are copied and
// multiplied).
// NW waves of 16 targets each: TT = 16 NW targets per tile (the uniform
// grid's work unit has 64).
template <int P, int PREC, bool ADAPT, int NW = 4, bool ORD = false>
__global__ __launch_bounds__(64 * NW) void k_m2l_tile(int level, const void* __restrict__ Msrc, double* __restrict__ L,
                                                      const unsigned char* __restrict__ Kpk,
                                                      const int16_t* __restrict__ offlist,
                                                      const unsigned char* __restrict__ zero_row, const AdaptM2L ad) {
    constexpr int TT = 16 * NW;
    static_assert(ADAPT || NW == 4, "the uniform work unit has 64 targets");
    static_assert(ADAPT || !ORD, "orders per offset need the adaptive tables");
    using S = Tile<P, PREC, TT>;
    constexpr int NC = S::NC, LDM = S::LDM, R = S::R, NB = S::NB;
    constexpr int CU = S::CHB / 16;           // 16-byte units of one chunk
    constexpr int RU = S::BROW / 16;          // 16-byte units of one source row
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    unsigned char* Kb = lds;                              // [KBUF][KBYTES]
    unsigned char* Bb = lds + S::KBUF * S::KBYTES;        // [2][TT rows][BROW]
    __shared__ int tco[64];                               // packed target coords, -1 = none

    // work item = 8 * parent block + target octant; each XCD takes a contiguous
    // range, so the 8 octants of a block and neighbouring blocks share its L2
    const long long blk = xcd_remap(blockIdx.x, gridDim.x);
    const long long work = ADAPT ? ad.tile_base + blk / ad.nchunk : blk;
    const int chunk = ADAPT ? (int)(blk % ad.nchunk) : 0;
    // offsets of this tile: all 189, or the active ones listed for it; this
    // workgroup takes list entries [j0, j0 + nv)
    const int nv_all = (ADAPT && ad.ivcnt) ? ad.ivcnt[work] : 189;
    const int j0 = ADAPT ? (int)((long long)nv_all * chunk / ad.nchunk) : 0;
    const int nv = ADAPT ? (int)((long long)nv_all * (chunk + 1) / ad.nchunk) - j0 : 189;
    if (nv == 0) {
        if (ADAPT) m2l_zero_tile(L, ad, work, chunk, TT, LDM);
        return;
    }
    auto ivof = [&](int j) -> int {
        return (ADAPT && ad.ivlist) ? (int)ad.ivlist[189 * work + j0 + j] : j0 + j;
    };
    const int o = ADAPT ? ad.tiles[work].x : (int)(work & 7);
    const long long pb = work >> 3;
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n1 = 1 << level;
    const long long nparents = ADAPT ? 0 : 1ll << (3 * (level - 1));
    if (!ADAPT && tid < 64) {
        const long long par = (long long)pb * 64 + tid;
        int packed = -1;
        if (par < nparents) {
            const uint32_t t = (uint32_t)(par * 8 + o);
            packed = (int)(compact3(t) | (compact3(t >> 1) << 10) | (compact3(t >> 2) << 20));
        }
        tco[tid] = packed;
    }

    // Tables of this workgroup in LDS (read before any copy of an iteration
    // is issued, see below), per list position j: the offset, its operator
    // slot, its order, and (uniform grid) the packed offset.
    __shared__ int16_t s_iv[189], s_ks[189], s_off[ADAPT ? 1 : 189];
    __shared__ int8_t s_q[ORD ? 189 : 1];
    for (int x = tid; x < nv; x += 64 * NW) {
        const int iv = ivof(x);
        s_iv[x] = (int16_t)iv;
        if (ADAPT) {
            s_ks[x] = ad.kslot[o * 189 + iv];
        } else {
            s_off[ADAPT ? 0 : x] = offlist[o * 189 + iv];
            s_ks[x] = (int16_t)(NOFF - 1 - offlist[o * 189 + iv]);  // the operator is built for r = -v
        }
        if (ORD) s_q[ORD ? x : 0] = ad.ivord[189 * work + j0 + x];
    }
    // K_v of operator slot ks at order q: every chunk (fixed order) or the
    // first nup[q]
    auto stage_k = [&](int q, int ks, int buf) {
        const unsigned char* src = Kpk + (ORD ? (size_t)q * ad.kord_stride : 0) + (size_t)ks * S::KBYTES;
        unsigned char* dst = Kb + buf * S::KBYTES;
        const int ku = ORD ? ad.nup[q] * CU : S::NCH * CU;
        for (int i = w; i * 64 < ku; i += NW) {
            const int u = i * 64 + lane;
            if (u < ku) lds_copy16(src + (size_t)u * 16, dst + i * 1024);
        }
    };
    // Source rows of list position j.  The TT rows fill TT * RU units of LDS;
    // copy instruction k of wave w moves units g = 64 (k NW + w) + lane, i.e.
    // unit g % RU of row slot g / RU, so each lane needs the source row of the
    // slot of each of its NI copies.  Adaptive tiles read them from the tables
    // (vector loads), the uniform grid computes them (LDS reads).
    constexpr int NU = TT * RU;
    constexpr int NI = (NU + 64 * NW - 1) / (64 * NW);
    constexpr int RL = NI;
    // lanes past the last unit (only in the last copy, when NU is not a
    // multiple of 64 NW) are masked off in the copy and take the last slot
    auto unit_ok = [&](int k) { return (NU % (64 * NW) == 0 || k < NI - 1) || 64 * (k * NW + w) + lane < NU; };
    auto slot_of = [&](int k) {
        const int sl = (64 * (k * NW + w) + lane) / RU;
        return sl < TT ? sl : TT - 1;
    };
    // (adaptive: j is the offset iv itself, read from the table beforehand;
    // uniform grid: the list position)
    auto rows_of = [&](int j, int (&rows)[RL]) {
        if (ADAPT) {
            // unconditional loads: a register written before a load into it
            // would make the compiler wait for every outstanding copy
            const size_t e0 = (189 * (size_t)work + j) * TT;
#pragma unroll
            for (int k = 0; k < RL; ++k) rows[k] = ad.src[e0 + slot_of(k)];
            return;
        }
#pragma unroll
        for (int k = 0; k < RL; ++k) {
            int row = -1;
            {
                const int vs = s_off[ADAPT ? 0 : j];
                const int vx = vs % 7 - 3, vy = (vs / 7) % 7 - 3, vz = vs / 49 - 3;
                const int tc = tco[slot_of(k)];
                if (tc >= 0) {
                    const int sx = (tc & 1023) + vx, sy = ((tc >> 10) & 1023) + vy, sz = (tc >> 20) + vz;
                    if (sx >= 0 && sy >= 0 && sz >= 0 && sx < n1 && sy < n1 && sz < n1) row = (int)morton3(sx, sy, sz);
                }
            }
            rows[k] = row;
        }
    };
    // every lane copies one 16-byte unit per instruction; the destination of
    // an instruction is contiguous (64 units from its wave-uniform base)
    auto stage_b = [&](const int (&rows)[RL], int buf) {
        unsigned char* dst = Bb + buf * S::BBYTES;
        const unsigned char* Mb = reinterpret_cast<const unsigned char*>(Msrc);
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            if (unit_ok(k)) {
                const int g = 64 * (k * NW + w) + lane;
                const int sl = g / RU, u = g - sl * RU;
                const int rot = S::ROT ? sl % RU : 0;
                const int gu = u >= rot ? u - rot : u + RU - rot;  // the row's unit that LDS unit u holds
                const int row = rows[k];
                const unsigned char* src = row >= 0 ? Mb + (size_t)row * S::BROW + gu * 16 : zero_row + gu * 16;
                lds_copy16(src, dst + (size_t)64 * 16 * (k * NW + w));
            }
        }
    };

    // accumulators
    v4d acc64[PREC == PREC_F64 ? R : 1][2];
    v4f acc32[PREC == PREC_F32 ? R : 1][2];
    v4f accb[PREC == PREC_BF16X3 ? R : 1][6];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (PREC == PREC_F64) acc64[r][0] = acc64[r][1] = v4d{0.0, 0.0, 0.0, 0.0};
        if (PREC == PREC_F32) acc32[r][0] = acc32[r][1] = v4f{0.f, 0.f, 0.f, 0.f};
        if (PREC == PREC_BF16X3)
            for (int k = 0; k < 6; ++k) accb[r][k] = v4f{0.f, 0.f, 0.f, 0.f};
    }

    __syncthreads();  // the tables
    int rows_cur[RL], rows_nxt[RL];
    rows_of(ADAPT ? s_iv[0] : 0, rows_cur);
    stage_k(ORD ? (int)s_q[0] : P, s_ks[0], 0);
    stage_b(rows_cur, 0);
    if (nv > 1) rows_of(ADAPT ? s_iv[1] : 1, rows_nxt);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int trow = w * 16 + (lane & 15);  // this lane's target slot in B fragments
    const int kq = lane >> 4;
    const int trot = S::ROT ? trow % RU : 0;
    // LDS address of unit u (< RU) of this lane's B-fragment row
    auto bunit = [&](const unsigned char* Bc, int u) {
        const int x = u + trot;
        return Bc + 16 * (x >= RU ? x - RU : x);
    };
    // Each iteration first does all its LDS reads (FP32: this offset's
    // operands; the next offsets' table entries and, on the uniform grid,
    // source rows), then issues the copies of offset j + 1, then loads the
    // row indices of offset j + 2: reads of LDS behind outstanding
    // global->LDS copies wait for those copies, and the row indices of a
    // copy are in registers an iteration before it is issued.
    // FP32: this offset's operands are read from LDS into registers before
    // the next offset's copies are issued.  Reads of LDS behind outstanding
    // global->LDS copies wait for those copies, so issuing the copies first
    // would serialise them with this offset's matrix-core work.
    constexpr bool PRE = PREC == PREC_F32;
    float apre[PRE ? S::NCH : 1], bpre[PRE ? NB : 1];
    for (int j = 0; j < nv; ++j) {
        const int kb = S::KBUF == 2 ? (j & 1) : 0;
        const int bb = j & 1;
        const unsigned char* Kc = Kb + kb * S::KBYTES;
        const unsigned char* Bc = Bb + bb * S::BBYTES + trow * S::BROW;
        // order of this offset (wave-uniform): chunks of lowest rank above it are zero
        const int qj = ORD ? __builtin_amdgcn_readfirstlane((int)s_q[ORD ? j : 0]) : P;
        if (PRE) {
            const float* Kf = reinterpret_cast<const float*>(Kc);
            const int nupj = ORD ? ad.nup[qj] : S::NCH;
#pragma unroll
            for (int ch = 0; ch < (PRE ? S::NCH : 1); ++ch) {
                if (ORD && ch >= nupj) break;
                apre[ch] = Kf[ch * 64 + lane];
            }
#pragma unroll
            for (int c = 0; c < (PRE ? NB : 1); ++c) bpre[c] = reinterpret_cast<const float*>(bunit(Bc, c))[kq];
        }
        // table entries of the next offsets, read before any copy is issued
        const int j1 = j + 1 < nv ? j + 1 : 0;
        const int ks1 = s_ks[j1];
        const int q1 = ORD ? (int)s_q[ORD ? j1 : 0] : P;
        const int iv2 = ADAPT ? s_iv[j + 2 < nv ? j + 2 : 0] : 0;
        int rows_nn[RL];
        if (!ADAPT && j + 2 < nv) rows_of(j + 2, rows_nn);
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): every LDS read of the iteration is done
        if (j + 1 < nv) {
            if (S::KBUF == 2) stage_k(q1, ks1, kb ^ 1);
            stage_b(rows_nxt, bb ^ 1);
        }
        if (ADAPT && j + 2 < nv) rows_of(iv2, rows_nn);  // used after this iteration's wait
        if (PREC == PREC_F64) {
            const double* Kd = reinterpret_cast<const double*>(Kc);
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                if (ORD && S::minord(0, c) > qj) break;
                // double 4c + kq of the row: unit 2c + kq/2, half kq % 2
                const double b = reinterpret_cast<const double*>(bunit(Bc, 2 * c + (kq >> 1)))[kq & 1];
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (c < S::nch(r) && (!ORD || S::minord(r, c) <= qj)) {
                        const double a = Kd[S::pos(r, c) * 64 + lane];
                        acc64[r][c & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc64[r][c & 1], 0, 0, 0);
                    }
            }
        } else if (PREC == PREC_F32) {
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                if (ORD && S::minord(0, c) > qj) break;
                const float b = bpre[PRE ? c : 0];
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (c < S::nch(r) && (!ORD || S::minord(r, c) <= qj)) {
                        const float a = apre[PRE ? S::pos(r, c) : 0];
                        acc32[r][c & 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc32[r][c & 1], 0, 0, 0);
                    }
            }
        } else {
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                if (ORD && S::minord(0, c) > qj) break;
                // this lane's 8 consecutive k of its target (units 8c + 2kq and
                // the next), split into three BF16 pieces
                const v4f x0 = *reinterpret_cast<const v4f*>(bunit(Bc, 8 * c + 2 * kq));
                const v4f x1 = *reinterpret_cast<const v4f*>(bunit(Bc, 8 * c + 2 * kq + 1));
                bf16x8 b0, b1, b2;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float x = e < 4 ? x0[e] : x1[e - 4];
                    const uint16_t h0 = bf16_rne(x);
                    const float r1 = x - bf16_to_f(h0);
                    const uint16_t h1 = bf16_rne(r1);
                    const float r2 = r1 - bf16_to_f(h1);
                    const uint16_t h2 = bf16_rne(r2);
                    b0[e] = __builtin_bit_cast(__bf16, h0);
                    b1[e] = __builtin_bit_cast(__bf16, h1);
                    b2[e] = __builtin_bit_cast(__bf16, h2);
                }
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (c < S::nch(r) && (!ORD || S::minord(r, c) <= qj)) {
                        const bf16x8* A = reinterpret_cast<const bf16x8*>(Kc + S::pos(r, c) * S::CHB);
                        const bf16x8 a0 = A[lane], a1 = A[64 + lane], a2 = A[128 + lane];
                        accb[r][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, accb[r][0], 0, 0, 0);
                        accb[r][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, accb[r][1], 0, 0, 0);
                        accb[r][2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, accb[r][2], 0, 0, 0);
                        accb[r][3] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b2, accb[r][3], 0, 0, 0);
                        accb[r][4] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, accb[r][4], 0, 0, 0);
                        accb[r][5] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b0, accb[r][5], 0, 0, 0);
                    }
            }
        }
        if (S::KBUF == 1 && j + 1 < nv) {
            __syncthreads();  // every wave is done with this offset's K_v
            stage_k(q1, ks1, 0);
        }
        // unconditional, so that no load is outstanding at the top of the
        // loop on any path (the compiler turns any wait behind a mix of
        // loads and global->LDS copies into a wait for all of them); the
        // scheduling barrier keeps the matrix-core work above the wait
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (j + 1 < nv) {
#pragma unroll
            for (int k = 0; k < RL; ++k) rows_nxt[k] = rows_nn[k];
        }
    }
    long long trow_out;
    if (ADAPT) {
        trow_out = ad.tgt[TT * (size_t)work + w * 16 + (lane & 15)];
        if (trow_out < 0) return;
    } else {
        const long long par = (long long)pb * 64 + w * 16 + (lane & 15);
        if (par >= nparents) return;
        trow_out = par * 8 + o;
    }
    double* Lt = L + (ADAPT ? (size_t)chunk * ad.chunk_stride : 0) + (size_t)trow_out * LDM;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (PREC == PREC_F64) {
            // FP64 16x16 accumulator: element j holds row 16r + lane/16 + 4j
            const v4d sacc = acc64[r][0] + acc64[r][1];
            const int row0 = 16 * r + (lane >> 4);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (row0 + 4 * j < NC) Lt[row0 + 4 * j] = sacc[j];
        } else {
            // FP32 16x16 accumulator: element j holds row 16r + 4*(lane/16) + j
            const int row0 = 16 * r + 4 * (lane >> 4);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                double v;
                if (PREC == PREC_F32) {
                    v = (double)acc32[r][0][j] + (double)acc32[r][1][j];
                } else {
                    v = 0.0;
#pragma unroll
                    for (int k = 0; k < 6; ++k) v += (double)accb[r][k][j];
                }
                if (row0 + j < NC) Lt[row0 + j] = v;
            }
        }
    }
}

// ------------------------------------------------------------------ FP32 tile M2L, source rows in registers
//
// The adaptive tile M2L in FP32 with every wave loading the B fragments of
// its 16 targets straight into registers.  The FP32 copy of the multipoles
// is then stored k-quad major (k_to_f32_kq): element k of a row at
// (k mod 4) S32/4 + k/4, so the values of lane (target n, k-quad kq),
// B[4c + kq][n] for c < NB, are contiguous and arrive in 16-byte loads.
// Only K_v goes through LDS (global->LDS copies, double-buffered, shared by
// the waves).  Per offset, a wave first reads its A fragments from LDS, then
// issues the copies of the next K_v, the loads of the next B fragments and
// the row-table loads of the offset after, then the MFMAs; every load of the
// iteration is waited for at its end.  With an order q per offset (ORD), the
// order-P operators are used: only the chunks of the order-q prefix are
// copied, and in the chunks that straddle the truncation each lane zeroes its
// entries of rank(n) + rank(j) > q in registers (one operator set for every
// order keeps the operators' cache footprint that of the fixed order).
template <int P, int NW, bool ORD = false>
__global__ __launch_bounds__(64 * NW) void k_m2l_rb(const float* __restrict__ M32k, double* __restrict__ L,
                                                    const unsigned char* __restrict__ Kpk,
                                                    const float* __restrict__ zero_row, const AdaptM2L ad) {
    constexpr int TT = 16 * NW;
    using S = Tile<P, PREC_F32, TT>;
    constexpr int NC = S::NC, R = S::R, NB = S::NB, NCH = S::NCH;
    constexpr int SEG = S::S32 / 4;    // floats of one k-quad segment of a row
    constexpr int NBL = (NB + 3) / 4;  // 16-byte loads per lane and offset
    static_assert(4 * NBL <= SEG, "a lane's loads stay in its segment of the row");
    constexpr int KU = S::KBYTES / 16;
    constexpr int CU = S::CHB / 16;
    __shared__ __attribute__((aligned(16))) unsigned char Kb[2][S::KBYTES];
    __shared__ int16_t s_iv[189], s_ks[189];
    __shared__ int8_t s_q[ORD ? 189 : 1];
    const long long blk = xcd_remap(blockIdx.x, gridDim.x);
    const long long work = ad.tile_base + blk / ad.nchunk;
    const int chunk = (int)(blk % ad.nchunk);
    // this workgroup takes entries [j0, j0 + nv) of the tile's offsets (all
    // 189, or the active ones listed for it)
    const int nv_all = ad.ivcnt ? ad.ivcnt[work] : 189;
    const int j0 = (int)((long long)nv_all * chunk / ad.nchunk);
    const int nv = (int)((long long)nv_all * (chunk + 1) / ad.nchunk) - j0;
    // (a chunk without offsets runs no offset and writes zeros)
    const int o = ad.tiles[work].x;
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int x = tid; x < nv; x += 64 * NW) {
        const int iv = ad.ivlist ? (int)ad.ivlist[189 * work + j0 + x] : j0 + x;
        s_iv[x] = (int16_t)iv;
        s_ks[x] = ad.kslot[o * 189 + iv];
        if (ORD) s_q[ORD ? x : 0] = ad.ivord[189 * work + j0 + x];
    }
    // K_v of operator slot ks at order q: every chunk (fixed order) or the
    // first nup[q] (the others are zero)
    auto stage_k = [&](int q, int ks, int buf) {
        const unsigned char* src = Kpk + (size_t)ks * S::KBYTES;
        const int ku = ORD ? ad.nup[q] * CU : KU;
        for (int i = w; i * 64 < ku; i += NW) {
            const int u = i * 64 + lane;
            if (u < ku) lds_copy16(src + (size_t)u * 16, &Kb[buf][i * 1024]);
        }
    };
    const int kq = lane >> 4;
    // ranks of this lane's operator rows (16 r + lane % 16) for the truncation
    int rrow[R];
#pragma unroll
    for (int r = 0; r < R; ++r) rrow[r] = (int)sqrtf((float)(16 * r + (lane & 15)));
    // table entry of (offset 0, this lane's target slot 16 w + n)
    const size_t tab0 = 189 * (size_t)work * TT + 16 * w + (lane & 15);
    auto row_of = [&](int iv) { return ad.src[tab0 + (size_t)iv * TT]; };
    auto load_b = [&](int row, float (&b)[4 * NBL]) {
        const float* src = (row >= 0 ? M32k + (size_t)row * S::S32 : zero_row) + kq * SEG;
#pragma unroll
        for (int i = 0; i < NBL; ++i) {
            const float4 v = reinterpret_cast<const float4*>(src)[i];
            b[4 * i] = v.x;
            b[4 * i + 1] = v.y;
            b[4 * i + 2] = v.z;
            b[4 * i + 3] = v.w;
        }
    };
    v4f acc[R][2];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r][0] = acc[r][1] = v4f{0.f, 0.f, 0.f, 0.f};
    float bcur[4 * NBL], bnxt[4 * NBL], apre[NCH];
    __syncthreads();  // the tables
    // (without offsets: operator slot 0 and the zero row, unused)
    stage_k(ORD && nv ? (int)s_q[0] : P, nv ? (int)s_ks[0] : 0, 0);
    load_b(nv ? row_of(s_iv[0]) : -1, bcur);
    int rnxt = nv > 1 ? row_of(s_iv[1]) : -1;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int j = 0; j < nv; ++j) {
        const float* Kf = reinterpret_cast<const float*>(Kb[j & 1]);
        // this offset's order (wave-uniform).  Every chunk is read (an early
        // exit here would put apre in scratch memory); those past the order's
        // prefix hold stale data that no MFMA below uses (a chunk's position
        // is below nup[q] exactly when minord <= q)
        const int qj = ORD ? __builtin_amdgcn_readfirstlane((int)s_q[ORD ? j : 0]) : P;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) apre[ch] = Kf[ch * 64 + lane];
        // table entries of the next offsets, read before any copy is issued
        const int j1 = j + 1 < nv ? j + 1 : 0;
        const int ks1 = s_ks[j1];
        const int q1 = ORD ? (int)s_q[ORD ? j1 : 0] : P;
        const int iv2 = s_iv[j + 2 < nv ? j + 2 : 0];
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): the LDS reads of the iteration are done
        int rnn = -1;
        if (j + 1 < nv) {
            stage_k(q1, ks1, (j + 1) & 1);
            load_b(rnxt, bnxt);
        }
        if (j + 2 < nv) rnn = row_of(iv2);
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            if (ORD && S::minord(0, c) > qj) break;
            // rank of this lane's source component 4 c + kq
            const int rcol = ORD ? (int)sqrtf((float)(4 * c + kq)) : 0;
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (c < S::nch(r) && (!ORD || S::minord(r, c) <= qj)) {
                    float a = apre[S::pos(r, c)];
                    if (ORD && S::maxord(r, c) > qj && rrow[r] + rcol > qj) a = 0.f;
                    acc[r][c & 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bcur[c], acc[r][c & 1], 0, 0, 0);
                }
        }
        // every load of the iteration is waited for here (on every path); the
        // scheduling barrier keeps the MFMAs above the wait
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4 * NBL; ++i) bcur[i] = bnxt[i];
        rnxt = rnn;
    }
    const long long trow_out = ad.tgt[TT * (size_t)work + 16 * w + (lane & 15)];
    if (trow_out < 0) return;
    double* Lt = L + (size_t)chunk * ad.chunk_stride + (size_t)trow_out * S::LDM;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        // FP32 16x16 accumulator: element i holds row 16r + 4 kq + i
        const int row0 = 16 * r + 4 * kq;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double v = (double)acc[r][0][i] + (double)acc[r][1][i];
            if (row0 + i < NC) Lt[row0 + i] = v;
        }
    }
}

// FP32 copy of multipole rows in the k-quad-major order of k_m2l_rb: rows
// of S32 floats, element k at (k mod 4) S32/4 + k/4, zero past nc
__global__ void k_to_f32_kq(long long ncell, int nc, int ldm, int s32, const double* __restrict__ M,
                            float* __restrict__ M32) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= ncell * s32) return;
    const long long cell = gid / s32;
    const int pos = (int)(gid % s32), seg = s32 / 4;
    const int k = 4 * (pos % seg) + pos / seg;
    M32[gid] = k < nc ? (float)M[cell * ldm + k] : 0.0f;
}

// ------------------------------------------------------------------ FP32 halo M2L
//
// Same work unit (target octant o, 4x4x4 parent block), reorganised around
// the sources: for each source octant q the 6x6x6 halo of octant-q cells
// around the block (parents base-1 .. base+4) is staged in LDS once, and the
// 27 parent offsets u (v = 2u + q - o, the adjacent ones skipped) are all
// served from it: 189 offsets cost 8 halo stagings instead of 189 source
// stagings.  K_v does not go through LDS: every wave loads its A fragments
// straight into registers from the four-chunk layout (16-byte loads), one
// offset ahead in a second register set, so the offsets need no barrier,
// only the 8 stagings do; the waves of a workgroup read the same K_v, which
// the vector L1 cache serves.
template <int P>
struct Halo32 {
    using T = Tile<P, PREC_F32>;
    static constexpr int U = T::S32 / 4;           // 16-byte units per row
    // rows padded by 16 bytes so consecutive rows start on other banks (a
    // rotation of the units within each row, conflict-free, measured slower:
    // its per-read address arithmetic costs more than the 2-way conflicts)
    static constexpr int HROWB = T::S32 * 4 + 16;
    static constexpr int HBYTES = 216 * HROWB;
};

template <int P>
__global__ __launch_bounds__(256) void k_m2l_halo32(int level, const float* __restrict__ M32, double* __restrict__ L,
                                                     const float* __restrict__ Kf, const int16_t* __restrict__ hlist,
                                                     const unsigned char* __restrict__ zero_row,
                                                     const double* __restrict__ Lpar, const double* __restrict__ l2l_t) {
    using S = Tile<P, PREC_F32>;
    using H = Halo32<P>;
    constexpr int NC = S::NC, LDM = S::LDM, R = S::R, NB = S::NB, NCH = S::NCH, U = H::U;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    unsigned char* Hb = lds;  // [216][S32] floats, rows padded
    const long long work = xcd_remap(blockIdx.x, gridDim.x);
    const int o = (int)(work & 7);
    const long long pb = work >> 3;
    constexpr int NW = 4;
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int np1 = 1 << (level - 1);
    const long long nparents = (long long)np1 * np1 * np1;
    const uint32_t base_m = (uint32_t)(pb * 64);
    const int bx = (int)compact3(base_m), by = (int)compact3(base_m >> 1), bz = (int)compact3(base_m >> 2);
    const int tloc = w * 16 + (lane & 15);
    const int tx = (int)compact3((uint32_t)tloc), ty = (int)compact3((uint32_t)tloc >> 1),
              tz = (int)compact3((uint32_t)tloc >> 2);
    const int kq = lane >> 4;
    // the octant's offset list in LDS (read per offset without a memory wait)
    __shared__ int16_t qu_list[189], ks_list[189];
    for (int x = tid; x < 189; x += 64 * NW) {
        qu_list[x] = hlist[o * 189 + x];
        ks_list[x] = hlist[8 * 189 + o * 189 + x];
    }
    __syncthreads();
    // The halo of octant q is loaded into registers (NHU 16-byte units per
    // thread) while the previous octant's offsets run, and written to LDS at
    // the switch.  Cell h of the halo is the octant-q child of parent
    // (bx-1 + h%6, by-1 + h/6%6, bz-1 + h/36): row 8 morton(parent) + q, or
    // none outside the grid (hrow = -1).
    __shared__ int hrow[216];
    for (int h = tid; h < 216; h += 64 * NW) {
        const int px = bx - 1 + h % 6, py = by - 1 + (h / 6) % 6, pz = bz - 1 + h / 36;
        hrow[h] = (px >= 0 && py >= 0 && pz >= 0 && px < np1 && py < np1 && pz < np1) ? (int)(8 * morton3(px, py, pz))
                                                                                     : -1;
    }
    __syncthreads();
    constexpr int NHU = (216 * U + 64 * NW - 1) / (64 * NW);
    float hv[4 * NHU];
    auto load_halo = [&](int q) {
#pragma unroll
        for (int k = 0; k < NHU; ++k) {
            const int unit = k * 64 * NW + tid;
            if (unit < 216 * U) {
                const int h = unit / U, uu = unit - h * U;
                const int row = hrow[h];
                const float4* g = row >= 0 ? reinterpret_cast<const float4*>(M32 + (size_t)(row + q) * S::S32) + uu
                                           : reinterpret_cast<const float4*>(zero_row) + uu;
                const float4 v = *g;
                hv[4 * k] = v.x;
                hv[4 * k + 1] = v.y;
                hv[4 * k + 2] = v.z;
                hv[4 * k + 3] = v.w;
            }
        }
        // the row-table reads first, then the loads (else each load waits
        // for its own table read)
        __builtin_amdgcn_sched_group_barrier(0x100, NHU, 0);
        __builtin_amdgcn_sched_group_barrier(0x020, NHU, 0);
    };
    auto store_halo = [&]() {
#pragma unroll
        for (int k = 0; k < NHU; ++k) {
            const int unit = k * 64 * NW + tid;
            if (unit < 216 * U) {
                const int h = unit / U, uu = unit - h * U;
                *reinterpret_cast<float4*>(Hb + (size_t)h * H::HROWB + uu * 16) =
                    make_float4(hv[4 * k], hv[4 * k + 1], hv[4 * k + 2], hv[4 * k + 3]);
            }
        }
    };
    constexpr int NQ = (NCH + 3) / 4;  // 16-byte loads per lane and offset
    auto load_a = [&](int ks, float (&a)[4 * NQ]) {
        const float4* ka = reinterpret_cast<const float4*>(Kf) + (size_t)ks * (NQ * 64) + lane;
#pragma unroll
        for (int g = 0; g < NQ; ++g) {
            const float4 v = ka[g * 64];
            a[4 * g] = v.x;
            a[4 * g + 1] = v.y;
            a[4 * g + 2] = v.z;
            a[4 * g + 3] = v.w;
        }
    };
    v4f acc[R][2];
    v4f acc0[4];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r][0] = acc[r][1] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 4; ++k) acc0[k] = v4f{0.f, 0.f, 0.f, 0.f};
    int qcur = -1;
    // list entries read a step ahead (their LDS reads then never wait): the
    // octant and parent offset of this step's offset, the operator slot of
    // the next one
    int qu_c = qu_list[0], ks_n = ks_list[1];
    auto step = [&](int iv, const float (&a)[4 * NQ], float (&an)[4 * NQ]) {
        const int qu = __builtin_amdgcn_readfirstlane(qu_c);
        const int ks1 = __builtin_amdgcn_readfirstlane(ks_n);
        qu_c = qu_list[iv + 1 < 189 ? iv + 1 : iv];
        ks_n = ks_list[iv + 2 < 189 ? iv + 2 : 188];
        const int q = qu >> 5, u = qu & 31;
        if (q != qcur) {
            __syncthreads();  // every wave is done with the previous halo
            store_halo();
            __syncthreads();
            qcur = q;
            // the next octant's halo (offsets are grouped by octant) arrives
            // while this one's offsets run
            int qn = -1;
            for (int j = iv + 1; j < 189 && qn < 0; ++j)
                if ((qu_list[j] >> 5) != q) qn = qu_list[j] >> 5;
            if (qn >= 0) load_halo(__builtin_amdgcn_readfirstlane(qn));
        }
        load_a(ks1, an);  // the next offset's fragments (the last offset's again past the end)
        // keep those loads here: otherwise they are sunk to their first use
        // in the next step, which then waits for them
        __asm__ volatile("" ::: "memory");
        const int ux = u % 3 - 1, uy = (u / 3) % 3 - 1, uz = u / 9 - 1;
        const int h = (tx + 1 + ux) + 6 * (ty + 1 + uy) + 36 * (tz + 1 + uz);
        const float* Bf = reinterpret_cast<const float*>(Hb + (size_t)h * H::HROWB);
        // all B values of the offset first (one wait, not one per column)
        float b[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) b[c] = Bf[4 * c + kq];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            acc0[c & 3] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[S::pos(0, c)], b[c], acc0[c & 3], 0, 0, 0);
#pragma unroll
            for (int r = 1; r < R; ++r)
                if (c < S::nch(r))
                    acc[r][c & 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[S::pos(r, c)], b[c], acc[r][c & 1], 0, 0, 0);
        }
        // the B reads as one group ahead of the MFMAs (the compiler would
        // move each read down to its first use and wait for it there)
        __builtin_amdgcn_sched_group_barrier(0x100, NB, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, NCH, 0);
    };
    float a0[4 * NQ], a1[4 * NQ];
    load_halo(__builtin_amdgcn_readfirstlane((int)qu_list[0] >> 5));
    load_a(__builtin_amdgcn_readfirstlane((int)ks_list[0]), a0);
    for (int iv = 0; iv < 189; iv += 2) {
        step(iv, a0, a1);
        if (iv + 1 >= 189) break;
        step(iv + 1, a1, a0);
    }
    const long long par = pb * 64 + tloc;
    auto m2l_sum = [&](int r, int j) {
        return r == 0 ? ((double)acc0[0][j] + (double)acc0[1][j]) + ((double)acc0[2][j] + (double)acc0[3][j])
                      : (double)acc[r][0][j] + (double)acc[r][1][j];
    };
    if (!Lpar) {
        if (par >= nparents) return;
        double* Lt = L + (size_t)(par * 8 + o) * LDM;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int row0 = 16 * r + 4 * kq;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (row0 + j < NC) Lt[row0 + j] = m2l_sum(r, j);
        }
        return;
    }
    // With the parents' local expansions (levels below the first): L2L from
    // the parent, child L~ += B_o L~_parent (Eq. L2L in scaled form), added
    // here in FP64 on the matrix cores, so that L is written once.  The
    // 16x16 FP64 accumulators hold rows 16r + lane/16 + 4j, the FP32 ones
    // rows 16r + 4 lane/16 + j: the M2L sums go through LDS (the halo's
    // space, 128 rows per target) into the FP64 layout.  B_o[n][j] vanishes
    // for rank(j) < rank(n), so row tile r starts at column rank(16 r)^2.
    static_assert(64 * 16 * R * 8 <= H::HBYTES, "the M2L sums fit the halo's LDS");
    __syncthreads();  // every wave is done with the halo
    double* Ls = reinterpret_cast<double*>(Hb) + (size_t)tloc * 16 * R;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < 4; ++j) Ls[16 * r + 4 * kq + j] = m2l_sum(r, j);
    constexpr int NKC = (NC + 3) / 4;
    const bool valid = par < nparents;
    const double* lp = Lpar + (size_t)(valid ? par : 0) * LDM;
    double bp[NKC];
#pragma unroll
    for (int c = 0; c < NKC; ++c) bp[c] = (valid && 4 * c + kq < NC) ? lp[4 * c + kq] : 0.0;
    const double* Bo = l2l_t + (size_t)o * NIND * NIND;
    double* Lt = L + (size_t)(valid ? par * 8 + o : 0) * LDM;
    // the operator fragments of row tile r + 1 are loaded while r runs
    double af0[NKC], af1[NKC];
    auto load_af = [&](int r, double (&af)[NKC]) {
        const int n = 16 * r + (lane & 15);
#pragma unroll
        for (int c = 0; c < NKC; ++c) {
            const int jj = 4 * c + kq;
            af[c] = (c >= rank_ce(16 * r) * rank_ce(16 * r) / 4 && n < NC && jj < NC) ? Bo[(size_t)jj * NIND + n] : 0.0;
        }
    };
    auto tile = [&](int r, const double (&af)[NKC]) {
        v4d a64;
#pragma unroll
        for (int j = 0; j < 4; ++j) a64[j] = Ls[16 * r + kq + 4 * j];
#pragma unroll
        for (int c = 0; c < NKC; ++c)
            if (c >= rank_ce(16 * r) * rank_ce(16 * r) / 4)
                a64 = __builtin_amdgcn_mfma_f64_16x16x4f64(af[c], bp[c], a64, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = 16 * r + kq + 4 * j;
            if (valid && row < NC) Lt[row] = a64[j];
        }
    };
    load_af(0, af0);
#pragma unroll
    for (int r = 0; r < R; r += 2) {
        if (r + 1 < R) load_af(r + 1, af1);
        __asm__ volatile("" ::: "memory");  // (keeps the loads ahead of the MFMAs)
        tile(r, af0);
        if (r + 1 >= R) break;
        if (r + 2 < R) load_af(r + 2, af0);
        __asm__ volatile("" ::: "memory");
        tile(r + 1, af1);
    }
}

template <int P>
hipError_t m2l_halo32_impl(hipStream_t s, int level, const float* M32, double* L, const int16_t* hlist,
                           const unsigned char* zero_row, const float* Kq, const double* Lpar, const double* l2l_t) {
    if (!Kq) return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_m2l_halo32<P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           Halo32<P>::HBYTES);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const long long nparents = 1ll << (3 * (level - 1));
    const long long nblk = (nparents + 63) / 64;
    hipLaunchKernelGGL(k_m2l_halo32<P>, dim3((unsigned)(8 * nblk)), dim3(256), Halo32<P>::HBYTES, s, level, M32, L,
                       Kq, hlist, zero_row, Lpar, l2l_t);
    return hipGetLastError();
}

template <int P, int PREC, bool ADAPT, int NW = 4, bool ORD = false>
hipError_t m2l_tile_impl(hipStream_t s, int level, long long nwork, const void* Msrc, double* L,
                         const unsigned char* Kpk, const int16_t* offlist, const unsigned char* zero_row,
                         const AdaptM2L& ad_in) {
    using S = Tile<P, PREC, 16 * NW>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_m2l_tile<P, PREC, ADAPT, NW, ORD>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, S::LDS);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    AdaptM2L ad = ad_in;
    for (int q = 0; q <= P; ++q) ad.nup[q] = S::PT.nup[q];
    hipLaunchKernelGGL((k_m2l_tile<P, PREC, ADAPT, NW, ORD>), dim3((unsigned)nwork), dim3(64 * NW), S::LDS, s, level,
                       Msrc, L, Kpk, offlist, zero_row, ad);
    return hipGetLastError();
}

template <int P, int PREC>
hipError_t m2l_tile_impl(hipStream_t s, int level, const void* Msrc, double* L, const unsigned char* Kpk,
                         const int16_t* offlist, const unsigned char* zero_row) {
    const long long nparents = 1ll << (3 * (level - 1));
    const long long nblk = (nparents + 63) / 64;
    return m2l_tile_impl<P, PREC, false>(s, level, 8 * nblk, Msrc, L, Kpk, offlist, zero_row, AdaptM2L{});
}

template <int P, int PREC>
void pack_k_impl(hipStream_t s, const double* Kt, unsigned char* Kpk, int pmask) {
    using S = Tile<P, PREC>;
    const long long tot = (long long)NOFF * S::NCH * 64;
    hipLaunchKernelGGL((k_pack_k<P, PREC>), dim3(cdiv(tot, 256)), dim3(256), 0, s, Kt, Kpk, pmask);
}

#define CTFMM_P_CASES(X) X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10)

template <int PREC>
static size_t tile_query(int p, int what) {
    switch (p) {
#define CASE(PP) \
    case PP: return what == 0 ? (size_t)NOFF * Tile<PP, PREC>::KBYTES : what == 1 ? (size_t)Tile<PP, PREC>::LDS : 0;
        CTFMM_P_CASES(CASE)
#undef CASE
        default: return 0;
    }
}

size_t m2l_packed_bytes(int p, int prec) {
    return prec == PREC_F64 ? tile_query<PREC_F64>(p, 0) : prec == PREC_F32 ? tile_query<PREC_F32>(p, 0)
                                                                            : tile_query<PREC_BF16X3>(p, 0);
}

template <int PREC, int TT>
static size_t tile_lds(int p) {
    switch (p) {
#define CASE(PP) case PP: return (size_t)Tile<PP, PREC, TT>::LDS;
        CTFMM_P_CASES(CASE)
#undef CASE
        default: return 0;
    }
}

template <int TT>
static size_t tile_lds_prec(int p, int prec) {
    return prec == PREC_F64 ? tile_lds<PREC_F64, TT>(p) : prec == PREC_F32 ? tile_lds<PREC_F32, TT>(p)
                                                                           : tile_lds<PREC_BF16X3, TT>(p);
}

size_t m2l_tile_lds_bytes(int p, int prec, int tt) {
    return STATIC_LDS +
           (tt == 32 ? tile_lds_prec<32>(p, prec) : tt == 128 ? tile_lds_prec<128>(p, prec) : tile_lds_prec<64>(p, prec));
}

size_t m2l_lds_bytes(int p, int prec) {
    if (prec == PREC_F32) {
        switch (p) {
#define CASE(PP) case PP: return (size_t)Halo32<PP>::HBYTES + 1024;
            CTFMM_P_CASES(CASE)
#undef CASE
            default: return 0;
        }
    }
    return prec == PREC_F64 ? tile_query<PREC_F64>(p, 1) : tile_query<PREC_BF16X3>(p, 1);
}

void launch_pack_k(hipStream_t s, int p, int prec, const double* Kt, unsigned char* Kpk, int pmask) {
    switch (p) {
#define CASE(PP)                                                                    \
    case PP:                                                                        \
        if (prec == PREC_F64) pack_k_impl<PP, PREC_F64>(s, Kt, Kpk, pmask);        \
        else if (prec == PREC_F32) pack_k_impl<PP, PREC_F32>(s, Kt, Kpk, pmask);   \
        else pack_k_impl<PP, PREC_BF16X3>(s, Kt, Kpk, pmask);                      \
        break;
        CTFMM_P_CASES(CASE)
#undef CASE
        default: break;
    }
}

void launch_to_f32(hipStream_t s, int p, long long ncell, const double* M, float* M32) {
    const int nc = (p + 1) * (p + 1);
    const int s32 = ((nc + 31) / 32) * 32;
    hipLaunchKernelGGL(k_to_f32, dim3(cdiv(ncell * s32, 256)), dim3(256), 0, s, ncell, nc, ldm_of(p), s32, M, M32);
}

__global__ void k_quad_k(long long total, int nch, int nq, const float* __restrict__ Kf, float* __restrict__ Kq) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= total) return;
    const int j = (int)(gid % 4), lane = (int)((gid / 4) % 64);
    const long long gq = gid / 256;
    const int g = (int)(gq % nq);
    const long long slot = gq / nq;
    const int ch = 4 * g + j;
    Kq[gid] = ch < nch ? Kf[(slot * nch + ch) * 64 + lane] : 0.0f;
}

size_t m2l_quad_bytes(int p) {
    size_t nch = 0;
    switch (p) {
#define CASE(PP) case PP: nch = Tile<PP, PREC_F32>::NCH; break;
        CTFMM_P_CASES(CASE)
#undef CASE
        default: break;
    }
    return (size_t)NOFF * ((nch + 3) / 4) * 256 * sizeof(float);
}

void launch_quad_k(hipStream_t s, int p, const unsigned char* Kpk, float* Kq) {
    int nch = 0;
    switch (p) {
#define CASE(PP) case PP: nch = Tile<PP, PREC_F32>::NCH; break;
        CTFMM_P_CASES(CASE)
#undef CASE
        default: return;
    }
    const int nq = (nch + 3) / 4;
    const long long total = (long long)NOFF * nq * 256;
    hipLaunchKernelGGL(k_quad_k, dim3((unsigned)cdiv(total, 256)), dim3(256), 0, s, total, nch, nq,
                       reinterpret_cast<const float*>(Kpk), Kq);
}

hipError_t launch_m2l(hipStream_t s, int p, int prec, int level, const void* Msrc, double* L, const unsigned char* Kpk,
                      const int16_t* offlist, const unsigned char* zero_row, const float* Kq, const double* Lpar,
                      const double* l2l_t) {
    switch (p) {
#define CASE(PP)                                                                                           \
    case PP:                                                                                               \
        if (prec == PREC_F64) return m2l_tile_impl<PP, PREC_F64>(s, level, Msrc, L, Kpk, offlist, zero_row); \
        if (prec == PREC_F32) return m2l_halo32_impl<PP>(s, level, (const float*)Msrc, L, offlist, zero_row, Kq, Lpar, l2l_t); \
        return m2l_tile_impl<PP, PREC_BF16X3>(s, level, Msrc, L, Kpk, offlist, zero_row);
        CTFMM_P_CASES(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

template <int P, int NW, bool ORD>
hipError_t m2l_tables_prec(hipStream_t s, int prec, int ntiles, const AdaptM2L& ad, const void* Msrc, double* L,
                           const unsigned char* Kpk, const unsigned char* zero_row) {
    if (prec == PREC_F64)
        return m2l_tile_impl<P, PREC_F64, true, NW, ORD>(s, 0, ntiles, Msrc, L, Kpk, nullptr, zero_row, ad);
    if (prec == PREC_F32)
        return m2l_tile_impl<P, PREC_F32, true, NW, ORD>(s, 0, ntiles, Msrc, L, Kpk, nullptr, zero_row, ad);
    return m2l_tile_impl<P, PREC_BF16X3, true, NW, ORD>(s, 0, ntiles, Msrc, L, Kpk, nullptr, zero_row, ad);
}

// L = the sum of the nslots partial slots, in slot order, over the M2L
// targets (rows from row0, the first nc of ldm columns); zero elsewhere
// (the slots hold nothing defined there)
__global__ void k_sum_chunks(int nslots, size_t stride, const double* __restrict__ part, double* __restrict__ L, int nc,
                             int ldm, long long row0) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= stride) return;
    double v = 0.0;
    if ((int)(i % ldm) < nc && (long long)(i / ldm) >= row0)
        for (int c = 0; c < nslots; ++c) v += part[c * stride + i];
    L[i] = v;
}

void launch_sum_chunks(hipStream_t s, int nslots, size_t stride, const double* part, double* L, int nc, int ldm,
                       long long row0) {
    if (stride == 0) return;
    hipLaunchKernelGGL(k_sum_chunks, dim3(cdiv((long long)stride, 256)), dim3(256), 0, s, nslots, stride, part, L, nc,
                       ldm, row0);
}

void launch_to_f32_kq(hipStream_t s, int p, long long ncell, const double* M, float* M32) {
    const int s32 = s32_of(p);
    if (ncell <= 0) return;
    hipLaunchKernelGGL(k_to_f32_kq, dim3(cdiv(ncell * s32, 256)), dim3(256), 0, s, ncell, (p + 1) * (p + 1), ldm_of(p),
                       s32, M, M32);
}

template <int P, int NW, bool ORD>
hipError_t m2l_rb_impl(hipStream_t s, int nwork, const AdaptM2L& ad_in, const float* M32k, double* L,
                       const unsigned char* Kpk, const unsigned char* zero_row) {
    AdaptM2L ad = ad_in;
    for (int q = 0; q <= P; ++q) ad.nup[q] = Tile<P, PREC_F32, 16 * NW>::PT.nup[q];
    hipLaunchKernelGGL((k_m2l_rb<P, NW, ORD>), dim3((unsigned)nwork), dim3(64 * NW), 0, s, M32k, L, Kpk,
                       reinterpret_cast<const float*>(zero_row), ad);
    return hipGetLastError();
}

hipError_t launch_m2l_rb(hipStream_t s, int p, int tt, int ntiles_in, const AdaptM2L& ad, const float* M32k, double* L,
                         const unsigned char* Kpk, const unsigned char* zero_row) {
    if (ntiles_in <= 0) return hipSuccess;
    if (tt != 32 && tt != 64 && tt != 128) return hipErrorInvalidValue;
    if (ad.nchunk < 1 || (ad.nchunk > 1 && !ad.acc) || (ad.ivord && !ad.ivlist)) return hipErrorInvalidValue;
    const int nwork = ntiles_in * ad.nchunk;
    const bool ord = ad.ivord != nullptr;
    switch (p) {
#define CASE(PP)                                                                                          \
    case PP:                                                                                              \
        if (tt == 32) return ord ? m2l_rb_impl<PP, 2, true>(s, nwork, ad, M32k, L, Kpk, zero_row)         \
                                 : m2l_rb_impl<PP, 2, false>(s, nwork, ad, M32k, L, Kpk, zero_row);       \
        if (tt == 128) return ord ? m2l_rb_impl<PP, 8, true>(s, nwork, ad, M32k, L, Kpk, zero_row)        \
                                  : m2l_rb_impl<PP, 8, false>(s, nwork, ad, M32k, L, Kpk, zero_row);      \
        return ord ? m2l_rb_impl<PP, 4, true>(s, nwork, ad, M32k, L, Kpk, zero_row)                       \
                   : m2l_rb_impl<PP, 4, false>(s, nwork, ad, M32k, L, Kpk, zero_row);
        CTFMM_P_CASES(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_m2l_tables(hipStream_t s, int p, int prec, int tt, int ntiles_in, const AdaptM2L& ad,
                             const void* Msrc, double* L, const unsigned char* Kpk, const unsigned char* zero_row) {
    if (ntiles_in <= 0) return hipSuccess;
    if (tt != 32 && tt != 64 && tt != 128) return hipErrorInvalidValue;
    if (ad.nchunk < 1 || (ad.nchunk > 1 && !ad.acc) || (ad.ivord && !ad.ivlist)) return hipErrorInvalidValue;
    const int ntiles = ntiles_in * ad.nchunk;  // workgroups
    const bool ord = ad.ivord != nullptr;
    switch (p) {
#define CASE(PP)                                                                                                  \
    case PP:                                                                                                      \
        if (tt == 32) return ord ? m2l_tables_prec<PP, 2, true>(s, prec, ntiles, ad, Msrc, L, Kpk, zero_row)      \
                                 : m2l_tables_prec<PP, 2, false>(s, prec, ntiles, ad, Msrc, L, Kpk, zero_row);    \
        if (tt == 128) return ord ? m2l_tables_prec<PP, 8, true>(s, prec, ntiles, ad, Msrc, L, Kpk, zero_row)     \
                                  : m2l_tables_prec<PP, 8, false>(s, prec, ntiles, ad, Msrc, L, Kpk, zero_row);   \
        return ord ? m2l_tables_prec<PP, 4, true>(s, prec, ntiles, ad, Msrc, L, Kpk, zero_row)                    \
                   : m2l_tables_prec<PP, 4, false>(s, prec, ntiles, ad, Msrc, L, Kpk, zero_row);
        CTFMM_P_CASES(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ctfmm
