// Device kernels of libctfmm (gfx950): tree keys, P2M, M2M, per-offset M2L
// operator matrices, M2L, L2L, L2P and the P2P near field.
//
// Expansions are stored in scaled form on a Morton-ordered uniform octree:
// level l holds 8^l cells, cell m at M[(m * nc) + k] with nc = (p+1)^2
// independent traceless components k (ordered by rank, then n_z, then n_x
// descending).  With h the cell side, M~_k = M_k / h^|k| and
// L~_k = L_k h^(|k|+1); then the M2L operator of an integer offset v is the
// same at every level (grad^n r^-1 is homogeneous of degree -n-1) and the
// M2M/L2L shifts are constant per octant.
#include <math.h>

#include "ctfmm_internal.h"

namespace ctfmm {

static inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

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

// One wavefront per leaf.  For each particle, the power table of
// u = (z - x)/h and |u|^2 is built in LDS; each lane then sums the compact
// detracer terms (Eq. Detracer3) of its independent slot(s).
__global__ __launch_bounds__(64) void k_p2m(int p, Box box, const int32_t* __restrict__ start,
                                            const double4* __restrict__ P, DevTables T, double* __restrict__ M) {
    const uint32_t c = blockIdx.x;
    const int lane = threadIdx.x;
    const int nc = (p + 1) * (p + 1);
    const int d = box.depth;
    const double h = box.side / (double)(1 << d);
    const double zx = box.lo[0] + ((double)compact3(c) + 0.5) * h;
    const double zy = box.lo[1] + ((double)compact3(c >> 1) + 0.5) * h;
    const double zz = box.lo[2] + ((double)compact3(c >> 2) + 0.5) * h;
    __shared__ double pw[4][PMAX + 1];
    double acc0 = 0.0, acc1 = 0.0;
    const int b = start[c], e = start[c + 1];
    const int s0 = lane, s1 = lane + 64;
    const int t0b = s0 < nc ? T.p2m_start[s0] : 0, t0e = s0 < nc ? T.p2m_start[s0 + 1] : 0;
    const int t1b = s1 < nc ? T.p2m_start[s1] : 0, t1e = s1 < nc ? T.p2m_start[s1 + 1] : 0;
    for (int s = b; s < e; ++s) {
        const double4 pt = P[s];
        const double ux = (zx - pt.x) / h, uy = (zy - pt.y) / h, uz = (zz - pt.z) / h;
        if (lane < 4 * (p + 1)) {
            const int dim = lane / (p + 1), ex = lane % (p + 1);
            const double base = dim == 0 ? ux : dim == 1 ? uy : dim == 2 ? uz : (ux * ux + uy * uy + uz * uz);
            double v = 1.0;
            for (int t = 0; t < ex; ++t) v *= base;
            pw[dim][ex] = v;
        }
        __syncthreads();
        double v0 = 0.0, v1 = 0.0;
        for (int t = t0b; t < t0e; ++t) {
            const int8_t* ex = T.p2m_exp + 4 * t;
            v0 += T.p2m_coef[t] * pw[0][ex[0]] * pw[1][ex[1]] * pw[2][ex[2]] * pw[3][ex[3]];
        }
        for (int t = t1b; t < t1e; ++t) {
            const int8_t* ex = T.p2m_exp + 4 * t;
            v1 += T.p2m_coef[t] * pw[0][ex[0]] * pw[1][ex[1]] * pw[2][ex[2]] * pw[3][ex[3]];
        }
        acc0 += pt.w * v0;
        acc1 += pt.w * v1;
        __syncthreads();
    }
    double* Mc = M + (size_t)c * nc;
    if (s0 < nc) Mc[s0] = acc0;
    if (s1 < nc) Mc[s1] = acc1;
}

void launch_p2m(hipStream_t s, int p, Box box, const int32_t* start, const double4* P, const DevTables& T, double* M) {
    const long long nleaves = 1ll << (3 * box.depth);
    hipLaunchKernelGGL(k_p2m, dim3((unsigned)nleaves), dim3(64), 0, s, p, box, start, P, T, M);
}

// ------------------------------------------------------------------ M2M

// parent M~ = sum over the 8 children o of A_o M~_child (Eq. M2M in scaled form)
__global__ __launch_bounds__(128) void k_m2m(int p, const double* __restrict__ Mc, double* __restrict__ Mp,
                                             const double* __restrict__ m2m_t) {
    const uint32_t P = blockIdx.x;
    const int nc = (p + 1) * (p + 1);
    __shared__ double ch[8 * NIND];
    const double* src = Mc + (size_t)8 * P * nc;
    for (int t = threadIdx.x; t < 8 * nc; t += 128) ch[(t / nc) * NIND + (t % nc)] = src[t];
    __syncthreads();
    const int n = threadIdx.x;
    if (n < nc) {
        double acc = 0.0;
        for (int o = 0; o < 8; ++o) {
            const double* A = m2m_t + (size_t)o * NIND * NIND;
            for (int j = 0; j < nc; ++j) acc += A[(size_t)j * NIND + n] * ch[o * NIND + j];
        }
        Mp[(size_t)P * nc + n] = acc;
    }
}

void launch_m2m(hipStream_t s, int p, int parent_level, const double* Mchild, double* Mparent, const DevTables& T) {
    const long long np = 1ll << (3 * parent_level);
    hipLaunchKernelGGL(k_m2m, dim3((unsigned)np), dim3(128), 0, s, p, Mchild, Mparent, T.m2m_t);
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

__device__ inline int rank_of(int k) {
    int r = 0;
    while ((r + 1) * (r + 1) <= k) ++r;
    return r;
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

// ------------------------------------------------------------------ M2L (FP64)

// One target cell per workgroup: L~_T = sum over the ws=1 interaction list
// (children of the parent's neighbours that are not adjacent to T) of
// K_{T-S} M~_S.
__global__ __launch_bounds__(128) void k_m2l_fp64(int p, int level, const double* __restrict__ M,
                                                  double* __restrict__ L, const double* __restrict__ Kt) {
    const uint32_t T = blockIdx.x;
    const int nc = (p + 1) * (p + 1);
    const int n1 = 1 << level;
    const int ix = compact3(T), iy = compact3(T >> 1), iz = compact3(T >> 2);
    const int I = ix >> 1, J = iy >> 1, K = iz >> 1;
    __shared__ double Ms[NIND];
    const int n = threadIdx.x;
    double acc = 0.0;
    for (int c = 2 * K - 2; c <= 2 * K + 3; ++c) {
        if (c < 0 || c >= n1) continue;
        for (int b = 2 * J - 2; b <= 2 * J + 3; ++b) {
            if (b < 0 || b >= n1) continue;
            for (int a = 2 * I - 2; a <= 2 * I + 3; ++a) {
                if (a < 0 || a >= n1) continue;
                if (abs(a - ix) <= 1 && abs(b - iy) <= 1 && abs(c - iz) <= 1) continue;
                const uint32_t S = morton3(a, b, c);
                __syncthreads();
                if (n < nc) Ms[n] = M[(size_t)S * nc + n];
                __syncthreads();
                const int vs = (ix - a + 3) + 7 * (iy - b + 3) + 49 * (iz - c + 3);
                const double* Kv = Kt + (size_t)vs * nc * nc;
                if (n < nc)
                    for (int j = 0; j < nc; ++j) acc += Kv[(size_t)j * nc + n] * Ms[j];
            }
        }
    }
    if (n < nc) L[(size_t)T * nc + n] = acc;
}

void launch_m2l_fp64(hipStream_t s, int p, int level, const double* M, double* L, const double* Kt) {
    const long long ncell = 1ll << (3 * level);
    hipLaunchKernelGGL(k_m2l_fp64, dim3((unsigned)ncell), dim3(128), 0, s, p, level, M, L, Kt);
}

// ------------------------------------------------------------------ L2L

// child L~_o += B_o L~_parent (Eq. L2L in scaled form)
__global__ __launch_bounds__(256) void k_l2l(int p, const double* __restrict__ Lp, double* __restrict__ Lc,
                                             const double* __restrict__ l2l_t) {
    const uint32_t P = blockIdx.x;
    const int nc = (p + 1) * (p + 1);
    __shared__ double lp[NIND];
    for (int t = threadIdx.x; t < nc; t += 256) lp[t] = Lp[(size_t)P * nc + t];
    __syncthreads();
    for (int t = threadIdx.x; t < 8 * nc; t += 256) {
        const int o = t / nc, n = t % nc;
        const double* B = l2l_t + (size_t)o * NIND * NIND;
        double acc = 0.0;
        for (int j = 0; j < nc; ++j) acc += B[(size_t)j * NIND + n] * lp[j];
        Lc[((size_t)8 * P + o) * nc + n] += acc;
    }
}

void launch_l2l(hipStream_t s, int p, int parent_level, const double* Lparent, double* Lchild, const DevTables& T) {
    const long long np = 1ll << (3 * parent_level);
    hipLaunchKernelGGL(k_l2l, dim3((unsigned)np), dim3(256), 0, s, p, Lparent, Lchild, T.l2l_t);
}

// ------------------------------------------------------------------ L2P + P2P

// position of (a,b,c) in full storage: rank-major, a descending, b descending
__host__ __device__ constexpr int full_slot(int a, int b, int c) {
    const int n = a + b + c;
    return n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + (n - a - b);
}

__device__ inline void pair_add(double xb, double yb, double zb, double4 src, double& f, double& gx, double& gy,
                                double& gz) {
    const double dx = xb - src.x, dy = yb - src.y, dz = zb - src.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) return;
    const double ir = 1.0 / sqrt(r2);
    f += src.w * ir;
    const double ir3 = src.w * ir * ir * ir;
    gx -= ir3 * dx;
    gy -= ir3 * dy;
    gz -= ir3 * dz;
}

// L2P (Eq. L2P): one workgroup per leaf.  The leaf's local expansion is
// expanded to full components divided by n! in LDS, together with the
// coefficient arrays of its three first derivatives; each particle then
// evaluates the four degree-p polynomials at r = (x - z)/h by nested Horner
// steps in x, y and z.  Results (far field, sorted order) go to F[s].
template <int P>
__global__ __launch_bounds__(64) void k_l2p(Box box, const int32_t* __restrict__ start, const double4* __restrict__ Pt,
                                            const double* __restrict__ L, DevTables T, double4* __restrict__ F) {
    constexpr int NC = (P + 1) * (P + 1);
    constexpr int NF = (P + 1) * (P + 2) * (P + 3) / 6;
    const uint32_t c = blockIdx.x;
    const int b0 = start[c], e0 = start[c + 1];
    if (b0 == e0) return;  // uniform across the workgroup
    const int d = box.depth;
    const double h = box.side / (double)(1 << d);
    const double zx = box.lo[0] + ((double)compact3(c) + 0.5) * h;
    const double zy = box.lo[1] + ((double)compact3(c >> 1) + 0.5) * h;
    const double zz = box.lo[2] + ((double)compact3(c >> 2) + 0.5) * h;
    __shared__ double W[4][NF];  // potential, d/dx, d/dy, d/dz coefficients
    const double* Lc = L + (size_t)c * NC;
    for (int f = threadIdx.x; f < NF; f += 64) {
        double v = 0.0;
        for (int t = T.exp_start[f]; t < T.exp_start[f + 1]; ++t) v += (double)T.exp_coef[t] * Lc[T.exp_slot[t]];
        W[0][f] = v * T.inv_mfact[f];
    }
    __syncthreads();
    for (int f = threadIdx.x; f < NF; f += 64) {
        const int a = T.full[3 * f], b = T.full[3 * f + 1], cc = T.full[3 * f + 2];
        const bool inner = a + b + cc < P;
        W[1][f] = inner ? (double)(a + 1) * W[0][full_slot(a + 1, b, cc)] : 0.0;
        W[2][f] = inner ? (double)(b + 1) * W[0][full_slot(a, b + 1, cc)] : 0.0;
        W[3][f] = inner ? (double)(cc + 1) * W[0][full_slot(a, b, cc + 1)] : 0.0;
    }
    __syncthreads();
    for (int s = b0 + threadIdx.x; s < e0; s += 64) {
        const double4 pt = Pt[s];
        const double rx = (pt.x - zx) / h, ry = (pt.y - zy) / h, rz = (pt.z - zz) / h;
        double f0 = 0.0, f1 = 0.0, f2 = 0.0, f3 = 0.0;
        for (int cz = P; cz >= 0; --cz) {
            double y0 = 0.0, y1 = 0.0, y2 = 0.0, y3 = 0.0;
            for (int by = P - cz; by >= 0; --by) {
                double x0 = 0.0, x1 = 0.0, x2 = 0.0, x3 = 0.0;
                for (int ax = P - by - cz; ax >= 0; --ax) {
                    const int sl = full_slot(ax, by, cz);
                    x0 = x0 * rx + W[0][sl];
                    x1 = x1 * rx + W[1][sl];
                    x2 = x2 * rx + W[2][sl];
                    x3 = x3 * rx + W[3][sl];
                }
                y0 = y0 * ry + x0;
                y1 = y1 * ry + x1;
                y2 = y2 * ry + x2;
                y3 = y3 * ry + x3;
            }
            f0 = f0 * rz + y0;
            f1 = f1 * rz + y1;
            f2 = f2 * rz + y2;
            f3 = f3 * rz + y3;
        }
        const double ih2 = 1.0 / (h * h);
        F[s] = make_double4(f0 / h, f1 * ih2, f2 * ih2, f3 * ih2);
    }
}

// P2P: one thread per (sorted) target particle; sources are the particles
// of the 27 adjacent-or-equal leaves (Appendix C near field), self excluded.
// Adds the far field F[s] (if given) and writes the outputs in input order.
__global__ __launch_bounds__(256) void k_p2p(int n, Box box, const uint32_t* __restrict__ keys,
                                             const int32_t* __restrict__ start, const double4* __restrict__ Pt,
                                             const int32_t* __restrict__ idx, const double4* __restrict__ F,
                                             double* __restrict__ phi, double* __restrict__ grad) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
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
                    pair_add(pt.x, pt.y, pt.z, Pt[s2], f, gx, gy, gz);
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

void launch_l2p(hipStream_t s, int p, Box box, const int32_t* start, const double4* P, const double* L,
                const DevTables& T, double4* F) {
    const long long nleaves = 1ll << (3 * box.depth);
    switch (p) {
#define CASE(PP)                                                                                              \
    case PP:                                                                                                  \
        hipLaunchKernelGGL(k_l2p<PP>, dim3((unsigned)nleaves), dim3(64), 0, s, box, start, P, L, T, F); \
        break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

void launch_p2p(hipStream_t s, int n, Box box, const uint32_t* keys, const int32_t* start, const double4* P,
                const int32_t* idx, const double4* F, double* phi, double* grad) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_p2p, dim3(cdiv(n, 256)), dim3(256), 0, s, n, box, keys, start, P, idx, F, phi, grad);
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
    double v = X[(size_t)m * nc + k];
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
// one small GEMM  L~[:, tile] += K_v[:, :] * M~[:, tile + v].
// Per offset, K_v (only its non-zero 16x4 blocks: rows of rank a need
// columns of rank <= p - a) and the 64 source multipoles are staged in LDS
// in MFMA fragment order; wave w owns targets 16w..16w+15 and all row tiles.

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

__host__ __device__ constexpr int rank_ce(int k) {
    int r = 0;
    while ((r + 1) * (r + 1) <= k) ++r;
    return r;
}

}  // namespace

template <int P>
struct Shape64 {
    static constexpr int NC = (P + 1) * (P + 1);
    static constexpr int R = (NC + 15) / 16;  // 16-row tiles
    // 4-column chunks needed by row tile r (its first row has the lowest rank)
    static constexpr int nch(int r) {
        const int m = P - rank_ce(16 * r) + 1;
        return (m * m + 3) / 4;
    }
    static constexpr int cb(int r) {
        int s = 0;
        for (int i = 0; i < r; ++i) s += nch(i);
        return s;
    }
    static constexpr int NCH = cb(R);  // packed chunks of one K_v
    static constexpr int NB = nch(0);  // chunks of one source multipole
};

// pack K_v into fragments: Kpk[v][chunk][lane], lane -> (row 16r + lane%16, col 4c + lane/16)
template <int P>
__global__ void k_pack_k64(const double* __restrict__ Kt, double* __restrict__ Kpk) {
    using S = Shape64<P>;
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (long long)NOFF * S::NCH * 64) return;
    const int lane = (int)(gid % 64);
    const int ch = (int)((gid / 64) % S::NCH);
    const int v = (int)(gid / (64ll * S::NCH));
    int r = 0;
    while (r + 1 < S::R && S::cb(r + 1) <= ch) ++r;
    const int c = ch - S::cb(r);
    const int row = 16 * r + (lane % 16), col = 4 * c + lane / 16;
    double val = 0.0;
    if (row < S::NC && col < S::NC) val = Kt[((size_t)v * S::NC + col) * S::NC + row];
    Kpk[gid] = val;
}

template <int P>
__global__ __launch_bounds__(256) void k_m2l_mfma64(int level, const double* __restrict__ M, double* __restrict__ L,
                                                    const double* __restrict__ Kpk,
                                                    const int16_t* __restrict__ offlist) {
    using S = Shape64<P>;
    constexpr int NC = S::NC, R = S::R, NCH = S::NCH, NB = S::NB;
    extern __shared__ double lds[];
    double* Ks = lds;                 // [NCH][64]
    double* Bs = lds + NCH * 64;      // [4][NB][64]
    __shared__ int srcrow[64];
    __shared__ int tgtrow[64];

    const int o = blockIdx.x & 7;
    const int pb = blockIdx.x >> 3;
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int n1 = 1 << level;
    const long long nparents = 1ll << (3 * (level - 1));
    if (tid < 64) {
        const long long par = (long long)pb * 64 + tid;
        tgtrow[tid] = par < nparents ? (int)(par * 8 + o) : -1;
    }

    v4d acc[R][2];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r][0] = acc[r][1] = v4d{0.0, 0.0, 0.0, 0.0};

    for (int iv = 0; iv < 189; ++iv) {
        const int vs = offlist[o * 189 + iv];
        const int vx = vs % 7 - 3, vy = (vs / 7) % 7 - 3, vz = vs / 49 - 3;
        __syncthreads();  // previous offset's fragments are consumed; tgtrow visible
        if (tid < 64) {
            const int t = tgtrow[tid];
            int row = -1;
            if (t >= 0) {
                const int sx = (int)compact3((uint32_t)t) + vx, sy = (int)compact3((uint32_t)t >> 1) + vy,
                          sz = (int)compact3((uint32_t)t >> 2) + vz;
                if (sx >= 0 && sy >= 0 && sz >= 0 && sx < n1 && sy < n1 && sz < n1) row = (int)morton3(sx, sy, sz);
            }
            srcrow[tid] = row;
        }
        // v is source - target; the operator is built for r = target - source = -v
        const double* Kv = Kpk + (size_t)(NOFF - 1 - vs) * NCH * 64;
        for (int i = tid; i < NCH * 64; i += 256) Ks[i] = Kv[i];
        __syncthreads();
        for (int e = tid; e < 4 * NB * 64; e += 256) {
            const int ln = e & 63;
            const int c = (e >> 6) % NB;
            const int ww = e / (64 * NB);
            const int row = srcrow[ww * 16 + (ln & 15)];
            const int k = 4 * c + (ln >> 4);
            Bs[e] = (row >= 0 && k < NC) ? M[(size_t)row * NC + k] : 0.0;
        }
        __syncthreads();
        const double* Bw = Bs + w * NB * 64;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const double b = Bw[c * 64 + lane];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (c < S::nch(r)) {
                    const double a = Ks[(S::cb(r) + c) * 64 + lane];
                    acc[r][c & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[r][c & 1], 0, 0, 0);
                }
            }
        }
    }
    // FP64 16x16 accumulator: element j of lane holds row 16r + lane/16 + 4j of target lane%16
    const int t = tgtrow[w * 16 + (lane & 15)];
    if (t >= 0) {
        double* Lt = L + (size_t)t * NC;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const v4d s = acc[r][0] + acc[r][1];
            const int row0 = 16 * r + (lane >> 4);
            if (row0 + 0 < NC) Lt[row0 + 0] = s.x;
            if (row0 + 4 < NC) Lt[row0 + 4] = s.y;
            if (row0 + 8 < NC) Lt[row0 + 8] = s.z;
            if (row0 + 12 < NC) Lt[row0 + 12] = s.w;
        }
    }
}

template <int P>
size_t m2l64_lds_bytes() {
    using S = Shape64<P>;
    return (size_t)(S::NCH * 64 + 4 * S::NB * 64) * sizeof(double);
}

template <int P>
void pack_k64_impl(hipStream_t s, const double* Kt, double* Kpk) {
    using S = Shape64<P>;
    const long long tot = (long long)NOFF * S::NCH * 64;
    hipLaunchKernelGGL(k_pack_k64<P>, dim3(cdiv(tot, 256)), dim3(256), 0, s, Kt, Kpk);
}

template <int P>
hipError_t m2l64_impl(hipStream_t s, int level, const double* M, double* L, const double* Kpk, const int16_t* offlist) {
    const size_t lds = m2l64_lds_bytes<P>();
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_m2l_mfma64<P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const long long nparents = 1ll << (3 * (level - 1));
    const long long nblk = (nparents + 63) / 64;
    hipLaunchKernelGGL(k_m2l_mfma64<P>, dim3((unsigned)(8 * nblk)), dim3(256), lds, s, level, M, L, Kpk, offlist);
    return hipGetLastError();
}

size_t m2l64_packed_doubles(int p) {
    switch (p) {
#define CASE(PP) case PP: return (size_t)NOFF * Shape64<PP>::NCH * 64;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: return 0;
    }
}

size_t m2l64_lds(int p) {
    switch (p) {
#define CASE(PP) case PP: return m2l64_lds_bytes<PP>();
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: return 0;
    }
}

void launch_pack_k64(hipStream_t s, int p, const double* Kt, double* Kpk) {
    switch (p) {
#define CASE(PP) case PP: pack_k64_impl<PP>(s, Kt, Kpk); break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

hipError_t launch_m2l_mfma64(hipStream_t s, int p, int level, const double* M, double* L, const double* Kpk,
                             const int16_t* offlist) {
    switch (p) {
#define CASE(PP) case PP: return m2l64_impl<PP>(s, level, M, L, Kpk, offlist);
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ctfmm
