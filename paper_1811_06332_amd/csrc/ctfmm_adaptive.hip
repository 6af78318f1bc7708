// Adaptive octree of libctfmm (gfx950): the tree and its interaction lists
// are built on the device from sorted 63-bit Morton keys, and the operators
// act on node lists.
//
// A node at level l is the set of particles whose key shares its top 3l bits
// (its Morton prefix).  A node holding more than leaf_max particles is split
// into its non-empty octants, down to level AMAX (Appendix C recommends a
// geometric split at the cell centre for inhomogeneous distributions).
// Interactions (the adaptive lists; every one evaluated with the paper's
// operators):
//   V(B): children of the same-level neighbours of parent(B) that are not
//         adjacent to B                                   -> M2L (Eq. M2L)
//   U(B), B a leaf: every leaf adjacent to B, B included  -> direct sum
//   W(B), B a leaf: descendants of B's same-level neighbours that are not
//         adjacent to B while their parent is             -> the multipole
//         expansion evaluated at B's particles
//   X(B): the leaves C with B in W(C); these are the leaves coarser than B
//         that touch parent(B) but not B                  -> the local
//         expansion of C's particles about B's centre
// "Adjacent" means that the closed cubes touch or overlap.
//
// Nodes are stored level by level (level l occupies a contiguous index
// range, Morton order inside it).  Every node keeps a 27-entry neighbour
// table: entry d = (dx+1) + 3 (dy+1) + 9 (dz+1) holds the same-level node
// at offset d if it exists, otherwise the coarser leaf covering that cell
// if there is one, otherwise -1.  It is built top-down from the parent's
// table, and every list above is read off these tables.
#include <math.h>

#include "ctfmm_internal.h"

namespace ctfmm {

namespace {

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

__device__ inline int node_level(int info) { return info & 0xff; }
__device__ inline bool node_leaf(int info) { return (info >> 8) & 1; }

struct NodeGeom {
    double zx, zy, zz, h;
};

__device__ inline NodeGeom node_geom(const ABox& box, uint64_t key, int level) {
    NodeGeom g;
    g.h = box.side / (double)(1ll << level);
    g.zx = box.lo[0] + ((double)compact21(key) + 0.5) * g.h;
    g.zy = box.lo[1] + ((double)compact21(key >> 1) + 0.5) * g.h;
    g.zz = box.lo[2] + ((double)compact21(key >> 2) + 0.5) * g.h;
    return g;
}

// closed cubes of (level la, prefix ka) and (level lb, prefix kb) touch or overlap
__device__ inline bool adjacent(uint64_t ka, int la, uint64_t kb, int lb) {
    const int sa = AMAX - la, sb = AMAX - lb;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const uint32_t a = compact21(ka >> d), b = compact21(kb >> d);
        const uint32_t alo = a << sa, ahi = (a + 1) << sa;
        const uint32_t blo = b << sb, bhi = (b + 1) << sb;
        if (alo > bhi || blo > ahi) return false;
    }
    return true;
}

// from the table filled by k_node_geo once per tree
__device__ inline NodeGeom node_geom(const ABox* boxes, const ATree& t, int g) {
    const double4 q = t.geo[g];
    return NodeGeom{q.x, q.y, q.z, q.w};
}

// position of i among the sorted offsets off[0..m] (off[k] <= i < off[k+1])
__device__ inline int seg_of(const int32_t* off, int m, int i) {
    int lo = 0, hi = m;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace

// ------------------------------------------------------------------ root cube

// per-block min and max of x, y, z
__global__ __launch_bounds__(256) void k_bbox_partial(int n, const double* __restrict__ xyz, double* __restrict__ part) {
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double v = xyz[3 * i + d];
            mn[d] = fmin(mn[d], v);
            mx[d] = fmax(mx[d], v);
        }
    }
    __shared__ double s[6][256];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        s[d][threadIdx.x] = mn[d];
        s[3 + d][threadIdx.x] = mx[d];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                s[d][threadIdx.x] = fmin(s[d][threadIdx.x], s[d][threadIdx.x + w]);
                s[3 + d][threadIdx.x] = fmax(s[3 + d][threadIdx.x], s[3 + d][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[(size_t)blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

// reduce the partials; out = (lo[3], side): the cube centred on the bounding
// box with side = largest extent * (1 + 2^-20), or 1 when all points coincide
__global__ __launch_bounds__(256) void k_bbox_final(int nparts, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double s6[6][256];
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nparts; b += 256)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            v[d] = fmin(v[d], part[6 * b + d]);
            v[3 + d] = fmax(v[3 + d], part[6 * b + 3 + d]);
        }
#pragma unroll
    for (int k = 0; k < 6; ++k) s6[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                s6[d][threadIdx.x] = fmin(s6[d][threadIdx.x], s6[d][threadIdx.x + w]);
                s6[3 + d][threadIdx.x] = fmax(s6[3 + d][threadIdx.x], s6[3 + d][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double mn[3] = {s6[0][0], s6[1][0], s6[2][0]}, mx[3] = {s6[3][0], s6[4][0], s6[5][0]};
    double s = 0.0;
    for (int d = 0; d < 3; ++d)
        if (mx[d] - mn[d] > s) s = mx[d] - mn[d];
    if (!(s > 0.0)) s = 1.0;
    s = s * (1.0 + 1.0 / 1048576.0);
    for (int d = 0; d < 3; ++d) {
        const double mid = (mn[d] + mx[d]) * 0.5;
        const double half = s * 0.5;
        out[d] = mid - half;
    }
    out[3] = s;
}

// one block per system: its automatic root cube (as k_bbox_final)
__global__ __launch_bounds__(256) void k_bbox_systems(ASys sy, const double* __restrict__ xyz, ABox* __restrict__ boxes) {
    const int sidx = blockIdx.x;
    const long long b = sy.gbase[sidx], cnt = sy.goff[sidx + 1] - sy.goff[sidx];
    __shared__ double s6[6][256];
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (long long i = threadIdx.x; i < cnt; i += 256)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double x = xyz[3 * (b + i) + d];
            v[d] = fmin(v[d], x);
            v[3 + d] = fmax(v[3 + d], x);
        }
#pragma unroll
    for (int k = 0; k < 6; ++k) s6[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                s6[d][threadIdx.x] = fmin(s6[d][threadIdx.x], s6[d][threadIdx.x + w]);
                s6[3 + d][threadIdx.x] = fmax(s6[3 + d][threadIdx.x], s6[3 + d][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double mn[3] = {s6[0][0], s6[1][0], s6[2][0]}, mx[3] = {s6[3][0], s6[4][0], s6[5][0]};
    double sd = 0.0;
    for (int d = 0; d < 3; ++d)
        if (mx[d] - mn[d] > sd) sd = mx[d] - mn[d];
    if (!(sd > 0.0)) sd = 1.0;
    sd = sd * (1.0 + 1.0 / 1048576.0);
    ABox bx;
    for (int d = 0; d < 3; ++d) {
        const double mid = (mn[d] + mx[d]) * 0.5;
        const double half = sd * 0.5;
        bx.lo[d] = cnt > 0 ? mid - half : 0.0;
    }
    bx.side = sd;
    boxes[sidx] = bx;
}

void launch_bbox_systems(hipStream_t s, const ASys& sy, const double* xyz, ABox* boxes) {
    hipLaunchKernelGGL(k_bbox_systems, dim3(sy.nsys), dim3(256), 0, s, sy, xyz, boxes);
}

void launch_bbox(hipStream_t s, int n, const double* xyz, double* part, int nparts, double* out) {
    hipLaunchKernelGGL(k_bbox_partial, dim3(nparts), dim3(256), 0, s, n, xyz, part);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(256), 0, s, nparts, part, out);
}

// ------------------------------------------------------------------ keys

// cell coordinate floor((x - lo)/side * 2^AMAX), clamped to [0, 2^AMAX - 1]
__device__ inline uint64_t acoord(double x, double lo, double side) {
    const double s = floor((x - lo) / side * (double)(1ll << AMAX));
    const long long top = (1ll << AMAX) - 1;
    if (!(s >= 0.0)) return 0;
    if (s > (double)top) return (uint64_t)top;
    return (uint64_t)s;
}

__global__ void k_clear_i32(int n, int32_t* __restrict__ a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0;
}

__device__ inline uint64_t morton63(double x, double y, double z, const ABox& box) {
    return spread21(acoord(x, box.lo[0], box.side)) | (spread21(acoord(y, box.lo[1], box.side)) << 1) |
           (spread21(acoord(z, box.lo[2], box.side)) << 2);
}

// keys[i]: the 63-bit Morton key of particle i of its system; k32[i] its top
// 32 bits (levels 1..10 and two bits of level 11)
// keys[i] = the 63-bit key, or with composite (several systems) the system
// index above the top 32 key bits, so that one radix sort orders the
// particles by system and then by cell down to level 10.
__global__ void k_keys64(int n, ASys sy, const double* __restrict__ xyz, const ABox* __restrict__ boxes,
                         uint64_t* __restrict__ keys, uint32_t* __restrict__ k32, int32_t* __restrict__ idx,
                         int* __restrict__ err, int composite) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int sidx = sy.nsys == 1 ? 0 : seg_of(sy.goff, sy.nsys, i);
    const size_t gi = (size_t)sy.gbase[sidx] + (size_t)(i - sy.goff[sidx]);
    const ABox box = boxes[sidx];
    const double x = xyz[3 * gi], y = xyz[3 * gi + 1], z = xyz[3 * gi + 2];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) atomicOr(err, 1);
    const uint64_t k = morton63(x, y, z, box);
    const uint32_t top = (uint32_t)(k >> (3 * AMAX - 32));
    keys[i] = composite ? ((uint64_t)sidx << 32) | top : k;
    k32[i] = top;
    idx[i] = (int32_t)gi;
}

void launch_keys64(hipStream_t s, int n, const ASys& sy, const double* xyz, const ABox* boxes, uint64_t* keys,
                   uint32_t* k32, int32_t* idx, int* err, bool composite) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_keys64, dim3(cdiv(n, 256)), dim3(256), 0, s, n, sy, xyz, boxes, keys, k32, idx, err,
                       composite ? 1 : 0);
}

// P and the full key of every sorted position j (the particle idx[j] of its system)
__global__ void k_gather_keyed(int n, ASys sy, const int32_t* __restrict__ idx, const double* __restrict__ xyz,
                               const double* __restrict__ q, const ABox* __restrict__ boxes, double4* __restrict__ P,
                               uint64_t* __restrict__ keys) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int sidx = sy.nsys == 1 ? 0 : seg_of(sy.goff, sy.nsys, j);
    const size_t gi = (size_t)idx[j];
    const double x = xyz[3 * gi], y = xyz[3 * gi + 1], z = xyz[3 * gi + 2];
    P[j] = make_double4(x, y, z, q[gi]);
    keys[j] = morton63(x, y, z, boxes[sidx]);
}

void launch_gather_keyed(hipStream_t s, int n, const ASys& sy, const int32_t* idx, const double* xyz, const double* q,
                         const ABox* boxes, double4* P, uint64_t* keys) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_keyed, dim3(cdiv(n, 256)), dim3(256), 0, s, n, sy, idx, xyz, q, boxes, P, keys);
}

// *flag |= 1 when some cell of level 10 holds more than leaf_max particles of
// one system (positions j and j + leaf_max share the 30-bit prefix), i.e. when
// the tree goes deeper than the 32-bit sort orders
// the top 32 key bits of the sorted composite keys (system << 32 | bits)
__global__ void k_low32(int n, const uint64_t* __restrict__ kc, uint32_t* __restrict__ k32s) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) k32s[j] = (uint32_t)kc[j];
}

void launch_low32(hipStream_t s, int n, const uint64_t* kc, uint32_t* k32s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_low32, dim3(cdiv(n, 256)), dim3(256), 0, s, n, kc, k32s);
}

__global__ void k_deep_check(int n, ASys sy, const uint32_t* __restrict__ k32s, int leaf_max, int* __restrict__ flag) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j + leaf_max >= n) return;
    if ((k32s[j] >> 2) != (k32s[j + leaf_max] >> 2)) return;
    if (sy.nsys > 1 && seg_of(sy.goff, sy.nsys, j) != seg_of(sy.goff, sy.nsys, j + leaf_max)) return;
    atomicOr(flag, 1);
}

void launch_deep_check(hipStream_t s, int n, const ASys& sy, const uint32_t* k32s, int leaf_max, int* flag) {
    hipLaunchKernelGGL(k_clear_i32, dim3(1), dim3(64), 0, s, 1, flag);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_deep_check, dim3(cdiv(n, 256)), dim3(256), 0, s, n, sy, k32s, leaf_max, flag);
}

// ------------------------------------------------------------------ tree

// one root per system: its forest positions, level 0, neighbour table = itself
__global__ void k_roots(ASys sy, ATree t) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= sy.nsys) return;
    t.key[r] = 0;
    t.pb[r] = sy.goff[r];
    t.pe[r] = sy.goff[r + 1];
    t.par[r] = -1;
    t.info[r] = 0;
    t.sys[r] = r;
    for (int d = 0; d < 27; ++d) t.nb[27 * (size_t)r + d] = d == 13 ? r : -1;
}

void launch_roots(hipStream_t s, const ASys& sy, const ATree& t) {
    hipLaunchKernelGGL(k_roots, dim3(cdiv(sy.nsys, 64)), dim3(64), 0, s, sy, t);
}

// For each node of one level: leaf flag, and for a split node the particle
// range of each octant.  One wavefront per node; lanes 8o..8o+7 find the
// first particle of the node whose octant exceeds o by an 8-ary search of
// the sorted keys (8 probes per step, so about log8 of the node's size
// dependent loads).  flag[8i+o] = 1 for every non-empty octant of a split
// node, cstart[8i+o] its first particle.
__global__ __launch_bounds__(64) void k_split(int level, int first, int count, int leaf_max,
                                              const uint64_t* __restrict__ keys, ATree t, int32_t* __restrict__ flag,
                                              int32_t* __restrict__ cstart) {
    const int i = blockIdx.x;
    if (i >= count) return;
    const int lane = threadIdx.x;
    const int g = first + i;
    const int b = t.pb[g], e = t.pe[g];
    const bool split = (e - b) > leaf_max && level < AMAX;
    if (lane == 0) t.info[g] = level | (split ? 0 : 1 << 8);
    if (lane < 8) t.child[8 * (size_t)g + lane] = -1;
    if (!split) {
        if (lane < 8) flag[8 * i + lane] = 0;
        return;
    }
    const int sh = 3 * (AMAX - level - 1);
    const uint64_t lim = t.key[g] * 8 + (uint64_t)(lane >> 3);  // octant prefix bound of this group
    const int o = lane >> 3, k = lane & 7;
    int lo = b, hi = e;  // the bound lies in [lo, hi]
    while (__any(lo < hi)) {
        const bool more = lo < hi;
        const int pk = lo + (int)(((long long)(hi - lo) * k) >> 3);
        const bool pred = more ? (keys[pk] >> sh) > lim : true;
        const unsigned bits = (unsigned)(__ballot(pred) >> (8 * o)) & 0xFFu;
        const int c = 8 - __popc(bits);  // probes at or below the bound's octant
        if (more) {
            const int nlo = c >= 1 ? lo + (int)(((long long)(hi - lo) * (c - 1)) >> 3) + 1 : lo;
            const int nhi = c < 8 ? lo + (int)(((long long)(hi - lo) * c) >> 3) : hi;
            lo = nlo;
            hi = nhi;
        }
    }
    const int prev = __shfl(lo, (lane + 56) & 63);  // the bound of octant o - 1
    if (k == 0) {
        const int s0 = o == 0 ? b : prev;
        flag[8 * i + o] = lo > s0 ? 1 : 0;
        cstart[8 * i + o] = s0;
    }
}

// children of the split nodes of a level, at next_first + (inclusive scan - 1)
__global__ void k_emit(int level, int first, int count, int next_first, const int32_t* __restrict__ flag,
                       const int32_t* __restrict__ incl, const int32_t* __restrict__ cstart, ATree t,
                       int* __restrict__ host, const int32_t* __restrict__ deep) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0 && host) {  // the next level's node count (and the depth check) for the host, in pinned memory
        host[0] = incl[8 * count - 1];
        if (deep) host[1] = *deep;
    }
    if (j >= 8 * count) return;
    if (!flag[j]) return;
    const int i = j >> 3, o = j & 7;
    const int g = first + i;
    const int c = next_first + incl[j] - 1;
    const int cb = cstart[j];
    // the octant's range ends where the next non-empty octant starts, or at the parent's end
    int ce = t.pe[g];
    for (int k = o + 1; k < 8; ++k)
        if (flag[8 * i + k]) {
            ce = cstart[8 * i + k];
            break;
        }
    t.key[c] = t.key[g] * 8 + (uint64_t)o;
    t.pb[c] = cb;
    t.pe[c] = ce;
    t.par[c] = g;
    t.info[c] = level + 1;
    t.sys[c] = t.sys[g];
    t.child[8 * (size_t)g + o] = c;
}

void launch_split(hipStream_t s, int level, int first, int count, int leaf_max, const uint64_t* keys, const ATree& t,
                  int32_t* flag, int32_t* cstart) {
    hipLaunchKernelGGL(k_split, dim3(count), dim3(64), 0, s, level, first, count, leaf_max, keys, t, flag, cstart);
}

void launch_emit(hipStream_t s, int level, int first, int count, int next_first, const int32_t* flag,
                 const int32_t* incl, const int32_t* cstart, const ATree& t, int* host, const int32_t* deep) {
    hipLaunchKernelGGL(k_emit, dim3(cdiv(8ll * count, 256)), dim3(256), 0, s, level, first, count, next_first, flag,
                       incl, cstart, t, host, deep);
}

// neighbour tables of one level (level >= 1) from the parents' tables
__global__ void k_nb(int first, int count, ATree t) {
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 27ll * count) return;
    const int g = first + (int)(gid / 27);
    const int d = (int)(gid % 27);
    const uint64_t key = t.key[g];
    const int P = t.par[g];
    int res = -1;
    int cidx = 0;
    int pd = 0;
#pragma unroll
    for (int k = 0, m = 1; k < 3; ++k, m *= 3) {
        const int o = (int)((key >> k) & 1);
        const int dd = (d / m) % 3 - 1;
        const int s = o + dd;  // -1..2: the cell's octant inside the parent-level cell at offset floor(s/2)
        pd += ((s >> 1) + 1) * m;
        cidx |= (s & 1) << k;
    }
    const int Q = t.nb[27 * (size_t)P + pd];
    if (Q >= 0) res = node_leaf(t.info[Q]) ? Q : t.child[8 * (size_t)Q + cidx];
    t.nb[27 * (size_t)g + d] = res;
}

void launch_nb(hipStream_t s, int first, int count, const ATree& t) {
    hipLaunchKernelGGL(k_nb, dim3(cdiv(27ll * count, 256)), dim3(256), 0, s, first, count, t);
}

// sorted particle position -> its leaf
__global__ void k_leaf_of(int nn, ATree t, int32_t* __restrict__ leaf_of) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nn || !node_leaf(t.info[g])) return;
    for (int s = t.pb[g]; s < t.pe[g]; ++s) leaf_of[s] = g;
}

void launch_leaf_of(hipStream_t s, int nn, const ATree& t, int32_t* leaf_of) {
    hipLaunchKernelGGL(k_leaf_of, dim3(cdiv(nn, 128)), dim3(128), 0, s, nn, t, leaf_of);
}

// (centre, side) of every node's cube, from its key, level and root cube
__global__ void k_node_geo(int nn, const ABox* __restrict__ boxes, ATree t) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nn) return;
    const NodeGeom G = node_geom(boxes[t.sys[g]], t.key[g], node_level(t.info[g]));
    t.geo[g] = make_double4(G.zx, G.zy, G.zz, G.h);
}

void launch_node_geo(hipStream_t s, int nn, const ABox* boxes, const ATree& t) {
    if (nn <= 0) return;
    hipLaunchKernelGGL(k_node_geo, dim3(cdiv(nn, 256)), dim3(256), 0, s, nn, boxes, t);
}

// ------------------------------------------------------------------ U, W, X lists

// One thread per node c, from the neighbour tables only:
//   U_d(c), c a leaf: the adjacent leaves of c's level or coarser (c itself
//           included), the distinct leaf entries of its table;
//   X(c):   the coarser leaves touching parent(c) but not c.
// The rest of the lists are transposes of these:
//   U(B) = U_d(B) + {finer leaves c : B in U_d(c)} (every finer adjacent
//          leaf lists B, the coarser leaf covering its neighbour cell);
//   W(B) = {c : B in X(c)} (c is below a same-level neighbour of B, not
//          adjacent to B while its parent is).
// FILL = false counts (the transposed entries with integer atomics), FILL =
// true writes: own entries in table order, transposed ones at atomically
// taken slots, put in ascending order afterwards (segmented sorts).
template <bool FILL>
__global__ void k_lists(int nn, ATree t, int32_t* __restrict__ ucnt, int32_t* __restrict__ wcnt,
                        int32_t* __restrict__ xcnt, int32_t* __restrict__ ufcnt, const int32_t* __restrict__ uoff,
                        const int32_t* __restrict__ woff, const int32_t* __restrict__ xoff,
                        int32_t* __restrict__ ulist, int32_t* __restrict__ wlist, int32_t* __restrict__ xlist,
                        int32_t* __restrict__ wfill, int32_t* __restrict__ ufill) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nn) return;
    const int info = t.info[c];
    const int lc = node_level(info);
    const uint64_t kc = t.key[c];
    int nu = 0, nx = 0;
    int nbv[27];  // a neighbour table in registers (the duplicate checks compare all pairs)
    if (node_leaf(info)) {
        const int32_t* nbc = t.nb + 27 * (size_t)c;
#pragma unroll
        for (int d = 0; d < 27; ++d) nbv[d] = nbc[d];
#pragma unroll
        for (int d = 0; d < 27; ++d) {
            const int C = nbv[d];
            bool dup = C < 0;
#pragma unroll
            for (int e = 0; e < d; ++e) dup |= nbv[e] == C;
            if (dup) continue;
            const int ci = t.info[C];
            if (!node_leaf(ci)) continue;
            if (FILL) ulist[uoff[c] + nu] = C;
            ++nu;
            if (node_level(ci) < lc) {  // c is a finer adjacent leaf of C
                if (!FILL) atomicAdd(&ufcnt[C], 1);
                else ulist[uoff[C] + ucnt[C] + atomicAdd(&ufill[C], 1)] = c;
            }
        }
    }
    if (lc >= 2) {
        const int32_t* nbP = t.nb + 27 * (size_t)t.par[c];
#pragma unroll
        for (int d = 0; d < 27; ++d) nbv[d] = nbP[d];
#pragma unroll
        for (int d = 0; d < 27; ++d) {
            const int C = nbv[d];
            bool dup = C < 0;
#pragma unroll
            for (int e = 0; e < d; ++e) dup |= nbv[e] == C;
            if (dup) continue;
            const int ci = t.info[C];
            if (!node_leaf(ci)) continue;
            if (adjacent(t.key[C], node_level(ci), kc, lc)) continue;
            if (FILL) xlist[xoff[c] + nx] = C;
            ++nx;
            if (!FILL) atomicAdd(&wcnt[C], 1);
            else wlist[woff[C] + atomicAdd(&wfill[C], 1)] = c;
        }
    }
    if (!FILL) {
        ucnt[c] = nu;
        xcnt[c] = nx;
    }
}

__global__ void k_add_i32(int n, const int32_t* __restrict__ a, const int32_t* __restrict__ b,
                          int32_t* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] + b[i];
}

// Each segment [beg[g], end[g]) of in, sorted ascending into the same range of
// out, one wavefront per segment: an entry's position is the number of entries
// of its segment that are smaller, or equal and earlier (segments are short
// lists of node indices; chunks of 64 entries are compared lane by lane).
__global__ __launch_bounds__(64) void k_rank_sort(const int32_t* __restrict__ beg, const int32_t* __restrict__ end,
                                                  const int32_t* __restrict__ in, int32_t* __restrict__ out) {
    const int g = blockIdx.x;
    const int b = beg[g], len = end[g] - b;
    if (len <= 0) return;
    const int lane = threadIdx.x;
    for (int i0 = 0; i0 < len; i0 += 64) {
        const int i = i0 + lane;
        const int v = i < len ? in[b + i] : 0;
        int rank = 0;
        for (int j0 = 0; j0 < len; j0 += 64) {
            const int w = j0 + lane < len ? in[b + j0 + lane] : 0;
            const int m = min(64, len - j0);
            for (int k = 0; k < m; ++k) {
                const int u = __builtin_amdgcn_readlane(w, k);
                rank += (u < v || (u == v && j0 + k < i)) ? 1 : 0;
            }
        }
        if (i < len) out[b + rank] = v;
    }
}

void launch_rank_sort(hipStream_t s, int nseg, const int32_t* beg, const int32_t* end, const int32_t* in,
                      int32_t* out) {
    if (nseg <= 0) return;
    hipLaunchKernelGGL(k_rank_sort, dim3(nseg), dim3(64), 0, s, beg, end, in, out);
}

void launch_lists(hipStream_t s, bool fill, int nn, const ATree& t, int32_t* ucnt, int32_t* wcnt, int32_t* xcnt,
                  int32_t* ufcnt, const int32_t* uoff, const int32_t* woff, const int32_t* xoff, int32_t* ulist,
                  int32_t* wlist, int32_t* xlist, int32_t* wfill, int32_t* ufill) {
    if (nn <= 0) return;
    if (fill)
        hipLaunchKernelGGL(k_lists<true>, dim3(cdiv(nn, 128)), dim3(128), 0, s, nn, t, ucnt, wcnt, xcnt, ufcnt, uoff,
                           woff, xoff, ulist, wlist, xlist, wfill, ufill);
    else
        hipLaunchKernelGGL(k_lists<false>, dim3(cdiv(nn, 128)), dim3(128), 0, s, nn, t, ucnt, wcnt, xcnt, ufcnt, uoff,
                           woff, xoff, ulist, wlist, xlist, wfill, ufill);
}

void launch_add_i32(hipStream_t s, int n, const int32_t* a, const int32_t* b, int32_t* out) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_add_i32, dim3(cdiv(n, 256)), dim3(256), 0, s, n, a, b, out);
}

// ------------------------------------------------------------------ M2L tiles

// sort key of a node: level and octant (targets of one tile share the octant)
__global__ void k_lvloct(int nn, ATree t, uint32_t* __restrict__ k, int32_t* __restrict__ v) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nn) return;
    k[g] = ((uint32_t)node_level(t.info[g]) << 3) | (uint32_t)(t.key[g] & 7);
    v[g] = g;
}


// bucket [bstart, bend) of every (level, octant) key in the sorted order
__global__ void k_buckets(int nn, const uint32_t* __restrict__ sk, int32_t* __restrict__ bstart,
                          int32_t* __restrict__ bend) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    const uint32_t k = sk[i];
    if (i == 0 || sk[i - 1] != k) bstart[k] = i;
    if (i == nn - 1 || sk[i + 1] != k) bend[k] = i + 1;
}

void launch_lvloct(hipStream_t s, int nn, const ATree& t, uint32_t* k, int32_t* v) {
    hipLaunchKernelGGL(k_lvloct, dim3(cdiv(nn, 256)), dim3(256), 0, s, nn, t, k, v);
}

void launch_buckets(hipStream_t s, int nn, const uint32_t* sk, int32_t* bstart, int32_t* bend) {
    hipLaunchKernelGGL(k_clear_i32, dim3(1), dim3(256), 0, s, 256, bstart);
    hipLaunchKernelGGL(k_clear_i32, dim3(1), dim3(256), 0, s, 256, bend);
    hipLaunchKernelGGL(k_buckets, dim3(cdiv(nn, 256)), dim3(256), 0, s, nn, sk, bstart, bend);
}

// One wavefront per tile: the targets of the tile (tt of them, 64 slots per
// pass) and, for each offset, the source cell of each target (child q of the
// parent's neighbour u, or -1); vcount = sources that exist per (tile,
// offset).  An offset of octant o is one (u, q) pair (qu_list[o][iv] =
// u | q << 5); the wavefront walks the 27 neighbours u of each target's parent
// once, reads their 8 children, and files child q under the offset of (u, q)
// (inverse table in LDS), so the loads per target are independent and few.
__global__ __launch_bounds__(64) void k_m2l_tables(int tt, const int4* __restrict__ tiles,
                                                   const int32_t* __restrict__ sorted, ATree t,
                                                   const int16_t* __restrict__ qu_list, int32_t* __restrict__ tgt_tab,
                                                   int32_t* __restrict__ src_tab, int32_t* __restrict__ vcount) {
    const int tile = blockIdx.x;
    const int lane = threadIdx.x;
    const int4 d = tiles[tile];  // (octant, first sorted position, count, level)
    __shared__ int16_t inv[256];
    __shared__ int cnt[189];
    for (int x = lane; x < 256; x += 64) inv[x] = -1;
    for (int x = lane; x < 189; x += 64) cnt[x] = 0;
    __syncthreads();
    for (int x = lane; x < 189; x += 64) inv[qu_list[d.x * 189 + x]] = (int16_t)x;
    __syncthreads();
    for (int r0 = 0; r0 < tt; r0 += 64) {
        const int r = r0 + lane;
        const int tg = r < d.z ? sorted[d.y + r] : -1;
        if (r < tt) tgt_tab[tt * (size_t)tile + r] = tg;
        const int par = tg >= 0 ? t.par[tg] : -1;
        for (int u = 0; u < 27; ++u) {
            const int Q = par >= 0 ? t.nb[27 * (size_t)par + u] : -1;
            const bool inner = Q >= 0 && !node_leaf(t.info[Q]);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int iv = inv[u | (q << 5)];  // the same in every lane
                if (iv < 0) continue;
                const int src = inner ? t.child[8 * (size_t)Q + q] : -1;
                if (r < tt) src_tab[(189 * (size_t)tile + iv) * tt + r] = src;
                const int c = __popcll(__ballot(src >= 0));
                if (lane == 0) cnt[iv] += c;
            }
        }
    }
    __syncthreads();
    for (int x = lane; x < 189; x += 64) vcount[189 * (size_t)tile + x] = cnt[x];
}

// Sort key of an M2L tile: the parent of its first target, then the octant.
// Nodes are numbered level by level in the order of the sorted keys, so the
// tiles of the 8 octants over the same parents come out next to each other:
// they read nearly the same source rows.
__global__ void k_tile_keys(int ntiles, const int4* __restrict__ tiles, const int32_t* __restrict__ sorted, ATree t,
                            uint64_t* __restrict__ key, int32_t* __restrict__ idx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntiles) return;
    const int4 d = tiles[i];  // (octant, first sorted position, count, level)
    key[i] = ((uint64_t)t.par[sorted[d.y]] << 3) | (uint64_t)d.x;
    idx[i] = i;
}

__global__ void k_gather_int4(int n, const int32_t* __restrict__ idx, const int4* __restrict__ in,
                              int4* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[idx[i]];
}

void launch_tile_keys(hipStream_t s, int ntiles, const int4* tiles, const int32_t* sorted, const ATree& t,
                      uint64_t* key, int32_t* idx) {
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(k_tile_keys, dim3(cdiv(ntiles, 256)), dim3(256), 0, s, ntiles, tiles, sorted, t, key, idx);
}

void launch_gather_int4(hipStream_t s, int n, const int32_t* idx, const int4* in, int4* out) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_int4, dim3(cdiv(n, 256)), dim3(256), 0, s, n, idx, in, out);
}

void launch_m2l_tables(hipStream_t s, int tt, int ntiles, const int4* tiles, const int32_t* sorted, const ATree& t,
                       const int16_t* qu_list, int32_t* tgt_tab, int32_t* src_tab, int32_t* vcount) {
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(k_m2l_tables, dim3(ntiles), dim3(64), 0, s, tt, tiles, sorted, t, qu_list, tgt_tab, src_tab,
                       vcount);
}

// ------------------------------------------------------------------ P2M, M2M, L2L on node lists

// P2M of every leaf among nodes [first, first+count): one wavefront per node
template <int PP>
__global__ __launch_bounds__(64) void k_p2m_nodes(int first, const ABox* __restrict__ boxes, ATree t,
                                                  const double4* __restrict__ P, DevTables T, double* __restrict__ M) {
    const int g = first + blockIdx.x;
    const int info = t.info[g];
    if (!node_leaf(info)) return;
    const NodeGeom G = node_geom(boxes, t, g);
    p2m_cell<PP>(G.zx, G.zy, G.zz, G.h, t.pb[g], t.pe[g], P, T, M + (size_t)g * ldm_of(PP));
}

void launch_p2m_nodes(hipStream_t s, int p, int first, int count, const ABox* boxes, const ATree& t, const double4* P,
                      const DevTables& T, double* M) {
    if (count <= 0) return;
    switch (p) {
#define CASE(PP) case PP: hipLaunchKernelGGL(k_p2m_nodes<PP>, dim3(count), dim3(64), 0, s, first, boxes, t, P, T, M); break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

constexpr int ANP = 4;  // parents per workgroup in M2M/L2L

__host__ __device__ constexpr int m2m_block(int p) { return (8 * (p + 1) * (p + 1) + 63) & ~63; }

__device__ inline int rank_of_a(int k) {
    int r = 0;
    while ((r + 1) * (r + 1) <= k) ++r;
    return r;
}

// M~(parent) = sum over existing children of A_o M~(child), for the non-leaf
// nodes among [first, first+count) (the leaves keep their P2M result).  One
// thread per (octant o, component n) and ANP parents per workgroup: the
// children rows sit in LDS, each operator coefficient A_o[n][j] (rank(j) <=
// rank(n)) is read once per workgroup and used for every parent, and the 8
// octant sums meet in LDS, added in octant order.
template <int P>
__global__ __launch_bounds__(1024) void k_m2m_nodes(int first, int count, ATree t, double* __restrict__ M,
                                                    const double* __restrict__ m2m_t) {
    constexpr int NC = (P + 1) * (P + 1);
    const int P0 = first + blockIdx.x * ANP;
    const int np = min(ANP, first + count - P0);
    const int ldm = ldm_of(P);
    __shared__ double ch[ANP][8][NC];
    __shared__ double red[ANP][8][NC];
    __shared__ int live;
    if (threadIdx.x == 0) {
        int any = 0;
        for (int pp = 0; pp < np; ++pp) any |= !node_leaf(t.info[P0 + pp]);
        live = any;
    }
    __syncthreads();
    if (!live) return;
    for (int x = threadIdx.x; x < ANP * 8 * NC; x += blockDim.x) {
        const int pp = x / (8 * NC), r = x % (8 * NC), o = r / NC, j = r % NC;
        const int c = pp < np ? t.child[8 * (size_t)(P0 + pp) + o] : -1;
        ch[pp][o][j] = c >= 0 ? M[(size_t)c * ldm + j] : 0.0;
    }
    __syncthreads();
    const int o = threadIdx.x / NC, n = threadIdx.x % NC;
    if (o < 8) {
        const int r = rank_of_a(n);
        const int jmax = (r + 1) * (r + 1);
        const double* A = m2m_t + (size_t)o * NIND * NIND + n;
        double acc[ANP];
#pragma unroll
        for (int pp = 0; pp < ANP; ++pp) acc[pp] = 0.0;
#pragma unroll 4
        for (int j = 0; j < jmax; ++j) {
            const double a = A[(size_t)j * NIND];
#pragma unroll
            for (int pp = 0; pp < ANP; ++pp) acc[pp] += a * ch[pp][o][j];
        }
#pragma unroll
        for (int pp = 0; pp < ANP; ++pp) red[pp][o][n] = acc[pp];
    }
    __syncthreads();
    // whole rows: the padding after the (P+1)^2 components is kept zero (M2L
    // stages complete rows)
    for (int x = threadIdx.x; x < np * ldm; x += blockDim.x) {
        const int pp = x / ldm, k = x % ldm;
        if (node_leaf(t.info[P0 + pp])) continue;
        double v = 0.0;
        if (k < NC)
#pragma unroll
            for (int q = 0; q < 8; ++q) v += red[pp][q][k];
        M[(size_t)(P0 + pp) * ldm + k] = v;
    }
}

void launch_m2m_nodes(hipStream_t s, int p, int first, int count, const ATree& t, double* M, const DevTables& T) {
    if (count <= 0) return;
    switch (p) {
#define CASE(PP)                                                                                                  \
    case PP:                                                                                                      \
        hipLaunchKernelGGL(k_m2m_nodes<PP>, dim3(cdiv(count, ANP)), dim3(m2m_block(PP)), 0, s, first, count, t, M,  \
                           T.m2m_t);                                                                              \
        break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

// L~(child) += B_o L~(parent) for the existing children of the non-leaf nodes
// among [first, first+count).  One thread per (octant o, component n) and ANP
// parents per workgroup; each coefficient B_o[n][j] (rank(j) >= rank(n)) is
// read once per workgroup.
template <int P>
__global__ __launch_bounds__(1024) void k_l2l_nodes(int first, int count, ATree t, double* __restrict__ L,
                                                    const double* __restrict__ l2l_t) {
    constexpr int NC = (P + 1) * (P + 1);
    const int P0 = first + blockIdx.x * ANP;
    const int np = min(ANP, first + count - P0);
    const int ldm = ldm_of(P);
    __shared__ double lp[ANP][NC];
    __shared__ int cid[ANP][8];
    if ((int)threadIdx.x < ANP * 8) {
        const int pp = threadIdx.x / 8, o = threadIdx.x % 8;
        cid[pp][o] = pp < np ? t.child[8 * (size_t)(P0 + pp) + o] : -1;
    }
    for (int x = threadIdx.x; x < ANP * NC; x += blockDim.x)
        lp[x / NC][x % NC] = x / NC < np ? L[(size_t)(P0 + x / NC) * ldm + x % NC] : 0.0;
    __syncthreads();
    const int o = threadIdx.x / NC, n = threadIdx.x % NC;
    if (o >= 8) return;
    bool any = false;
#pragma unroll
    for (int pp = 0; pp < ANP; ++pp) any |= cid[pp][o] >= 0;
    if (!any) return;
    const int r = rank_of_a(n);
    const double* Bm = l2l_t + (size_t)o * NIND * NIND + n;
    double acc[ANP];
#pragma unroll
    for (int pp = 0; pp < ANP; ++pp) acc[pp] = 0.0;
#pragma unroll 4
    for (int j = r * r; j < NC; ++j) {
        const double bcoef = Bm[(size_t)j * NIND];
#pragma unroll
        for (int pp = 0; pp < ANP; ++pp) acc[pp] += bcoef * lp[pp][j];
    }
#pragma unroll
    for (int pp = 0; pp < ANP; ++pp) {
        const int c = cid[pp][o];
        if (c >= 0) L[(size_t)c * ldm + n] += acc[pp];
    }
}

void launch_l2l_nodes(hipStream_t s, int p, int first, int count, const ATree& t, double* L, const DevTables& T) {
    if (count <= 0) return;
    switch (p) {
#define CASE(PP)                                                                                                  \
    case PP:                                                                                                      \
        hipLaunchKernelGGL(k_l2l_nodes<PP>, dim3(cdiv(count, ANP)), dim3(m2m_block(PP)), 0, s, first, count, t, L,  \
                           T.l2l_t);                                                                              \
        break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

// ------------------------------------------------------------------ X list: direct local expansions

// L~_n(B) += q D~_n(u), u = (z_B - x_a)/h_B, for the particles a of every
// leaf in X(B) (Eq. M2L with the multipole of a single charge at its own
// position, in the scaled variables).  With D_n(u) = (-1)^n (2n-1)!! D[u^n]
// |u|^-(2n+1) (D the traceless projection) and w = u/|u|^2 this is
//   L~_n(B) += (-1)^n (2n-1)!! D[S]_n,   S_f = sum_a (q_a/|u_a|) w_a^f,
// i.e. the detracer rows of P2M applied to the full monomial moments S of
// the inverted points.  One wavefront per node B: lanes over the particles
// of X(B) (P2L_KP per lane per round), the moments in blocks of at most MB
// monomials (compile-time blocks of whole (a, b) rows, hidx order) summed
// over the lanes through LDS; then the detracer rows, once per node.
constexpr int MB = 24;
struct MRow {
    int a, b, start, len;  // w^(a, b, c) for c = 0..len-1 at positions start..
};
__host__ __device__ constexpr int mrows(int P) { return (P + 1) * (P + 2) / 2; }
__host__ __device__ constexpr MRow mrow(int P, int r) {
    int start = 0;
    for (int a = 0; a <= P; ++a)
        for (int b = 0; b <= P - a; ++b) {
            const int len = P - a - b + 1;
            if (r == 0) return MRow{a, b, start, len};
            --r;
            start += len;
        }
    return MRow{0, 0, start, 0};
}
struct MBlock {
    int r0, r1, start, len;
};
__host__ __device__ constexpr int mblocks(int P) {
    int g = 0, len = 0;
    for (int r = 0; r < mrows(P); ++r) {
        const int l = mrow(P, r).len;
        if (r == 0 || len + l > MB) {
            ++g;
            len = 0;
        }
        len += l;
    }
    return g;
}
__host__ __device__ constexpr MBlock mblock(int P, int g) {
    int k = -1, len = 0, r0 = 0;
    for (int r = 0; r < mrows(P); ++r) {
        const int l = mrow(P, r).len;
        if (r == 0 || len + l > MB) {
            if (k == g) return MBlock{r0, r, mrow(P, r0).start, len};
            ++k;
            len = 0;
            r0 = r;
        }
        len += l;
    }
    return MBlock{r0, mrows(P), mrow(P, r0).start, len};
}

// acc[start - m0 + c] += q x^a y^b z^c over the rows [r, r1)
template <int P, int r, int r1>
__device__ __forceinline__ void mrows_acc(double q, const double (&xp)[P + 1], const double (&yp)[P + 1], double z,
                                          int m0, double (&acc)[MB]) {
    constexpr MRow R = mrow(P, r);
    double m = q * xp[R.a] * yp[R.b];
#pragma unroll
    for (int c = 0; c < R.len; ++c) {
        acc[R.start - m0 + c] += m;
        if (c + 1 < R.len) m *= z;
    }
    if constexpr (r + 1 < r1) mrows_acc<P, r + 1, r1>(q, xp, yp, z, m0, acc);
}

// Moment block g over the first kp of the KP particles each lane holds
// (q = 0 for an empty slot; slots past kp are empty in every lane), summed
// over the lanes through red and added into S (LDS, full-slot order); then
// the next block.
template <int P, int g, int KP>
__device__ __forceinline__ void p2l_blocks(const double (&wx)[KP], const double (&wy)[KP], const double (&wz)[KP],
                                           const double (&qq)[KP], int kp, double* S, double (*red)[65], double tok) {
    constexpr MBlock K = mblock(P, g);
    const int lane = threadIdx.x;
    double acc[MB];
#pragma unroll
    for (int j = 0; j < MB; ++j) acc[j] = 0.0;
#pragma unroll
    for (int j = 0; j < KP; ++j) {
        if (j >= kp) break;  // wave-uniform
        // particle j's powers only after particle j-1 is accumulated (one set
        // of power tables live at a time), the first after the previous block
        double x1 = wx[j], y1 = wy[j];
        __asm__ volatile("" : "+v"(x1), "+v"(y1) : "v"(j == 0 ? tok : acc[K.len - 1]));
        double xp[P + 1], yp[P + 1];
        xp[0] = yp[0] = 1.0;
#pragma unroll
        for (int k = 1; k <= P; ++k) {
            xp[k] = xp[k - 1] * x1;
            yp[k] = yp[k - 1] * y1;
        }
        mrows_acc<P, K.r0, K.r1>(qq[j], xp, yp, wz[j], K.start, acc);
    }
#pragma unroll
    for (int j = 0; j < K.len; ++j) red[j][lane] = acc[j];
    __syncthreads();
    if (lane < K.len) {
        double v = 0.0;
#pragma unroll 8
        for (int k = 0; k < 64; ++k) v += red[lane][k];
        // (a, b, c) of position K.start + lane, then its full slot
        int a = 0, bb = 0, r = K.start + lane;
        while (r >= (P - a + 1) * (P - a + 2) / 2) r -= (P - a + 1) * (P - a + 2) / 2, ++a;
        while (r >= P - a - bb + 1) r -= P - a - bb + 1, ++bb;
        const int n = a + bb + r;
        S[n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + (n - a - bb)] += v;
    }
    __syncthreads();
    if constexpr (g + 1 < mblocks(P)) p2l_blocks<P, g + 1, KP>(wx, wy, wz, qq, kp, S, red, acc[K.len - 1]);
}

// The particles of X(B) are numbered in list order, 64 entries at a time
// (their first particles and the prefix sums of their sizes staged in LDS);
// each round, lane l holds numbers base + l + 64 j (j < KP) in registers for
// every moment block.
constexpr int P2L_KP = 5;
template <int P>
__global__ __launch_bounds__(64) void k_p2l(const ABox* __restrict__ boxes, ATree t, const int32_t* __restrict__ xoff,
                                            const int32_t* __restrict__ xlist, const double4* __restrict__ Pt,
                                            DevTables T, double* __restrict__ L) {
    constexpr int NC = (P + 1) * (P + 1);
    constexpr int NF = (P + 1) * (P + 2) * (P + 3) / 6;
    constexpr int KP = P2L_KP;
    const int B = blockIdx.x;
    const int x0 = xoff[B], x1 = xoff[B + 1];
    if (x0 == x1) return;
    const int lane = threadIdx.x;
    __shared__ double S[NF];
    __shared__ double red[MB][65];
    __shared__ int epb[64], epre[65];
    for (int k = lane; k < NF; k += 64) S[k] = 0.0;
    const NodeGeom G = node_geom(boxes, t, B);
    for (int e0 = x0; e0 < x1; e0 += 64) {
        const int ne = min(64, x1 - e0);
        int sz = 0;
        if (lane < ne) {
            const int C = xlist[e0 + lane];
            epb[lane] = t.pb[C];
            sz = t.pe[C] - t.pb[C];
        }
        int incl = sz;  // inclusive scan over the lanes
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int o = __shfl_up(incl, d);
            if (lane >= d) incl += o;
        }
        epre[lane + 1] = incl;
        if (lane == 0) epre[0] = 0;
        __syncthreads();
        const int tot = epre[ne];
        for (int base = 0; base < tot; base += 64 * KP) {
            double wx[KP], wy[KP], wz[KP], qq[KP];
#pragma unroll
            for (int j = 0; j < KP; ++j) {
                const int gi = base + lane + 64 * j;
                wx[j] = wy[j] = wz[j] = qq[j] = 0.0;
                if (gi < tot) {
                    int lo = 0, hi = ne;  // entry e with epre[e] <= gi < epre[e + 1]
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (epre[mid] <= gi) lo = mid; else hi = mid;
                    }
                    const double4 pt = Pt[epb[lo] + gi - epre[lo]];
                    const double ux = (G.zx - pt.x) / G.h, uy = (G.zy - pt.y) / G.h, uz = (G.zz - pt.z) / G.h;
                    const double ir2 = 1.0 / (ux * ux + uy * uy + uz * uz);
                    qq[j] = pt.w * sqrt(ir2);
                    wx[j] = ux * ir2;
                    wy[j] = uy * ir2;
                    wz[j] = uz * ir2;
                }
            }
            p2l_blocks<P, 0, KP>(wx, wy, wz, qq, min(KP, (tot - base + 63) / 64), S, red, 0.0);
        }
        __syncthreads();  // the entry table is read before it is restaged
    }
    double* Lb = L + (size_t)B * ldm_of(P);
    for (int n = lane; n < NC; n += 64) {
        double v = 0.0;
        for (int k = T.det_start[n]; k < T.det_start[n + 1]; ++k) v += T.det_coef[k] * S[T.det_full[k]];
        int r = 0;
        while ((r + 1) * (r + 1) <= n) ++r;
        double w = 1.0;  // (-1)^r (2r-1)!!
        for (int i = 1; i <= r; ++i) w *= -(double)(2 * i - 1);
        Lb[n] += w * v;
    }
}

// ------------------------------------------------------------------ W list and near field

// Coefficients of the multipole-at-a-particle polynomial (W list).  Against
// a traceless M only the r^n part of D_n survives:
//   sum_{|m|=n} M_m D_m(r)/m! = (-1)^n (2n-1)!! |r|^(-2n-1) sum_{|m|=n} M_m r^m/m!
// so the potential of cell C at scaled offset u is |u|^-1 Q(w), w = u/|u|^2,
// with the polynomial Q(w) = sum_{|m|<=p} c_m w^m and
//   c_m = (-1)^|m| (2|m|-1)!! M~_m / m!
// over every full component m (the dependent ones expanded from the
// independent ones by the trace relation).  Row layout (rows of ldc_of(p)
// doubles), the order in which m2p_horner consumes the coefficients: first
// the ranks < p with a, b and c descending, then the rank-p ones with a and
// b descending (hpos).
__host__ __device__ constexpr int nfull_of(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
__host__ __device__ constexpr int ldc_of(int p) { return (nfull_of(p) + 7) & ~7; }
// position of (a, b, c) in a row (a + b + c <= p)
__host__ __device__ constexpr int hidx(int p, int a, int b, int c) {
    int r = c;
    for (int i = 0; i < a; ++i) r += (p - i + 1) * (p - i + 2) / 2;  // rows a' < a
    for (int j = 0; j < b; ++j) r += p - a - j + 1;                  // rows b' < b within a
    return r;
}
// position of c_(a,b,c) in a coefficient row of order p
__host__ __device__ constexpr int hpos(int p, int a, int b, int c) {
    return a + b + c < p ? nfull_of(p - 1) - 1 - hidx(p - 1, a, b, c)
                         : nfull_of(p - 1) + (p - a) * (p - a + 1) / 2 + (p - a - b);
}

// The terms of every coefficient of order P, in row order k: c_k = sum_t
// coef[t] * M~[slot[t]] over t in [start[k], start[k+1]), with the factor
// (-1)^n (2n-1)!! / m! folded into coef and the dependent components of M~
// expanded into independent ones by the trace relation
// (A_{a,b,2s+t} = (-1)^s sum_i C(s,i) A_{a+2i, b+2(s-i), t}).
template <int P>
struct M2PCoefRows {
    static constexpr int NF = nfull_of(P), NT = NF * (P / 2 + 1);
    int start[NF + 1];
    int slot[NT];
    double coef[NT];
    static constexpr int ind_slot(int a, int b, int t) {
        const int n = a + b + t;
        return t == 0 ? n * n + (n - a) : n * n + (n + 1) + (n - 1 - a);
    }
    static constexpr double binom(int n, int k) {
        double r = 1.0;
        for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
        return r;
    }
    static constexpr M2PCoefRows make() {
        M2PCoefRows tb{};
        int at[NF] = {}, bt[NF] = {}, ct[NF] = {};
        for (int n = 0; n <= P; ++n)
            for (int a = 0; a <= n; ++a)
                for (int b = 0; b <= n - a; ++b) {
                    const int k = hpos(P, a, b, n - a - b);
                    at[k] = a;
                    bt[k] = b;
                    ct[k] = n - a - b;
                }
        int t = 0;
        for (int k = 0; k < NF; ++k) {
            tb.start[k] = t;
            const int a = at[k], b = bt[k], c = ct[k], n = a + b + c;
            double w = 1.0;  // (-1)^n (2n-1)!! / (a! b! c!)
            for (int i = 1; i <= n; ++i) w *= -(double)(2 * i - 1);
            for (int i = 2; i <= a; ++i) w /= i;
            for (int i = 2; i <= b; ++i) w /= i;
            for (int i = 2; i <= c; ++i) w /= i;
            const int sh = c / 2, tz = c % 2;
            for (int i = 0; i <= sh; ++i) {
                tb.slot[t] = ind_slot(a + 2 * i, b + 2 * (sh - i), tz);
                tb.coef[t] = w * (sh % 2 ? -1.0 : 1.0) * binom(sh, i);
                ++t;
            }
        }
        tb.start[NF] = t;
        return tb;
    }
};
template <int P>
struct M2PCoefTab {
    static constexpr int NF = M2PCoefRows<P>::NF;
    static constexpr M2PCoefRows<P> tab = M2PCoefRows<P>::make();
};

template <int P>
__global__ void k_m2p_coef(int first, int count, const double* __restrict__ M, double* __restrict__ Cm) {
    using TB = M2PCoefTab<P>;
    constexpr int ldc = ldc_of(P);
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (long long)count * ldc) return;
    const int k = (int)(gid % ldc);
    const size_t row = (size_t)first + gid / ldc;
    double v = 0.0;
    if (k < TB::NF) {
        const double* Mr = M + row * ldm_of(P);
        for (int t = TB::tab.start[k]; t < TB::tab.start[k + 1]; ++t) v += TB::tab.coef[t] * Mr[TB::tab.slot[t]];
    }
    Cm[row * ldc + k] = v;
}

void launch_m2p_coef(hipStream_t s, int p, int first, int count, const double* M, const DevTables& T, double* Cm) {
    (void)T;
    if (count <= 0) return;
    switch (p) {
#define CASE(PP)                                                                                                  \
    case PP:                                                                                                      \
        hipLaunchKernelGGL(k_m2p_coef<PP>, dim3(cdiv((long long)count * ldc_of(PP), 256)), dim3(256), 0, s, first, \
                           count, M, Cm);                                                                         \
        break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

size_t m2p_coef_ld(int p) { return (size_t)ldc_of(p); }



// Far field of one sorted particle s (one thread each) from the local
// expansion of its leaf B (Eq. L2P, nested Horner over the full polynomial
// coefficients, each formed from the leaf's independent ones as it is
// needed; zero for leaves above level 2), plus its
// near field Fn[s]: the total goes to phi and grad in input order, or with
// to_F back into F[s].
template <int P>
__global__ __launch_bounds__(256) void k_l2p_adaptive(int n, const ABox* __restrict__ boxes, ATree t, const int32_t* __restrict__ leaf_of,
                                                      const double4* __restrict__ Pt, const double* __restrict__ L,
                                                      double4* __restrict__ F, const double4* __restrict__ Fn,
                                                      const int32_t* __restrict__ idx, bool to_F,
                                                      double* __restrict__ phi, double* __restrict__ grad) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int B = leaf_of[s];
    const int lb = node_level(t.info[B]);
    double4 out = make_double4(0.0, 0.0, 0.0, 0.0);
    if (lb >= 2) {
        const double4 pt = Pt[s];
        const NodeGeom G = node_geom(boxes, t, B);
        double lf = 0.0, lx = 0.0, ly = 0.0, lz = 0.0;
        gen_l2p_hg<P>((pt.x - G.zx) / G.h, (pt.y - G.zy) / G.h, (pt.z - G.zz) / G.h, L + (size_t)B * ldm_of(P), lf,
                      lx, ly, lz);
        const double ih2 = 1.0 / (G.h * G.h);
        out = make_double4(lf / G.h, lx * ih2, ly * ih2, lz * ih2);
    }
    const double4 b = Fn[s];
    const double4 v = make_double4(out.x + b.x, out.y + b.y, out.z + b.z, out.w + b.w);
    if (to_F) {
        F[s] = v;
        return;
    }
    const size_t o = (size_t)idx[s];
    if (phi) phi[o] = v.x;
    if (grad) {
        grad[3 * o] = v.y;
        grad[3 * o + 1] = v.z;
        grad[3 * o + 2] = v.w;
    }
}

// A wave-uniform zero that depends on dep0, dep1 and dep2: loads at
// c + after(...) cannot be issued before those are computed, and keep c's
// address space and aliasing facts (scalar loads).  Without it every load of the
// unrolled polynomial is hoisted to the top and the rows' values stay live.
__device__ __forceinline__ int after(double dep0, double dep1, double dep2) {
    int z = 0;
    __asm__ volatile("" : "+s"(z) : "v"(dep0), "v"(dep1), "v"(dep2));
    return z;
}

// The rows of a coefficient row, in memory order: first the Horner rows of
// fl, (a, b) for a = P-1..0, b = P-1-a..0, holding c = P-1-a-b..0; then the
// rows of ft, a = P..0, holding b = P-a..0 (c = P-a-b).
struct HRow {
    int kind, a, b, start, len;  // kind 0: fl row, 1: ft row
};
__host__ __device__ constexpr int hrows(int P) { return P * (P + 1) / 2 + P + 1; }
__host__ __device__ constexpr HRow hrow(int P, int r) {
    int start = 0;
    for (int a = P - 1; a >= 0; --a)
        for (int b = P - 1 - a; b >= 0; --b) {
            const int len = P - a - b;
            if (r == 0) return HRow{0, a, b, start, len};
            --r;
            start += len;
        }
    for (int a = P; a >= 0; --a) {
        const int len = P - a + 1;
        if (r == 0) return HRow{1, a, 0, start, len};
        --r;
        start += len;
    }
    return HRow{2, 0, 0, start, 0};
}

struct HState {
    double V, Vx, Vy, Vz, T, U, Uy, Uz;
};

// Rows are fetched in groups of consecutive rows holding at most HG
// coefficients (a group is a contiguous range of the coefficient row).
constexpr int HG = 16;
struct HGroup {
    int r0, r1, start, len;  // rows [r0, r1)
};
__host__ __device__ constexpr int hgroups(int P) {
    int g = 0, len = 0;
    for (int r = 0; r < hrows(P); ++r) {
        const int l = hrow(P, r).len;
        if (r == 0 || len + l > HG) {
            ++g;
            len = 0;
        }
        len += l;
    }
    return g;
}
__host__ __device__ constexpr HGroup hgroup(int P, int g) {
    int k = -1, len = 0, r0 = 0;
    for (int r = 0; r < hrows(P); ++r) {
        const int l = hrow(P, r).len;
        if (r == 0 || len + l > HG) {
            if (k == g) return HGroup{r0, r, hrow(P, r0).start, len};
            ++k;
            len = 0;
            r0 = r;
        }
        len += l;
    }
    return HGroup{r0, hrows(P), hrow(P, r0).start, len};
}

// Evaluates row r (held in w, a group buffer starting at coefficient w0),
// then the rows after it up to r1.
template <int P, int r, int r1>
__device__ __forceinline__ void hrows_run(double x, double y, double z, const double (&zp)[P + 1], int w0,
                                          const double (&w)[HG], HState& s) {
    constexpr int D = P - 1;
    constexpr HRow R = hrow(P, r);
    const int o = R.start - w0;
    if constexpr (R.kind == 0) {
        constexpr int a = R.a, b = R.b;
        double v = w[o], d = 0.0;
#pragma unroll
        for (int j = 1; j < R.len; ++j) {
            d = (j == 1) ? v : d * z + v;
            v = v * z + w[o + j];
        }
        if constexpr (b == D - a) {  // first row of the group: no derivatives yet
            s.U = v;
            s.Uy = 0.0;
            s.Uz = 0.0;
        } else if constexpr (b == D - a - 1) {
            s.Uy = s.U;
            s.U = s.U * y + v;
            s.Uz = d;
        } else {
            s.Uy = s.Uy * y + s.U;
            s.U = s.U * y + v;
            s.Uz = s.Uz * y + d;
        }
        if constexpr (b == 0) {  // last row of the group: fold into the x level
            if constexpr (a == D) {
                s.V = s.U;
            } else if constexpr (a == D - 1) {
                s.Vx = s.V;
                s.V = s.V * x + s.U;
                s.Vy = s.Uy;
                s.Vz = s.Uz;
            } else {
                s.Vx = s.Vx * x + s.V;
                s.V = s.V * x + s.U;
                s.Vy = s.Vy * x + s.Uy;
                s.Vz = s.Vz * x + s.Uz;
            }
        }
    } else {
        double S = w[o];
#pragma unroll
        for (int j = 1; j < R.len; ++j) S = S * y + w[o + j] * zp[j];
        s.T = (R.a == P) ? S : s.T * x + S;
    }
    if constexpr (r + 1 < r1) hrows_run<P, r + 1, r1>(x, y, z, zp, w0, w, s);
}

// Group g (held in cur): the loads of group g+1 are issued first (they wait
// only for the result of group g-1), then the rows of group g are evaluated;
// group g+1 follows with the buffers swapped.
template <int P, int g>
__device__ __forceinline__ void hgroups_run(double x, double y, double z, const double (&zp)[P + 1],
                                            const double* __restrict__ c, HState& s, double (&cur)[HG],
                                            double (&nxt)[HG]) {
    constexpr HGroup G = hgroup(P, g);
    if constexpr (g + 1 < hgroups(P)) {
        constexpr HGroup Gn = hgroup(P, g + 1);
        const double* cn = c + after(s.U, s.T, s.V);
#pragma unroll
        for (int k = 0; k < Gn.len; ++k) nxt[k] = cn[Gn.start + k];
    }
    hrows_run<P, G.r0, G.r1>(x, y, z, zp, G.start, cur, s);
    if constexpr (g + 1 < hgroups(P)) hgroups_run<P, g + 1>(x, y, z, zp, c, s, nxt, cur);
}

// Q(w) of one cell from its coefficient row c: fl = sum_{|m|<=P-1} c_m w^m
// and its gradient by nested Horner (z innermost, derivatives carried along;
// the first step of every chain peeled, so no products with zero), and
// ft = the rank-P part.  The gradient takes ranks 0..P-1 only: the rank-1
// local components of M2L are truncated at |m| <= P-1.  Coefficients arrive
// by scalar loads, one group ahead of their use.
template <int P>
__device__ __forceinline__ void m2p_horner(double x, double y, double z, const double* __restrict__ c, double& fl,
                                           double& ft, double& gx, double& gy, double& gz) {
    double zp[P + 1];
    zp[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= P; ++k) zp[k] = zp[k - 1] * z;
    HState s{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double b0[HG], b1[HG];
    constexpr HGroup G0 = hgroup(P, 0);
#pragma unroll
    for (int k = 0; k < G0.len; ++k) b0[k] = c[G0.start + k];
    hgroups_run<P, 0>(x, y, z, zp, c, s, b0, b1);
    fl = s.V;
    ft = s.T;
    gx = s.Vx;
    gy = s.Vy;
    gz = s.Vz;
}

// W(B): the multipole of each cell C in W(B) evaluated at B's particles (Eq.
// M2L taken to the particle position, ranks 0 and 1 of the result), as
// |u|^-1 Q(w) (see k_m2p_coef) with the gradient by the chain rule through w.
// One workgroup of MW wavefronts per leaf B, lanes over its particles (64 at
// a time); wavefront k takes the entries k, k + MW, ... of W(B), which are
// wave-uniform, so each coefficient row arrives through scalar loads.  The
// MW partial sums meet in LDS and are added to F[s] (the L2P result) in
// wavefront order.
constexpr int MW = 4;
template <int P>
__global__ __launch_bounds__(64 * MW) void k_m2p_leaf(const ABox* __restrict__ boxes, ATree t,
                                                      const double4* __restrict__ Pt, const double* __restrict__ Cm,
                                                      const int32_t* __restrict__ woff,
                                                      const int32_t* __restrict__ wlist, double4* __restrict__ F) {
    __shared__ double4 part[MW][64];
    const int B = blockIdx.x;
    const int w0 = woff[B], w1 = woff[B + 1];
    if (w0 == w1) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int b = t.pb[B], e = t.pe[B];
    for (int s0 = b; s0 < e; s0 += 64) {
        const int s = s0 + lane;
        const bool act = s < e;
        const double4 pt = Pt[act ? s : b];
        double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
#pragma nounroll
        for (int i = w0 + wv; i < w1; i += MW) {
            const int C = __builtin_amdgcn_readfirstlane(wlist[i]);
            const NodeGeom G = node_geom(boxes, t, C);
            const double ux = (pt.x - G.zx) / G.h, uy = (pt.y - G.zy) / G.h, uz = (pt.z - G.zz) / G.h;
            const double r2 = ux * ux + uy * uy + uz * uz;
            const double ir2 = 1.0 / r2;
            const double ir = sqrt(ir2);
            double fl, ft, g0, g1, g2;
            m2p_horner<P>(ux * ir2, uy * ir2, uz * ir2, Cm + (size_t)C * ldc_of(P), fl, ft, g0, g1, g2);
            const double ih = 1.0 / G.h;
            // grad_u [ |u|^-1 Q(w) ] = -u |u|^-3 Q + |u|^-1 (g/|u|^2 - 2 u (u.g)/|u|^4), Q = ranks < P
            const double ug = ux * g0 + uy * g1 + uz * g2;
            const double aa = -ir * ir2 * fl - 2.0 * ir * ir2 * ir2 * ug;
            const double bb = ir * ir2;
            const double ih2 = ih * ih;
            v.x += ir * (fl + ft) * ih;
            v.y += (aa * ux + bb * g0) * ih2;
            v.z += (aa * uy + bb * g1) * ih2;
            v.w += (aa * uz + bb * g2) * ih2;
        }
        part[wv][lane] = v;
        __syncthreads();
        if (wv == 0 && act) {
            double4 f = F[s];
#pragma unroll
            for (int k = 0; k < MW; ++k) {
                const double4 c = part[k][lane];
                f.x += c.x;
                f.y += c.y;
                f.z += c.z;
                f.w += c.w;
            }
            F[s] = f;
        }
        __syncthreads();
    }
}

// Near field, one wavefront per leaf B: the particles of the leaves in U(B)
// (B included; the particle itself contributes nothing) are staged in LDS,
// P2P_KS per lane per round, numbered in list order (entry offsets and
// first particles in LDS, found by binary search).  Lane = (target t,
// source group g): with n targets in a chunk the sources are split over
// G = 64/n groups (source j to group j mod G), whose sums are added in group
// order.  A chunk takes every remaining target when its G n lanes fill at
// least 7/8 of the wavefront, else the largest power of two of them (which
// fills it exactly).  The near field goes to Fn[s] (sorted order); it needs
// nothing of the far field, so it runs beside the expansion passes.
constexpr int P2P_KS = 3;
__global__ __launch_bounds__(64) void k_p2p_leaf(ATree t, const double4* __restrict__ Pt,
                                                 const int32_t* __restrict__ uoff, const int32_t* __restrict__ ulist,
                                                 double4* __restrict__ Fn) {
    constexpr int KS = P2P_KS;
    __shared__ double4 S[64 * KS];
    double4* red = S;  // the group sums, once the sources are no longer read
    __shared__ int epb[64], epre[65];
    const int B = blockIdx.x;
    if (!node_leaf(t.info[B])) return;
    const int lane = threadIdx.x;
    const int b = t.pb[B], e = t.pe[B];
    const int u0 = uoff[B], u1 = uoff[B + 1];
    for (int t0 = b; t0 < e;) {
        int ntc = min(64, e - t0);
        if ((64 / ntc) * ntc * 8 < 64 * 7) ntc = 1 << (31 - __builtin_clz(ntc));
        const int G = 64 / ntc;
        const int g = lane / ntc, tl = lane % ntc;
        const bool active = g < G;
        const int s = t0 + tl;
        const double4 pt = Pt[s];
        double f = 0.0, gx = 0.0, gy = 0.0, gz = 0.0, f2 = 0.0, gx2 = 0.0, gy2 = 0.0, gz2 = 0.0;
        for (int e0 = u0; e0 < u1; e0 += 64) {
            const int ne = min(64, u1 - e0);
            int sz = 0;
            if (lane < ne) {
                const int C = ulist[e0 + lane];
                epb[lane] = t.pb[C];
                sz = t.pe[C] - t.pb[C];
            }
            int incl = sz;  // inclusive scan over the lanes
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int o = __shfl_up(incl, d);
                if (lane >= d) incl += o;
            }
            epre[lane + 1] = incl;
            if (lane == 0) epre[0] = 0;
            __syncthreads();
            const int tot = epre[ne];
            for (int base = 0; base < tot; base += 64 * KS) {
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    const int j = base + lane + 64 * k;
                    if (j < tot) {
                        int lo = 0, hi = ne;  // entry with epre[lo] <= j < epre[lo + 1]
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
                    // are read ahead (indices clamped into the array, values
                    // past cnt unused)
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
        }
        red[lane] = make_double4(f + f2, gx + gx2, gy + gy2, gz + gz2);
        __syncthreads();
        if (g == 0) {
            double4 r = red[tl];
            for (int gg = 1; gg < G; ++gg) {
                const double4 v = red[tl + ntc * gg];
                r.x += v.x;
                r.y += v.y;
                r.z += v.z;
                r.w += v.w;
            }
            Fn[s] = r;
        }
        __syncthreads();
        t0 += ntc;
    }
}

// F (sorted order) -> phi, grad (input order)
__global__ __launch_bounds__(256) void k_scatter_out(int n, const int32_t* __restrict__ idx,
                                                     const double4* __restrict__ F, double* __restrict__ phi,
                                                     double* __restrict__ grad) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double4 v = F[s];
    const size_t o = (size_t)idx[s];
    if (phi) phi[o] = v.x;
    if (grad) {
        grad[3 * o] = v.y;
        grad[3 * o + 1] = v.z;
        grad[3 * o + 2] = v.w;
    }
}

void launch_scatter_out(hipStream_t s, int n, const int32_t* idx, const double4* F, double* phi, double* grad) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scatter_out, dim3(cdiv(n, 256)), dim3(256), 0, s, n, idx, F, phi, grad);
}

void launch_p2l(hipStream_t s, int p, int nn, const ABox* boxes, const ATree& t, const int32_t* xoff, const int32_t* xlist,
                const double4* P, const DevTables& T, double* L) {
    if (nn <= 0) return;
    switch (p) {
#define CASE(PP) case PP: hipLaunchKernelGGL(k_p2l<PP>, dim3(nn), dim3(64), 0, s, boxes, t, xoff, xlist, P, T, L); break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

void launch_p2p_near(hipStream_t s, int n, int nn, const ATree& t, const double4* P, const int32_t* uoff,
                     const int32_t* ulist, double4* Fn) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_p2p_leaf, dim3(nn), dim3(64), 0, s, t, P, uoff, ulist, Fn);
}

void launch_far_adaptive(hipStream_t s, int p, int n, int nn, bool wlists, const ABox* boxes, const ATree& t,
                         const int32_t* leaf_of, const double4* P, const double* L, const double* Cm,
                         const int32_t* woff, const int32_t* wlist, double4* F, double4* Fn, const int32_t* idx,
                         bool to_F, double* phi, double* grad) {
    if (n <= 0) return;
    const dim3 grid(cdiv(n, 256)), blk(256);
    switch (p) {
#define CASE(PP)                                                                                                  \
    case PP:                                                                                                      \
        if (wlists) hipLaunchKernelGGL(k_m2p_leaf<PP>, dim3(nn), dim3(64 * MW), 0, s, boxes, t, P, Cm, woff, wlist, Fn); \
        hipLaunchKernelGGL(k_l2p_adaptive<PP>, grid, blk, 0, s, n, boxes, t, leaf_of, P, L, F, Fn, idx, to_F, phi,     \
                           grad);                                                                                  \
        break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

void launch_wlist_adaptive(hipStream_t s, int p, int nn, const ABox* boxes, const ATree& t, const double4* P,
                           const double* Cm, const int32_t* woff, const int32_t* wlist, double4* F) {
    if (nn <= 0) return;
    switch (p) {
#define CASE(PP)                                                                                                   \
    case PP:                                                                                                       \
        hipLaunchKernelGGL(k_m2p_leaf<PP>, dim3(nn), dim3(64 * MW), 0, s, boxes, t, P, Cm, woff, wlist, F);         \
        break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

// ------------------------------------------------------------------ M2L orders per pair

// class of |v|^2 among the 15 occupied values (see k_mlp_decide)
__device__ inline int class_of_r2_a(int r2) {
    constexpr int8_t tab[28] = {-1, -1, -1, -1, 0, 1, 2, -1, 3, 4, 5, 6, 7, 8, 9, -1,
                                -1, 10, 11, 12, -1, -1, 13, -1, -1, -1, -1, 14};
    return (r2 >= 0 && r2 < 28) ? tab[r2] : -1;
}

// One wavefront per (tile, offset): the order of its M2L.  Each pair asks
// for ordn[source * 15 + class of |v|^2]; the tile's M2L at this offset runs
// at the largest order asked among its pairs (no pair gets less than it
// asked for, and the source rows are read once).  With a table by |v|^2
// every pair of a (tile, offset) asks for the same order.
__global__ __launch_bounds__(64) void k_m2l_orders(int tt, const int4* __restrict__ tiles,
                                                   const int32_t* __restrict__ src_tab,
                                                   const int16_t* __restrict__ kslot, const int8_t* __restrict__ ordn,
                                                   int8_t* __restrict__ tq, int32_t* __restrict__ ocnt) {
    const int tile = blockIdx.x / 189, iv = blockIdx.x % 189;
    const int lane = threadIdx.x;
    const int ks = kslot[tiles[tile].x * 189 + iv];  // slot of r = target - source
    const int rx = ks % 7 - 3, ry = (ks / 7) % 7 - 3, rz = ks / 49 - 3;
    const int cls = class_of_r2_a(rx * rx + ry * ry + rz * rz);
    int omax = -1, npair = 0;
    for (int r = lane; r < tt; r += 64) {
        const int src = src_tab[(189 * (size_t)tile + iv) * tt + r];
        if (src >= 0) {
            omax = max(omax, (int)ordn[(size_t)src * NCLASS + cls]);
            ++npair;
        }
    }
    for (int off = 1; off < 64; off <<= 1) {
        omax = max(omax, __shfl_xor(omax, off));
        npair += __shfl_xor(npair, off);
    }
    if (lane == 0) tq[blockIdx.x] = (int8_t)omax;
    // pairs per order (the chosen-order histogram)
    if (lane <= 10) ocnt[(size_t)lane * gridDim.x + blockIdx.x] = lane == omax ? npair : 0;
}

// One wavefront per tile: its active offsets in offset order (an order in
// tq >= 0, or with tq null a source in vcount), their orders (tq, or p).
__global__ __launch_bounds__(64) void k_active_offsets(int p, const int8_t* __restrict__ tq,
                                                       const int32_t* __restrict__ vcount,
                                                       int16_t* __restrict__ ivlist, int8_t* __restrict__ ivord,
                                                       int32_t* __restrict__ ivcnt) {
    const int tile = blockIdx.x;
    const int lane = threadIdx.x;
    int cnt = 0;
    for (int b = 0; b < 189; b += 64) {
        const int iv = b + lane;
        const size_t e = (size_t)tile * 189 + iv;
        int q = -1;
        if (iv < 189) q = tq ? (int)tq[e] : (vcount[e] > 0 ? p : -1);
        const bool on = q >= 0;
        const unsigned long long bal = __ballot(on);
        if (on) {
            const int k = cnt + __popcll(bal & ((1ull << lane) - 1ull));
            ivlist[(size_t)tile * 189 + k] = (int16_t)iv;
            ivord[(size_t)tile * 189 + k] = (int8_t)q;
        }
        cnt += __popcll(bal);
    }
    if (lane == 0) ivcnt[tile] = cnt;
}

__global__ void k_fill0(long long n, double* __restrict__ a) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0.0;
}

void launch_m2l_orders(hipStream_t s, int tt, int ntiles, const int4* tiles, const int32_t* src_tab,
                       const int16_t* kslot, const int8_t* ordn, int8_t* tq, int32_t* ocnt) {
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(k_m2l_orders, dim3(189 * ntiles), dim3(64), 0, s, tt, tiles, src_tab, kslot, ordn, tq, ocnt);
}

void launch_active_offsets(hipStream_t s, int ntiles, int p, const int8_t* tq, const int32_t* vcount,
                           int16_t* ivlist, int8_t* ivord, int32_t* ivcnt) {
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(k_active_offsets, dim3(ntiles), dim3(64), 0, s, p, tq, vcount, ivlist, ivord, ivcnt);
}

// FP32 <-> FP64 copies of the caller's arrays (the FP32 entry points)
__global__ void k_widen(long long n, const float* __restrict__ in, double* __restrict__ out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)in[i];
}
__global__ void k_narrow(long long n, const double* __restrict__ in, float* __restrict__ out) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

void launch_widen(hipStream_t s, long long n, const float* in, double* out) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_widen, dim3(cdiv(n, 256)), dim3(256), 0, s, n, in, out);
}

void launch_narrow(hipStream_t s, long long n, const double* in, float* out) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_narrow, dim3(cdiv(n, 256)), dim3(256), 0, s, n, in, out);
}

void launch_fill0(hipStream_t s, long long n, double* a) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill0, dim3(cdiv(n, 256)), dim3(256), 0, s, n, a);
}

}  // namespace ctfmm
