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

__device__ inline NodeGeom node_geom(const ABox* boxes, const ATree& t, int g) {
    return node_geom(boxes[t.sys[g]], t.key[g], node_level(t.info[g]));
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

__global__ void k_keys64(int n, ASys sy, const double* __restrict__ xyz, const ABox* __restrict__ boxes,
                         uint64_t* __restrict__ keys, int32_t* __restrict__ idx, int* __restrict__ err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int sidx = sy.nsys == 1 ? 0 : seg_of(sy.goff, sy.nsys, i);
    const size_t gi = (size_t)sy.gbase[sidx] + (size_t)(i - sy.goff[sidx]);
    const ABox box = boxes[sidx];
    const double x = xyz[3 * gi], y = xyz[3 * gi + 1], z = xyz[3 * gi + 2];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) atomicOr(err, 1);
    keys[i] = spread21(acoord(x, box.lo[0], box.side)) | (spread21(acoord(y, box.lo[1], box.side)) << 1) |
              (spread21(acoord(z, box.lo[2], box.side)) << 2);
    idx[i] = (int32_t)gi;
}

void launch_keys64(hipStream_t s, int n, const ASys& sy, const double* xyz, const ABox* boxes, uint64_t* keys,
                   int32_t* idx, int* err) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_keys64, dim3(cdiv(n, 256)), dim3(256), 0, s, n, sy, xyz, boxes, keys, idx, err);
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
// range of each octant (binary search of the sorted keys inside its range).
// flag[8i+o] = 1 for every non-empty octant of a split node.
__global__ void k_split(int level, int first, int count, int leaf_max, const uint64_t* __restrict__ keys, ATree t,
                        int32_t* __restrict__ flag, int32_t* __restrict__ cstart) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int g = first + i;
    const int b = t.pb[g], e = t.pe[g];
    const bool split = (e - b) > leaf_max && level < AMAX;
    t.info[g] = level | (split ? 0 : 1 << 8);
#pragma unroll
    for (int o = 0; o < 8; ++o) t.child[8 * (size_t)g + o] = -1;
    if (!split) {
#pragma unroll
        for (int o = 0; o < 8; ++o) flag[8 * i + o] = 0;
        return;
    }
    const int sh = 3 * (AMAX - level - 1);
    const uint64_t base = t.key[g] * 8;
    int s0 = b;
    for (int o = 0; o < 8; ++o) {
        // first position in [s0, e) whose octant prefix exceeds base + o
        int lo = s0, hi = e;
        while (lo < hi) {
            const int mid = lo + ((hi - lo) >> 1);
            if ((keys[mid] >> sh) <= base + (uint64_t)o) lo = mid + 1; else hi = mid;
        }
        flag[8 * i + o] = lo > s0 ? 1 : 0;
        cstart[8 * i + o] = s0;
        s0 = lo;
    }
}

// children of the split nodes of a level, at next_first + (inclusive scan - 1)
__global__ void k_emit(int level, int first, int count, int next_first, const int32_t* __restrict__ flag,
                       const int32_t* __restrict__ incl, const int32_t* __restrict__ cstart, ATree t) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
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
    hipLaunchKernelGGL(k_split, dim3(cdiv(count, 128)), dim3(128), 0, s, level, first, count, leaf_max, keys, t, flag,
                       cstart);
}

void launch_emit(hipStream_t s, int level, int first, int count, int next_first, const int32_t* flag,
                 const int32_t* incl, const int32_t* cstart, const ATree& t) {
    hipLaunchKernelGGL(k_emit, dim3(cdiv(8ll * count, 256)), dim3(256), 0, s, level, first, count, next_first, flag,
                       incl, cstart, t);
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

// ------------------------------------------------------------------ U, W, X lists

// One thread per node.  FILL = false counts the entries of each list,
// FILL = true writes them at the offsets of the exclusive scans.  Both passes
// enumerate in the same order.
template <bool FILL>
__global__ void k_lists(int nn, ATree t, int32_t* __restrict__ ucnt, int32_t* __restrict__ wcnt,
                        int32_t* __restrict__ xcnt, const int32_t* __restrict__ uoff, const int32_t* __restrict__ woff,
                        const int32_t* __restrict__ xoff, int32_t* __restrict__ ulist, int32_t* __restrict__ wlist,
                        int32_t* __restrict__ xlist) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= nn) return;
    const int info = t.info[B];
    const int lb = node_level(info);
    const uint64_t kb = t.key[B];
    int nu = 0, nw = 0, nx = 0;
    auto put_u = [&](int c) {
        if (FILL) ulist[uoff[B] + nu] = c;
        ++nu;
    };
    auto put_w = [&](int c) {
        if (FILL) wlist[woff[B] + nw] = c;
        ++nw;
    };
    auto put_x = [&](int c) {
        if (FILL) xlist[xoff[B] + nx] = c;
        ++nx;
    };
    const int32_t* nbB = t.nb + 27 * (size_t)B;
    if (node_leaf(info)) {
        // same-level and coarser adjacent leaves (a coarser leaf can fill several entries)
        for (int d = 0; d < 27; ++d) {
            const int C = nbB[d];
            if (C < 0 || !node_leaf(t.info[C])) continue;
            bool dup = false;
            for (int e = 0; e < d; ++e) dup |= nbB[e] == C;
            if (!dup) put_u(C);
        }
        // finer cells inside the same-level non-leaf neighbours: adjacent leaves
        // join U, non-adjacent cells (whose parent is adjacent) join W
        int stack[8 * AMAX + 8];
        for (int d = 0; d < 27; ++d) {
            const int Q = nbB[d];
            if (Q < 0 || node_leaf(t.info[Q])) continue;  // a non-leaf entry is always same-level
            int sp = 0;
            stack[sp++] = Q;
            while (sp > 0) {
                const int A = stack[--sp];
                for (int o = 0; o < 8; ++o) {
                    const int c = t.child[8 * (size_t)A + o];
                    if (c < 0) continue;
                    const int ci = t.info[c];
                    if (!adjacent(t.key[c], node_level(ci), kb, lb)) put_w(c);
                    else if (node_leaf(ci)) put_u(c);
                    else stack[sp++] = c;
                }
            }
        }
    }
    // X: leaves coarser than B that touch parent(B) but not B
    if (lb >= 2) {
        const int32_t* nbP = t.nb + 27 * (size_t)t.par[B];
        for (int d = 0; d < 27; ++d) {
            const int C = nbP[d];
            if (C < 0) continue;
            const int ci = t.info[C];
            if (!node_leaf(ci)) continue;
            bool dup = false;
            for (int e = 0; e < d; ++e) dup |= nbP[e] == C;
            if (dup) continue;
            if (!adjacent(t.key[C], node_level(ci), kb, lb)) put_x(C);
        }
    }
    if (!FILL) {
        ucnt[B] = nu;
        wcnt[B] = nw;
        xcnt[B] = nx;
    }
}

void launch_lists(hipStream_t s, bool fill, int nn, const ATree& t, int32_t* ucnt, int32_t* wcnt, int32_t* xcnt,
                  const int32_t* uoff, const int32_t* woff, const int32_t* xoff, int32_t* ulist, int32_t* wlist,
                  int32_t* xlist) {
    if (fill)
        hipLaunchKernelGGL(k_lists<true>, dim3(cdiv(nn, 64)), dim3(64), 0, s, nn, t, ucnt, wcnt, xcnt, uoff, woff,
                           xoff, ulist, wlist, xlist);
    else
        hipLaunchKernelGGL(k_lists<false>, dim3(cdiv(nn, 64)), dim3(64), 0, s, nn, t, ucnt, wcnt, xcnt, uoff, woff,
                           xoff, ulist, wlist, xlist);
}

// ------------------------------------------------------------------ M2L tiles

// sort key of a node: level and octant (targets of one tile share the octant)
__global__ void k_lvloct(int nn, ATree t, uint32_t* __restrict__ k, int32_t* __restrict__ v) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nn) return;
    k[g] = ((uint32_t)node_level(t.info[g]) << 3) | (uint32_t)(t.key[g] & 7);
    v[g] = g;
}

__global__ void k_clear_i32(int n, int32_t* __restrict__ a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0;
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

// One wave per (tile, offset): the targets of the tile (tt of them, lanes
// take slots lane, lane + 64) and the source cell of the offset for each
// (child q of the parent's neighbour u, or -1).  vcount = sources that exist.
__global__ __launch_bounds__(64) void k_m2l_tables(int tt, const int4* __restrict__ tiles,
                                                   const int32_t* __restrict__ sorted, ATree t,
                                                   const int16_t* __restrict__ qu_list, int32_t* __restrict__ tgt_tab,
                                                   int32_t* __restrict__ src_tab, int32_t* __restrict__ vcount) {
    const int tile = blockIdx.x / 189, iv = blockIdx.x % 189;
    const int lane = threadIdx.x;
    const int4 d = tiles[tile];  // (octant, first sorted position, count, level)
    const int qu = qu_list[d.x * 189 + iv];
    int cnt = 0;
    for (int r = lane; r < tt; r += 64) {
        const int tg = r < d.z ? sorted[d.y + r] : -1;
        if (iv == 0) tgt_tab[tt * (size_t)tile + r] = tg;
        int src = -1;
        if (tg >= 0) {
            const int Q = t.nb[27 * (size_t)t.par[tg] + (qu & 31)];
            if (Q >= 0 && !node_leaf(t.info[Q])) src = t.child[8 * (size_t)Q + (qu >> 5)];
        }
        src_tab[(189 * (size_t)tile + iv) * tt + r] = src;
        cnt += __popcll(__ballot(src >= 0));
    }
    if (lane == 0) vcount[blockIdx.x] = cnt;
}

void launch_m2l_tables(hipStream_t s, int tt, int ntiles, const int4* tiles, const int32_t* sorted, const ATree& t,
                       const int16_t* qu_list, int32_t* tgt_tab, int32_t* src_tab, int32_t* vcount) {
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(k_m2l_tables, dim3(189 * ntiles), dim3(64), 0, s, tt, tiles, sorted, t, qu_list, tgt_tab,
                       src_tab, vcount);
}

// ------------------------------------------------------------------ P2M, M2M, L2L on node lists

// P2M of every leaf among nodes [first, first+count): one wavefront per node
__global__ __launch_bounds__(64) void k_p2m_nodes(int p, int first, const ABox* __restrict__ boxes, ATree t, const double4* __restrict__ P,
                                                  DevTables T, double* __restrict__ M) {
    const int g = first + blockIdx.x;
    const int info = t.info[g];
    if (!node_leaf(info)) return;
    const NodeGeom G = node_geom(boxes, t, g);
    p2m_cell(p, G.zx, G.zy, G.zz, G.h, t.pb[g], t.pe[g], P, T, M + (size_t)g * ldm_of(p));
}

void launch_p2m_nodes(hipStream_t s, int p, int first, int count, const ABox* boxes, const ATree& t, const double4* P,
                      const DevTables& T, double* M) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_p2m_nodes, dim3(count), dim3(64), 0, s, p, first, boxes, t, P, T, M);
}

constexpr int ANP = 8;  // parents per workgroup in M2M/L2L

__device__ inline int rank_of_a(int k) {
    int r = 0;
    while ((r + 1) * (r + 1) <= k) ++r;
    return r;
}

// M~(parent) = sum over existing children of A_o M~(child), for the non-leaf
// nodes among [first, first+count) (the leaves keep their P2M result)
__global__ __launch_bounds__(128) void k_m2m_nodes(int p, int first, int count, ATree t, double* __restrict__ M,
                                                   const double* __restrict__ m2m_t) {
    const int P0 = blockIdx.x * ANP;
    const int nc = (p + 1) * (p + 1);
    const int ldm = ldm_of(p);
    __shared__ double ch[ANP][8][NIND];
    __shared__ int isleaf[ANP];
    const int np = min(ANP, count - P0);
    if ((int)threadIdx.x < ANP) isleaf[threadIdx.x] = (int)threadIdx.x < np ? node_leaf(t.info[first + P0 + threadIdx.x]) : 1;
    for (int x = threadIdx.x; x < np * 8 * nc; x += 128) {
        const int pp = x / (8 * nc), r = x % (8 * nc), o = r / nc, j = r % nc;
        const int c = t.child[8 * (size_t)(first + P0 + pp) + o];
        ch[pp][o][j] = c >= 0 ? M[(size_t)c * ldm + j] : 0.0;
    }
    __syncthreads();
    for (int n = threadIdx.x; n < ldm; n += 128) {
        double acc[ANP];
#pragma unroll
        for (int pp = 0; pp < ANP; ++pp) acc[pp] = 0.0;
        if (n < nc) {
            const int r = rank_of_a(n);
            const int jmax = (r + 1) * (r + 1);
            for (int o = 0; o < 8; ++o) {
                const double* A = m2m_t + (size_t)o * NIND * NIND;
                for (int j = 0; j < jmax; ++j) {
                    const double a = A[(size_t)j * NIND + n];
#pragma unroll
                    for (int pp = 0; pp < ANP; ++pp) acc[pp] += a * ch[pp][o][j];
                }
            }
        }
        for (int pp = 0; pp < np; ++pp)
            if (!isleaf[pp]) M[(size_t)(first + P0 + pp) * ldm + n] = acc[pp];
    }
}

void launch_m2m_nodes(hipStream_t s, int p, int first, int count, const ATree& t, double* M, const DevTables& T) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_m2m_nodes, dim3(cdiv(count, ANP)), dim3(128), 0, s, p, first, count, t, M, T.m2m_t);
}

// L~(child) += B_o L~(parent) for the existing children of the non-leaf nodes
// among [first, first+count)
__global__ __launch_bounds__(256) void k_l2l_nodes(int p, int first, int count, ATree t, double* __restrict__ L,
                                                   const double* __restrict__ l2l_t) {
    const int P0 = blockIdx.x * ANP;
    const int nc = (p + 1) * (p + 1);
    const int ldm = ldm_of(p);
    __shared__ double lp[ANP][NIND];
    __shared__ int cid[ANP][8];
    const int np = min(ANP, count - P0);
    if ((int)threadIdx.x < ANP * 8) {
        const int pp = threadIdx.x / 8, o = threadIdx.x % 8;
        cid[pp][o] = pp < np ? t.child[8 * (size_t)(first + P0 + pp) + o] : -1;
    }
    for (int x = threadIdx.x; x < np * nc; x += 256) lp[x / nc][x % nc] = L[(size_t)(first + P0 + x / nc) * ldm + x % nc];
    __syncthreads();
    for (int x = threadIdx.x; x < 8 * nc; x += 256) {
        const int o = x / nc, n = x % nc;
        const double* Bm = l2l_t + (size_t)o * NIND * NIND;
        double acc[ANP];
#pragma unroll
        for (int pp = 0; pp < ANP; ++pp) acc[pp] = 0.0;
        const int r = rank_of_a(n);
        for (int j = r * r; j < nc; ++j) {
            const double bcoef = Bm[(size_t)j * NIND + n];
#pragma unroll
            for (int pp = 0; pp < ANP; ++pp) acc[pp] += bcoef * lp[pp][j];
        }
        for (int pp = 0; pp < np; ++pp) {
            const int c = cid[pp][o];
            if (c >= 0) L[(size_t)c * ldm + n] += acc[pp];
        }
    }
}

void launch_l2l_nodes(hipStream_t s, int p, int first, int count, const ATree& t, double* L, const DevTables& T) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_l2l_nodes, dim3(cdiv(count, ANP)), dim3(256), 0, s, p, first, count, t, L, T.l2l_t);
}

// ------------------------------------------------------------------ X list: direct local expansions

// L~_n(B) += q D~_n((z_B - x_a)/h_B) for the particles a of every leaf in
// X(B) (Eq. M2L with the multipole of a single charge at its own position,
// in the scaled variables).  One wavefront per node; the particles of all its
// X leaves are taken 64 at a time as one sequence (lane i takes the i-th
// particle after a wave-uniform cursor), and the lanes' derivative tensors
// meet in LDS, where lane k sums component k.
template <int P>
__global__ __launch_bounds__(64) void k_p2l(const ABox* __restrict__ boxes, ATree t, const int32_t* __restrict__ xoff,
                                            const int32_t* __restrict__ xlist, const double4* __restrict__ Pt,
                                            double* __restrict__ L) {
    constexpr int NC = (P + 1) * (P + 1);
    constexpr int STR = NC | 1;
    const int B = blockIdx.x;
    const int x0 = xoff[B], x1 = xoff[B + 1];
    if (x0 == x1) return;
    const int lane = threadIdx.x;
    const NodeGeom G = node_geom(boxes, t, B);
    __shared__ double Ds[64 * STR];
    constexpr int KPL = (NC + 63) / 64;
    double acc[KPL];
#pragma unroll
    for (int k = 0; k < KPL; ++k) acc[k] = 0.0;
    int total = 0;
    for (int xi = x0; xi < x1; ++xi) {
        const int C = xlist[xi];
        total += t.pe[C] - t.pb[C];
    }
    int cx = x0, cs = t.pb[xlist[x0]];  // cursor: X entry and particle of the next chunk
    for (int base = 0; base < total; base += 64) {
        const int cnt = min(64, total - base);
        if (lane < cnt) {
            int li = cx, ls = cs, rem = lane;
            while (true) {
                const int avail = t.pe[xlist[li]] - ls;
                if (rem < avail) {
                    ls += rem;
                    break;
                }
                rem -= avail;
                ++li;
                ls = t.pb[xlist[li]];
            }
            const double4 pt = Pt[ls];
            double D[NC];
            gen_dtensor<P>((G.zx - pt.x) / G.h, (G.zy - pt.y) / G.h, (G.zz - pt.z) / G.h, D);
#pragma unroll
            for (int k = 0; k < NC; ++k) Ds[lane * STR + k] = pt.w * D[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KPL; ++k) {
            const int kk = lane + 64 * k;
            if (kk < NC)
                for (int i = 0; i < cnt; ++i) acc[k] += Ds[i * STR + kk];
        }
        __syncthreads();
        // advance the cursor by the chunk
        int rem = cnt;
        while (rem > 0) {
            const int avail = t.pe[xlist[cx]] - cs;
            if (rem < avail) {
                cs += rem;
                rem = 0;
            } else {
                rem -= avail;
                ++cx;
                if (cx < x1) cs = t.pb[xlist[cx]];
            }
        }
    }
    double* Lb = L + (size_t)B * ldm_of(P);
#pragma unroll
    for (int k = 0; k < KPL; ++k) {
        const int kk = lane + 64 * k;
        if (kk < NC) Lb[kk] += acc[k];
    }
}

// ------------------------------------------------------------------ W list and near field

// (-1)^n (2n-1)!! times the rank-n components: with these weights the
// multipole potential is a polynomial at the inverted point (k_near_adaptive)
__global__ void k_mhat(int p, int first, int count, const double* __restrict__ M, double* __restrict__ Mh) {
    const int nc = (p + 1) * (p + 1);
    const int ldm = ldm_of(p);
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (long long)count * ldm) return;
    const int k = (int)(gid % ldm);
    const size_t row = (size_t)first + gid / ldm;
    double w = 0.0;
    if (k < nc) {
        const int r = rank_of_a(k);
        w = 1.0;
        for (int i = 1; i <= r; ++i) w *= -(double)(2 * i - 1);
    }
    Mh[row * ldm + k] = w * M[row * ldm + k];
}

void launch_mhat(hipStream_t s, int p, int first, int count, const double* M, double* Mh) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_mhat, dim3(cdiv((long long)count * ldm_of(p), 256)), dim3(256), 0, s, p, first, count, M, Mh);
}

__device__ inline void pair_add_a(double xb, double yb, double zb, double4 src, double& f, double& gx, double& gy,
                                  double& gz) {
    const double dx = xb - src.x, dy = yb - src.y, dz = zb - src.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) return;  // coincident pair: contributes nothing
    double y = __builtin_amdgcn_rsq(r2);
    y = y * (1.5 - 0.5 * r2 * y * y);
    y = y * (1.5 - 0.5 * r2 * y * y);
    f += src.w * y;
    const double ir3 = src.w * y * y * y;
    gx -= ir3 * dx;
    gy -= ir3 * dy;
    gz -= ir3 * dz;
}

// Far field of one sorted particle s (one thread each) from the local
// expansion of its leaf B (Eq. L2P), into F[s]; zero for leaves above level 2.
template <int P>
__global__ __launch_bounds__(256) void k_l2p_adaptive(int n, const ABox* __restrict__ boxes, ATree t, const int32_t* __restrict__ leaf_of,
                                                      const double4* __restrict__ Pt, const double* __restrict__ L,
                                                      double4* __restrict__ F) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int B = leaf_of[s];
    const int lb = node_level(t.info[B]);
    double4 out = make_double4(0.0, 0.0, 0.0, 0.0);
    if (lb >= 2) {
        const double4 pt = Pt[s];
        const NodeGeom G = node_geom(boxes, t, B);
        double lf = 0.0, lx = 0.0, ly = 0.0, lz = 0.0;
        gen_l2p<P>((pt.x - G.zx) / G.h, (pt.y - G.zy) / G.h, (pt.z - G.zz) / G.h, L + (size_t)B * ldm_of(P), lf, lx,
                   ly, lz);
        const double ih2 = 1.0 / (G.h * G.h);
        out = make_double4(lf / G.h, lx * ih2, ly * ih2, lz * ih2);
    }
    F[s] = out;
}

// W(B): the multipole of each cell C in W(B) evaluated at B's particles (Eq.
// M2L at the particle, ranks 0 and 1 of the result).  Against a traceless M
// only the r^n part of D_n survives:
//   sum_{|m|=n} M_m D_m(r)/m! = (-1)^n (2n-1)!! |r|^(-2n-1) sum_{|m|=n} M_m r^m/m!
// which is |r|^-1 times the rank-n polynomial of the weighted M^ at the
// inverted point w = r/|r|^2.  The potential takes ranks 0..p; the gradient
// takes ranks 0..p-1 (the rank-1 local components are truncated at
// |m| <= p-1), by the chain rule through w.
template <int P>
__device__ inline double4 m2p_eval(const ABox* __restrict__ boxes, const ATree& t, int C, double4 pt, const double* __restrict__ Mh) {
    const NodeGeom G = node_geom(boxes, t, C);
    const double ux = (pt.x - G.zx) / G.h, uy = (pt.y - G.zy) / G.h, uz = (pt.z - G.zz) / G.h;
    const double r2 = ux * ux + uy * uy + uz * uz;
    const double ir2 = 1.0 / r2;
    const double ir = sqrt(ir2);
    double fl = 0.0, ft = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
    gen_m2p<P>(ux * ir2, uy * ir2, uz * ir2, Mh + (size_t)C * ldm_of(P), fl, ft, g0, g1, g2);
    const double ih = 1.0 / G.h;
    // grad_u [ |u|^-1 Q(w) ] = -u |u|^-3 Q + |u|^-1 (g/|u|^2 - 2 u (u.g)/|u|^4), Q = ranks < p
    const double ug = ux * g0 + uy * g1 + uz * g2;
    const double a = -ir * ir2 * fl - 2.0 * ir * ir2 * ir2 * ug;
    const double b = ir * ir2;
    const double ih2 = ih * ih;
    return make_double4(ir * (fl + ft) * ih, (a * ux + b * g0) * ih2, (a * uy + b * g1) * ih2,
                        (a * uz + b * g2) * ih2);
}

// number of (target particle, W entry) pairs of every node
__global__ void k_wpairs_count(int nn, ATree t, const int32_t* __restrict__ woff, long long* __restrict__ cnt) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= nn) return;
    cnt[B] = (long long)(woff[B + 1] - woff[B]) * (t.pe[B] - t.pb[B]);
}

void launch_wpairs_count(hipStream_t s, int nn, const ATree& t, const int32_t* woff, long long* cnt) {
    hipLaunchKernelGGL(k_wpairs_count, dim3(cdiv(nn, 256)), dim3(256), 0, s, nn, t, woff, cnt);
}

// One thread per pair g, ordered [leaf B][W entry i][target]: the pair's
// contribution into buf[g] (consecutive threads share the source cell)
template <int P>
__global__ __launch_bounds__(256) void k_m2p_pairs(long long npairs, int nn, const ABox* __restrict__ boxes, ATree t,
                                                   const double4* __restrict__ Pt, const double* __restrict__ Mh,
                                                   const int32_t* __restrict__ woff,
                                                   const int32_t* __restrict__ wlist,
                                                   const long long* __restrict__ poff, double4* __restrict__ buf) {
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= npairs) return;
    int lo = 0, hi = nn;  // last B with poff[B] <= g
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (poff[mid] <= g) lo = mid; else hi = mid;
    }
    const int B = lo;
    const int nt = t.pe[B] - t.pb[B];
    const long long r = g - poff[B];
    const int i = (int)(r / nt), tt = (int)(r % nt);
    buf[g] = m2p_eval<P>(boxes, t, wlist[woff[B] + i], Pt[t.pb[B] + tt], Mh);
}

// F[s] += the W contributions of particle s, summed in list order
__global__ __launch_bounds__(256) void k_m2p_reduce(int n, ATree t, const int32_t* __restrict__ leaf_of,
                                                    const int32_t* __restrict__ woff,
                                                    const long long* __restrict__ poff,
                                                    const double4* __restrict__ buf, double4* __restrict__ F) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int B = leaf_of[s];
    const int nw = woff[B + 1] - woff[B];
    if (nw == 0) return;
    const int nt = t.pe[B] - t.pb[B];
    const int tt = s - t.pb[B];
    double4 v = F[s];
    for (int i = 0; i < nw; ++i) {
        const double4 c = buf[poff[B] + (long long)i * nt + tt];
        v.x += c.x;
        v.y += c.y;
        v.z += c.z;
        v.w += c.w;
    }
    F[s] = v;
}

// Near field: one thread per sorted particle s in leaf B; direct sum over the
// particles of the leaves in U(B), self excluded, plus the far field F[s].
// Writes phi and grad in input order, or with to_F the total back into F[s].
__global__ __launch_bounds__(256) void k_p2p_adaptive(int n, ATree t, const int32_t* __restrict__ leaf_of,
                                                      const double4* __restrict__ Pt, double4* __restrict__ F,
                                                      const int32_t* __restrict__ uoff,
                                                      const int32_t* __restrict__ ulist,
                                                      const int32_t* __restrict__ idx, bool to_F,
                                                      double* __restrict__ phi, double* __restrict__ grad) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int B = leaf_of[s];
    const double4 pt = Pt[s];
    const double4 fv = F[s];
    double f = fv.x, gx = fv.y, gy = fv.z, gz = fv.w;
    for (int j = uoff[B]; j < uoff[B + 1]; ++j) {
        const int C = ulist[j];
        const int e = t.pe[C];
        for (int s2 = t.pb[C]; s2 < e; ++s2) {
            if (s2 == s) continue;
            pair_add_a(pt.x, pt.y, pt.z, Pt[s2], f, gx, gy, gz);
        }
    }
    if (to_F) {
        F[s] = make_double4(f, gx, gy, gz);
        return;
    }
    const size_t o = (size_t)idx[s];
    if (phi) phi[o] = f;
    if (grad) {
        grad[3 * o] = gx;
        grad[3 * o + 1] = gy;
        grad[3 * o + 2] = gz;
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
                const double4* P, double* L) {
    if (nn <= 0) return;
    switch (p) {
#define CASE(PP) case PP: hipLaunchKernelGGL(k_p2l<PP>, dim3(nn), dim3(64), 0, s, boxes, t, xoff, xlist, P, L); break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
}

void launch_near_adaptive(hipStream_t s, int p, int n, int nn, long long wpairs, const ABox* boxes, const ATree& t,
                          const int32_t* leaf_of, const double4* P, const double* L, const double* Mh,
                          const int32_t* woff, const int32_t* wlist, const long long* wpoff, double4* wbuf,
                          const int32_t* uoff, const int32_t* ulist, const int32_t* idx, double4* F, bool to_F,
                          double* phi, double* grad) {
    if (n <= 0) return;
    const dim3 grid(cdiv(n, 256)), blk(256);
    const dim3 wgrid((unsigned)((wpairs + 255) / 256));
    switch (p) {
#define CASE(PP)                                                                                                  \
    case PP:                                                                                                      \
        hipLaunchKernelGGL(k_l2p_adaptive<PP>, grid, blk, 0, s, n, boxes, t, leaf_of, P, L, F);                     \
        if (wpairs > 0) {                                                                                         \
            hipLaunchKernelGGL(k_m2p_pairs<PP>, wgrid, blk, 0, s, wpairs, nn, boxes, t, P, Mh, woff, wlist, wpoff,  \
                               wbuf);                                                                             \
            hipLaunchKernelGGL(k_m2p_reduce, grid, blk, 0, s, n, t, leaf_of, woff, wpoff, wbuf, F);               \
        }                                                                                                         \
        break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
#undef CASE
        default: break;
    }
    hipLaunchKernelGGL(k_p2p_adaptive, grid, blk, 0, s, n, t, leaf_of, P, F, uoff, ulist, idx, to_F, phi, grad);
}

// ------------------------------------------------------------------ M2L orders per pair

// class of |v|^2 among the 15 occupied values (see k_mlp_decide)
__device__ inline int class_of_r2_a(int r2) {
    constexpr int8_t tab[28] = {-1, -1, -1, -1, 0, 1, 2, -1, 3, 4, 5, 6, 7, 8, 9, -1,
                                -1, 10, 11, 12, -1, -1, 13, -1, -1, -1, -1, 14};
    return (r2 >= 0 && r2 < 28) ? tab[r2] : -1;
}

// One wavefront per (tile, offset): the order of its pairs into ord_tab
// (same layout as src_tab) and as a one-bit mask.  Each pair asks for
// ordn[source * 15 + class of |v|^2]; the tile's M2L at this offset runs at
// the largest order asked among its pairs (no pair gets less than it asked
// for, and the source rows are staged once).  With a table by |v|^2 every
// pair of a (tile, offset) asks for the same order.
__global__ __launch_bounds__(64) void k_m2l_orders(int tt, const int4* __restrict__ tiles,
                                                   const int32_t* __restrict__ src_tab,
                                                   const int16_t* __restrict__ kslot, const int8_t* __restrict__ ordn,
                                                   int8_t* __restrict__ ord_tab, uint16_t* __restrict__ omask,
                                                   int32_t* __restrict__ ocnt) {
    const int tile = blockIdx.x / 189, iv = blockIdx.x % 189;
    const int lane = threadIdx.x;
    const int ks = kslot[tiles[tile].x * 189 + iv];  // slot of r = target - source
    const int rx = ks % 7 - 3, ry = (ks / 7) % 7 - 3, rz = ks / 49 - 3;
    const int cls = class_of_r2_a(rx * rx + ry * ry + rz * rz);
    int omax = -1;
    for (int r = lane; r < tt; r += 64) {
        const int src = src_tab[(189 * (size_t)tile + iv) * tt + r];
        if (src >= 0) omax = max(omax, (int)ordn[(size_t)src * NCLASS + cls]);
    }
    for (int off = 1; off < 64; off <<= 1) omax = max(omax, __shfl_xor(omax, off));
    for (int r = lane; r < tt; r += 64) {
        const size_t e = (189 * (size_t)tile + iv) * tt + r;
        ord_tab[e] = src_tab[e] >= 0 ? (int8_t)omax : (int8_t)-1;
    }
    if (lane == 0) omask[blockIdx.x] = omax >= 0 ? (uint16_t)(1u << omax) : (uint16_t)0;
    // pairs per order (the chosen-order histogram)
    const size_t stride = (size_t)gridDim.x;
    for (int o = 0; o <= 10; ++o) {
        int cnt = 0;
        for (int r = lane; r < tt; r += 64) cnt += ord_tab[(189 * (size_t)tile + iv) * tt + r] == o;
        for (int off = 1; off < 64; off <<= 1) cnt += __shfl_xor(cnt, off);
        if (lane == 0) ocnt[o * stride + blockIdx.x] = cnt;
    }
}

// One wavefront per tile: for every order p' = 0..10 the offsets whose
// mask has p', in order: ivlist[p' ntiles 189 + 189 t ..], ivcnt[p' ntiles + t]
__global__ __launch_bounds__(64) void k_class_lists(int ntiles, const uint16_t* __restrict__ omask,
                                                    int16_t* __restrict__ ivlist, int32_t* __restrict__ ivcnt) {
    const int tile = blockIdx.x;
    const int lane = threadIdx.x;
    for (int c = 0; c <= 10; ++c) {
        int16_t* out = ivlist + ((size_t)c * ntiles + tile) * 189;
        int cnt = 0;
        for (int b = 0; b < 189; b += 64) {
            const int iv = b + lane;
            const bool on = iv < 189 && ((omask[(size_t)tile * 189 + iv] >> c) & 1u);
            const unsigned long long bal = __ballot(on);
            if (on) out[cnt + __popcll(bal & ((1ull << lane) - 1ull))] = (int16_t)iv;
            cnt += __popcll(bal);
        }
        if (lane == 0) ivcnt[(size_t)c * ntiles + tile] = cnt;
    }
}

__global__ void k_fill0(long long n, double* __restrict__ a) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0.0;
}

void launch_m2l_orders(hipStream_t s, int tt, int ntiles, const int4* tiles, const int32_t* src_tab,
                       const int16_t* kslot, const int8_t* ordn, int8_t* ord_tab, uint16_t* omask, int32_t* ocnt) {
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(k_m2l_orders, dim3(189 * ntiles), dim3(64), 0, s, tt, tiles, src_tab, kslot, ordn, ord_tab,
                       omask, ocnt);
}

void launch_class_lists(hipStream_t s, int ntiles, const uint16_t* omask, int16_t* ivlist, int32_t* ivcnt) {
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(k_class_lists, dim3(ntiles), dim3(64), 0, s, ntiles, omask, ivlist, ivcnt);
}

void launch_fill0(hipStream_t s, long long n, double* a) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill0, dim3(cdiv(n, 256)), dim3(256), 0, s, n, a);
}

}  // namespace ctfmm
