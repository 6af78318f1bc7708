// Expansion-order selection of libctfmm (gfx950): the 12-64-64-9 network
// (ReLU after the hidden layers) that predicts, for a (source cell,
// separation) pair, log10 of the relative field error of M2L truncated at
// each order p' = 2..10; its training data generated from the method's own
// M2L and L2P; its forward pass (FP32, and FP16 on the matrix cores with
// FP32 accumulation), backward pass and Adam step; and the per-(cell,
// distance class) order decisions the adaptive M2L uses.
//
// Parameters: one flat FP32 array of MLP_NPARAM = 5577 values, W1[64][12],
// b1[64], W2[64][64], b2[64], W3[9][64], b3[9] (row-major, y = W x + b).
#include <math.h>

#include "ctfmm_internal.h"

namespace ctfmm {

namespace {

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

constexpr int OW1 = 0, OB1 = OW1 + MLP_NH * MLP_NIN, OW2 = OB1 + MLP_NH, OB2 = OW2 + MLP_NH * MLP_NH,
              OW3 = OB2 + MLP_NH, OB3 = OW3 + MLP_NOUT * MLP_NH;
static_assert(OB3 + MLP_NOUT == MLP_NPARAM, "parameter layout");

__device__ inline int rank_of_m(int k) {
    int r = 0;
    while ((r + 1) * (r + 1) <= k) ++r;
    return r;
}

}  // namespace

// ------------------------------------------------------------------ FP32 network

// y = network(x), one thread per sample, parameters staged in LDS
__global__ __launch_bounds__(256) void k_mlp_forward32(long long n, const float* __restrict__ x,
                                                       const float* __restrict__ prm, float* __restrict__ y) {
    __shared__ float w[MLP_NPARAM];
    for (int i = threadIdx.x; i < MLP_NPARAM; i += 256) w[i] = prm[i];
    __syncthreads();
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    float xi[MLP_NIN];
#pragma unroll
    for (int k = 0; k < MLP_NIN; ++k) xi[k] = x[b * MLP_NIN + k];
    float h1[MLP_NH];
#pragma unroll
    for (int j = 0; j < MLP_NH; ++j) {
        float z = w[OB1 + j];
#pragma unroll
        for (int k = 0; k < MLP_NIN; ++k) z += w[OW1 + j * MLP_NIN + k] * xi[k];
        h1[j] = z > 0.f ? z : 0.f;
    }
    float h2[MLP_NH];
    for (int j = 0; j < MLP_NH; ++j) {
        float z = w[OB2 + j];
#pragma unroll
        for (int k = 0; k < MLP_NH; ++k) z += w[OW2 + j * MLP_NH + k] * h1[k];
        h2[j] = z > 0.f ? z : 0.f;
    }
#pragma unroll
    for (int j = 0; j < MLP_NOUT; ++j) {
        float z = w[OB3 + j];
#pragma unroll
        for (int k = 0; k < MLP_NH; ++k) z += w[OW3 + j * MLP_NH + k] * h2[k];
        y[b * MLP_NOUT + j] = z;
    }
}

// Backward, stage 1 (one thread per sample): the forward pass again, then
// the per-sample quantities the weight gradients are sums of:
//   dy = 2 (y - t) / (9 n), dz2 = (W3^T dy) [z2 > 0], dz1 = (W2^T dz2) [z1 > 0]
// stored with h1, h2 in act[b][5 * 64] = (h1, h2, dz1, dz2, dy (9) + pad);
// err[b] = sum_k (y_k - t_k)^2.
__global__ __launch_bounds__(128) void k_mlp_back1(long long n, const float* __restrict__ x, const float* __restrict__ t,
                                                   const float* __restrict__ prm, float* __restrict__ act,
                                                   float* __restrict__ err) {
    __shared__ float w[MLP_NPARAM];
    for (int i = threadIdx.x; i < MLP_NPARAM; i += 128) w[i] = prm[i];
    __syncthreads();
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    float xi[MLP_NIN];
    for (int k = 0; k < MLP_NIN; ++k) xi[k] = x[b * MLP_NIN + k];
    float* a = act + b * (5 * MLP_NH);
    float h1[MLP_NH], h2[MLP_NH];
    for (int j = 0; j < MLP_NH; ++j) {
        float z = w[OB1 + j];
        for (int k = 0; k < MLP_NIN; ++k) z += w[OW1 + j * MLP_NIN + k] * xi[k];
        h1[j] = z > 0.f ? z : 0.f;
        a[j] = h1[j];
    }
    for (int j = 0; j < MLP_NH; ++j) {
        float z = w[OB2 + j];
        for (int k = 0; k < MLP_NH; ++k) z += w[OW2 + j * MLP_NH + k] * h1[k];
        h2[j] = z > 0.f ? z : 0.f;
        a[MLP_NH + j] = h2[j];
    }
    float dy[MLP_NOUT];
    float e = 0.f;
    const float scale = 2.f / (float)(MLP_NOUT * n);
    for (int j = 0; j < MLP_NOUT; ++j) {
        float z = w[OB3 + j];
        for (int k = 0; k < MLP_NH; ++k) z += w[OW3 + j * MLP_NH + k] * h2[k];
        const float d = z - t[b * MLP_NOUT + j];
        e += d * d;
        dy[j] = scale * d;
        a[4 * MLP_NH + j] = dy[j];
    }
    err[b] = e;
    float dz2[MLP_NH];
    for (int k = 0; k < MLP_NH; ++k) {
        float s = 0.f;
        for (int j = 0; j < MLP_NOUT; ++j) s += w[OW3 + j * MLP_NH + k] * dy[j];
        dz2[k] = h2[k] > 0.f ? s : 0.f;
        a[3 * MLP_NH + k] = dz2[k];
    }
    for (int k = 0; k < MLP_NH; ++k) {
        float s = 0.f;
        for (int j = 0; j < MLP_NH; ++j) s += w[OW2 + j * MLP_NH + k] * dz2[j];
        a[2 * MLP_NH + k] = h1[k] > 0.f ? s : 0.f;
    }
}

// Backward, stage 2: the per-sample terms summed over the samples in a
// fixed order (gW = dz^T h, gb = sum dz).  Block (64 parameters, chunk of
// 256 samples): four slices of the chunk per parameter, combined in LDS,
// give one partial sum per (chunk, parameter).
__device__ inline float grad_term(int i, long long b, const float* __restrict__ x, const float* __restrict__ act) {
    constexpr int A = 5 * MLP_NH;
    const float* a = act + b * A;
    if (i < OB1) return a[2 * MLP_NH + i / MLP_NIN] * x[b * MLP_NIN + i % MLP_NIN];
    if (i < OW2) return a[2 * MLP_NH + (i - OB1)];
    if (i < OB2) return a[3 * MLP_NH + (i - OW2) / MLP_NH] * a[(i - OW2) % MLP_NH];
    if (i < OW3) return a[3 * MLP_NH + (i - OB2)];
    if (i < OB3) return a[4 * MLP_NH + (i - OW3) / MLP_NH] * a[MLP_NH + (i - OW3) % MLP_NH];
    return a[4 * MLP_NH + (i - OB3)];
}

__global__ __launch_bounds__(256) void k_mlp_back2(long long n, const float* __restrict__ x,
                                                   const float* __restrict__ act, float* __restrict__ part) {
    const int pl = threadIdx.x & 63, sl = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + pl;
    const long long b0 = (long long)blockIdx.y * 256, b1 = min(n, b0 + 256);
    float s = 0.f;
    if (i < MLP_NPARAM)
        for (long long b = b0 + sl; b < b1; b += 4) s += grad_term(i, b, x, act);
    __shared__ float red[4][64];
    red[sl][pl] = s;
    __syncthreads();
    if (sl == 0 && i < MLP_NPARAM)
        part[(size_t)blockIdx.y * MLP_NPARAM + i] = (red[0][pl] + red[1][pl]) + (red[2][pl] + red[3][pl]);
}

// stage 3: gradient = sum of the chunk partials; thread MLP_NPARAM sums the loss
__global__ __launch_bounds__(256) void k_mlp_back3(long long n, int nchunk, const float* __restrict__ part,
                                                   const float* __restrict__ err, float* __restrict__ grad,
                                                   float* __restrict__ loss) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > MLP_NPARAM) return;
    float s = 0.f;
    if (i == MLP_NPARAM) {
        for (long long b = 0; b < n; ++b) s += err[b];
        *loss = s / (float)(MLP_NOUT * n);
        return;
    }
    for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * MLP_NPARAM + i];
    grad[i] = s;
}

// Adam (Kingma and Ba): m, v moments, bias-corrected step of size lr
__global__ void k_adam(int step, float lr, float* __restrict__ prm, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MLP_NPARAM) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.f - powf(b1, (float)step));
    const float vh = vi / (1.f - powf(b2, (float)step));
    prm[i] -= lr * mh / (sqrtf(vh) + eps);
}

void launch_mlp_forward32(hipStream_t s, long long n, const float* x, const float* prm, float* y) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mlp_forward32, dim3(cdiv(n, 256)), dim3(256), 0, s, n, x, prm, y);
}

// act needs n * 5 * 64 floats followed by mlp_backward_part_floats(n) more
size_t mlp_backward_part_floats(long long n) { return (size_t)cdiv(n, 256) * MLP_NPARAM; }

void launch_mlp_backward(hipStream_t s, long long n, const float* x, const float* t, const float* prm, float* act,
                         float* err, float* grad, float* loss) {
    if (n <= 0) return;
    const int nchunk = cdiv(n, 256);
    float* part = act + (size_t)n * 5 * MLP_NH;
    hipLaunchKernelGGL(k_mlp_back1, dim3(cdiv(n, 128)), dim3(128), 0, s, n, x, t, prm, act, err);
    hipLaunchKernelGGL(k_mlp_back2, dim3(cdiv(MLP_NPARAM, 64), nchunk), dim3(256), 0, s, n, x, act, part);
    hipLaunchKernelGGL(k_mlp_back3, dim3(cdiv(MLP_NPARAM + 1, 256)), dim3(256), 0, s, n, nchunk, part, err, grad, loss);
}

// ------------------------------------------------------------------ allocation-free backward pass
//
// Scratch of the backward pass for callers that cannot allocate: a
// file-scope device array, one copy per GPU, held until the process ends.
// Its device address is looked up once per device (with that device
// current) and only that address is ever handed to kernels or copies.
constexpr long long MLP_NOALLOC_MAX = 4096;  // samples per call
constexpr size_t MLP_NOALLOC_FLOATS =
    (size_t)MLP_NOALLOC_MAX * 5 * MLP_NH + (size_t)((MLP_NOALLOC_MAX + 255) / 256) * MLP_NPARAM + MLP_NOALLOC_MAX;
static __device__ __align__(256) float scratch[MLP_NOALLOC_FLOATS];

namespace {
constexpr int MAX_DEVICES = 64;
float* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

long long mlp_noalloc_max() { return MLP_NOALLOC_MAX; }

hipError_t mlp_noalloc_setup(int device) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    if (g_scratch_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<float*>(ptr);
    return hipSuccess;
}

hipError_t launch_mlp_backward_noalloc(hipStream_t s, int device, long long n, const float* x, const float* t,
                                       const float* prm, float* grad, float* loss) {
    if (device < 0 || device >= MAX_DEVICES || !g_scratch_ptr[device]) return hipErrorNotInitialized;
    if (n < 1 || n > MLP_NOALLOC_MAX) return hipErrorInvalidValue;
    float* act = g_scratch_ptr[device];  // [n][5*64], then the chunk partials
    float* err = act + (size_t)n * 5 * MLP_NH + mlp_backward_part_floats(n);
    launch_mlp_backward(s, n, x, t, prm, act, err, grad, loss);
    return hipGetLastError();
}

void launch_adam(hipStream_t s, int step, float lr, float* prm, const float* g, float* m, float* v) {
    hipLaunchKernelGGL(k_adam, dim3(cdiv(MLP_NPARAM, 256)), dim3(256), 0, s, step, lr, prm, g, m, v);
}

// ------------------------------------------------------------------ FP16 network on the matrix cores

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// Each wavefront takes blocks of 16 samples (block w, w + nwaves, ...).  Every
// layer is computed transposed, out^T = W in^T, with the 16x16x16 FP16 MFMA
// (FP32 accumulation): the A operand is a 16x16 block of W (row = output
// unit, k = input unit), the B operand a 16x16 block of in^T (k = input
// unit, column = sample).  The accumulator of output block jb holds
// out^T[16 jb + 4 (lane/16) + e][lane%16], which is exactly the B operand
// layout of input block jb of the next layer, so the activations never leave
// registers.  The weights' A blocks, the biases and the standardisation
// constants are loaded once per wavefront and kept in registers for all its
// blocks.  Inputs are standardised ((x - mean) / std) on load when norm is
// given.
__global__ __launch_bounds__(256) void k_mlp_forward16(long long n, const float* __restrict__ x,
                                                       const float* __restrict__ prm,
                                                       const float* __restrict__ norm, float* __restrict__ y) {
    const int lane = threadIdx.x & 63;
    const long long wave = (long long)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const long long nwaves = (long long)gridDim.x * (blockDim.x / 64);
    if (wave * 16 >= n) return;
    const int col = lane & 15, kq = lane >> 4;
    half4_t w1[4], w2[4][4], w3[4];
    float b1[4][4], b2[4][4], b3[4], mu[4], sd[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * kq + e;
            w1[jb][e] = (_Float16)(k < MLP_NIN ? prm[OW1 + (16 * jb + col) * MLP_NIN + k] : 0.f);
            b1[jb][e] = prm[OB1 + 16 * jb + 4 * kq + e];
            b2[jb][e] = prm[OB2 + 16 * jb + 4 * kq + e];
        }
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int e = 0; e < 4; ++e) w2[jb][kb][e] = (_Float16)prm[OW2 + (16 * jb + col) * MLP_NH + 16 * kb + 4 * kq + e];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            w3[kb][e] = (_Float16)(col < MLP_NOUT ? prm[OW3 + col * MLP_NH + 16 * kb + 4 * kq + e] : 0.f);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int j = 4 * kq + e, k = 4 * kq + e;
        b3[e] = j < MLP_NOUT ? prm[OB3 + j] : 0.f;
        mu[e] = (norm && k < MLP_NIN) ? norm[k] : 0.f;
        sd[e] = (norm && k < MLP_NIN) ? norm[MLP_NIN + k] : 1.f;
    }
    for (long long base = wave * 16; base < n; base += nwaves * 16) {
        const long long smp = base + col;
        const bool valid = smp < n;
        // layer 1: in^T block (k = 4 kq + e, inputs padded from 12 to 16)
        half4_t bx;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * kq + e;
            float v = 0.f;
            if (valid && k < MLP_NIN) {
                v = x[smp * MLP_NIN + k];
                if (norm) v = (v - mu[e]) / sd[e];
            }
            bx[e] = (_Float16)v;
        }
        half4_t h1[4];
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
            f4_t acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x16f16(w1[jb], bx, acc, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float z = acc[e] + b1[jb][e];
                h1[jb][e] = (_Float16)(z > 0.f ? z : 0.f);
            }
        }
        half4_t h2[4];
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
            f4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x16f16(w2[jb][kb], h1[kb], acc, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float z = acc[e] + b2[jb][e];
                h2[jb][e] = (_Float16)(z > 0.f ? z : 0.f);
            }
        }
        f4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) acc = __builtin_amdgcn_mfma_f32_16x16x16f16(w3[kb], h2[kb], acc, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 4 * kq + e;
            if (valid && j < MLP_NOUT) y[smp * MLP_NOUT + j] = acc[e] + b3[e];
        }
    }
}

void launch_mlp_forward16(hipStream_t s, long long n, const float* x, const float* prm, const float* norm, float* y) {
    if (n <= 0) return;
    // at most 4096 wavefronts (16 per CU), each looping over its blocks
    const long long blocks = (n + 15) / 16;
    const long long waves = blocks < 4096 ? blocks : 4096;
    hipLaunchKernelGGL(k_mlp_forward16, dim3(cdiv(waves, 4)), dim3(256), 0, s, n, x, prm, norm, y);
}

// ------------------------------------------------------------------ features and truncation labels

// The 12 network inputs of (source multipole, offset v): |v| / (sqrt(3)/2),
// then log10 of the 2-norm of each rank of the independent components
// relative to the largest rank norm (same definition for training and use).
__device__ inline void mlp_features(const double* __restrict__ Mt, int r2, float* f) {
    double nrm[11];
    double mx = 0.0;
    for (int r = 0; r <= 10; ++r) {
        double s = 0.0;
        for (int k = r * r; k < (r + 1) * (r + 1); ++k) s += Mt[k] * Mt[k];
        nrm[r] = sqrt(s);
        mx = fmax(mx, nrm[r]);
    }
    f[0] = (float)(sqrt((double)r2) / (sqrt(3.0) / 2.0));
    for (int r = 0; r <= 10; ++r) f[1 + r] = (float)(log10(nrm[r] + 1e-300) - log10(mx + 1e-300));
}

// One wavefront per sample: the source's order-10 scaled multipole (row
// sel[i] of M, or row i without sel; rows mstride doubles apart) and the
// offset slot vs of target - source.  The local
// expansions of M2L truncated at p' = 2..10 come from one pass over the
// order-10 operator K_v (Kt[vs][m][n] = K[n][m]) with the terms binned by
// rank(n) + rank(m); each is evaluated by L2P of order 10 at the eight
// points (+-3/8)^3 of the target cell; the label of p' is log10 of the
// relative 2-norm difference of (phi, grad phi) against order 10, floored
// at 1e-15.
__global__ __launch_bounds__(64) void k_mlp_labels(long long n, const double* __restrict__ M, long long mstride,
                                                   const int32_t* __restrict__ sel, const int32_t* __restrict__ vslot,
                                                   const double* __restrict__ Kt, float* __restrict__ xout,
                                                   float* __restrict__ yout) {
    constexpr int NC = 121;
    const long long smp = blockIdx.x;
    if (smp >= n) return;
    const int lane = threadIdx.x;
    const int vs = vslot[smp];
    const double* Mt = M + (sel ? (long long)sel[smp] : smp) * mstride;
    __shared__ double Ms[NC];
    __shared__ double Lp[9][NC + 1];
    __shared__ double Fv[9][8][4];
    for (int k = lane; k < NC; k += 64) Ms[k] = Mt[k];
    __syncthreads();
    // bins[s] of component n = lane + 64 c: sum over m with rank(n) + rank(m) = s
    for (int c = 0; c < 2; ++c) {
        const int nn = lane + 64 * c;
        if (nn >= NC) continue;
        const int rn = rank_of_m(nn);
        double bins[11];
#pragma unroll
        for (int s = 0; s <= 10; ++s) bins[s] = 0.0;
        const double* Kv = Kt + (size_t)vs * NC * NC;
        for (int m = 0; m < NC; ++m) {
            const int sidx = rn + rank_of_m(m);
            if (sidx <= 10) bins[sidx] += Kv[(size_t)m * NC + nn] * Ms[m];
        }
        double acc = 0.0;
        for (int s = 0; s <= 10; ++s) {
            acc += bins[s];
            if (s >= 2) Lp[s - 2][nn] = rn <= s ? acc : 0.0;
        }
    }
    __syncthreads();
    // fields: lanes over (order, point), 72 of them
    for (int w = lane; w < 72; w += 64) {
        const int pp = w / 8, pt = w % 8;
        const double ux = (pt & 1) ? 0.375 : -0.375, uy = (pt & 2) ? 0.375 : -0.375, uz = (pt & 4) ? 0.375 : -0.375;
        double f = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
        gen_l2p<10>(ux, uy, uz, &Lp[pp][0], f, gx, gy, gz);
        Fv[pp][pt][0] = f;
        Fv[pp][pt][1] = gx;
        Fv[pp][pt][2] = gy;
        Fv[pp][pt][3] = gz;
    }
    __syncthreads();
    if (lane < 9) {
        double d2 = 0.0, r2 = 0.0;
        for (int pt = 0; pt < 8; ++pt)
            for (int c = 0; c < 4; ++c) {
                const double d = Fv[lane][pt][c] - Fv[8][pt][c];
                d2 += d * d;
                r2 += Fv[8][pt][c] * Fv[8][pt][c];
            }
        const double e = sqrt(d2) / sqrt(r2);
        yout[smp * MLP_NOUT + lane] = (float)log10(fmax(e, 1e-15));
    }
    if (lane == 0) {
        const int vx = vs % 7 - 3, vy = (vs / 7) % 7 - 3, vz = vs / 49 - 3;
        float f[MLP_NIN];
        mlp_features(Ms, vx * vx + vy * vy + vz * vz, f);
        for (int k = 0; k < MLP_NIN; ++k) xout[smp * MLP_NIN + k] = f[k];
    }
}

void launch_mlp_labels(hipStream_t s, long long n, const double* M, long long mstride, const int32_t* sel,
                       const int32_t* vslot, const double* Kt, float* x, float* y) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mlp_labels, dim3((unsigned)n), dim3(64), 0, s, n, M, mstride, sel, vslot, Kt, x, y);
}

// counter-based hash (splitmix64 finaliser) for sampling
__device__ inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Training pairs from a tree: sample i takes node first + (h1 mod count) and
// the far offset h2 mod 316 (|v|_inf in {2, 3}), h = hashes of (seed, i).
// Writes the node rows into sel and the offset slots into vs.
__global__ void k_mlp_pick(long long n, unsigned long long seed, int first, int count, int32_t* __restrict__ sel,
                           int32_t* __restrict__ vs) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t h1 = mix64(seed * 0x100000001B3ull + 2 * (uint64_t)i);
    const uint64_t h2 = mix64(seed * 0x100000001B3ull + 2 * (uint64_t)i + 1);
    sel[i] = first + (int)(h1 % (uint64_t)count);
    int k = (int)(h2 % 316ull);
    // k-th slot of [-3,3]^3 with max |v_d| >= 2
    int slot = 0;
    for (int s = 0; s < NOFF; ++s) {
        const int vx = s % 7 - 3, vy = (s / 7) % 7 - 3, vz = s / 49 - 3;
        if (abs(vx) <= 1 && abs(vy) <= 1 && abs(vz) <= 1) continue;
        if (k-- == 0) {
            slot = s;
            break;
        }
    }
    vs[i] = slot;
}

void launch_mlp_pick(hipStream_t s, long long n, unsigned long long seed, int first, int count, int32_t* sel,
                     int32_t* vs) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mlp_pick, dim3(cdiv(n, 256)), dim3(256), 0, s, n, seed, first, count, sel, vs);
}

// rows sel of an order-10 expansion buffer (stride ldm) into a dense [n][121] array
__global__ void k_gather_rows(long long n, const int32_t* __restrict__ sel, const double* __restrict__ M, int ldm,
                              double* __restrict__ out) {
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n * 121) return;
    const long long i = g / 121;
    const int k = (int)(g % 121);
    out[g] = M[(size_t)sel[i] * ldm + k];
}

void launch_gather_rows(hipStream_t s, long long n, const int32_t* sel, const double* M, int ldm, double* out) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_rows, dim3(cdiv(n * 121, 256)), dim3(256), 0, s, n, sel, M, ldm, out);
}

// ------------------------------------------------------------------ order decisions

// distance class of |v|^2 for the 15 occupied values 4..27 (-1 elsewhere)
__device__ inline int class_of_r2(int r2) {
    switch (r2) {
        case 4: return 0;
        case 5: return 1;
        case 6: return 2;
        case 8: return 3;
        case 9: return 4;
        case 10: return 5;
        case 11: return 6;
        case 12: return 7;
        case 13: return 8;
        case 14: return 9;
        case 17: return 10;
        case 18: return 11;
        case 19: return 12;
        case 22: return 13;
        case 27: return 14;
        default: return -1;
    }
}

__device__ __constant__ int8_t kClassR2[NCLASS] = {4, 5, 6, 8, 9, 10, 11, 12, 13, 14, 17, 18, 19, 22, 27};

// Features of every (node, class) for nodes [first, first + count): row
// (node - first) * 15 + class of x.  M holds order-p scaled multipoles (p =
// 10 for a learned model: the features use ranks 0..10).
__global__ void k_mlp_node_features(int first, int count, const double* __restrict__ M, int ldm, float* __restrict__ x) {
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)count * NCLASS) return;
    const int node = first + (int)(g / NCLASS), cls = (int)(g % NCLASS);
    float f[MLP_NIN];
    mlp_features(M + (size_t)node * ldm, kClassR2[cls], f);
    for (int k = 0; k < MLP_NIN; ++k) x[g * MLP_NIN + k] = f[k];
}

// Decisions: the smallest p' whose predicted log10 error is at most thr,
// else 10 (the fixed order is the fallback); ord[node * 15 + class].
__global__ void k_mlp_decide(int first, int count, const float* __restrict__ y, float thr, int8_t* __restrict__ ord) {
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)count * NCLASS) return;
    int o = 10;
    for (int k = 0; k < MLP_NOUT; ++k)
        if (y[g * MLP_NOUT + k] <= thr) {
            o = k + 2;
            break;
        }
    ord[(size_t)first * NCLASS + g] = (int8_t)o;
}

// Orders from a fixed table by |v|^2 (the same for every node)
__global__ void k_order_table(int count, const int32_t* __restrict__ tab, int8_t* __restrict__ ord) {
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)count * NCLASS) return;
    ord[g] = (int8_t)tab[kClassR2[g % NCLASS]];
}

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): the increment, then the two xor-shift-multiply
// rounds and the final xor-shift of its output function.
__device__ inline uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Reproducible orders per (source cell, distance class): pmin + h mod (p -
// pmin + 1), h = SplitMix64 chained over (seed ^ cell key), the cell's level,
// and 16 * its system + the class.
__global__ void k_order_hash(int count, ATree t, unsigned long long seed, int pmin, int p, int8_t* __restrict__ ord) {
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)count * NCLASS) return;
    const int node = (int)(g / NCLASS), cls = (int)(g % NCLASS);
    uint64_t z = splitmix64(seed ^ t.key[node]);
    z = splitmix64(z ^ (uint64_t)(t.info[node] & 0xff));
    z = splitmix64(z ^ (uint64_t)(16 * t.sys[node] + cls));
    ord[g] = (int8_t)(pmin + (int)(z % (uint64_t)(p - pmin + 1)));
}

void launch_order_hash(hipStream_t s, int count, const ATree& t, unsigned long long seed, int pmin, int p,
                       int8_t* ord) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_order_hash, dim3(cdiv((long long)count * NCLASS, 256)), dim3(256), 0, s, count, t, seed, pmin,
                       p, ord);
}

void launch_mlp_node_features(hipStream_t s, int first, int count, const double* M, int ldm, float* x) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_mlp_node_features, dim3(cdiv((long long)count * NCLASS, 128)), dim3(128), 0, s, first, count,
                       M, ldm, x);
}

void launch_mlp_decide(hipStream_t s, int first, int count, const float* y, float thr, int8_t* ord) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_mlp_decide, dim3(cdiv((long long)count * NCLASS, 256)), dim3(256), 0, s, first, count, y, thr,
                       ord);
}

void launch_order_table(hipStream_t s, int count, const int32_t* tab, int8_t* ord) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_order_table, dim3(cdiv((long long)count * NCLASS, 256)), dim3(256), 0, s, count, tab, ord);
}

}  // namespace ctfmm
