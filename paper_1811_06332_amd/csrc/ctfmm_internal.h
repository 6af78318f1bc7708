// Internal declarations shared by the kernels and the host side of libctfmm.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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

// ---- launchers (ctfmm_kernels.hip); every one enqueues on `s` ----
void launch_keys(hipStream_t s, int n, const double* xyz, Box box, uint32_t* keys, int32_t* idx, int* err);
void launch_gather(hipStream_t s, int n, const int32_t* idx, const double* xyz, const double* q, double4* P);
void launch_leaf_start(hipStream_t s, int nleaves, const uint32_t* keys, int n, int32_t* start);
void launch_p2m(hipStream_t s, int p, Box box, const int32_t* start, const double4* P, const DevTables& T, double* M);
void launch_m2m(hipStream_t s, int p, int parent_level, const double* Mchild, double* Mparent, const DevTables& T);
void launch_offset_dtensors(hipStream_t s, int p, double* Dv);
void launch_build_k(hipStream_t s, int p, const double* Dv, const DevTables& T, double* Kt);
void launch_l2l(hipStream_t s, int p, int parent_level, const double* Lparent, double* Lchild, const DevTables& T);
void launch_l2p(hipStream_t s, int p, int n, Box box, const uint32_t* keys, const double4* P, const double* L,
                double4* F);
void launch_p2p(hipStream_t s, int n, Box box, const uint32_t* keys, const int32_t* start, const double4* P,
                const int32_t* idx, const double4* F, double* phi, double* grad);
// M2L operand precision (ctfmm_precision values)
enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16X3 = 2 };
size_t m2l_packed_bytes(int p, int prec);
size_t m2l_lds_bytes(int p, int prec);
void launch_pack_k(hipStream_t s, int p, int prec, const double* Kt, unsigned char* Kpk);
void launch_to_f32(hipStream_t s, int p, long long ncell, const double* M, float* M32);
hipError_t launch_m2l(hipStream_t s, int p, int prec, int level, const void* Msrc, double* L,
                      const unsigned char* Kpk, const int16_t* offlist, const unsigned char* zero_row);
// row stride of the FP32 multipole copy: (p+1)^2 rounded up to a multiple of 32
__host__ __device__ constexpr int s32_of(int p) { return (((p + 1) * (p + 1) + 31) / 32) * 32; }
void launch_unscale_copy(hipStream_t s, int p, int level, int which, double side, const double* X, double* out);

}  // namespace ctfmm
