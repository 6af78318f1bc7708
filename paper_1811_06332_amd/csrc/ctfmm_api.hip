// Host side of libctfmm: context, workspace, operator tables and the C ABI
// declared in include/ctfmm.h.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ctfmm.h"
#include "ctfmm_internal.h"

using namespace ctfmm;

namespace {

constexpr int NPHASE_EV = 8 + 4 * (CTFMM_DEPTH_MAX + 1);

}  // namespace

struct ctfmm_ctx {
    ctfmm_params prm{};
    hipStream_t stream = nullptr;
    int device = 0;
    ctfmm_alloc_fn ualloc = nullptr;
    ctfmm_free_fn ufree = nullptr;
    void* uuser = nullptr;
    std::string err;

    // operator tables and per-offset M2L matrices (built once)
    void* tab_blob = nullptr;
    DevTables T{};
    double* Dv = nullptr;  // [NOFF][NIND] derivative tensors of the offsets
    double* Kt = nullptr;  // [NOFF][nc][nc] K_v transposed
    unsigned char* Kpk = nullptr;  // K_v as MFMA A-fragments of the M2L precision
    int16_t* offlist = nullptr;    // [8][189] offset slots of each target octant
    unsigned char* zero_row = nullptr;  // a zero source row (out-of-domain sources)
    float* M32 = nullptr;          // FP32 copy of one level's multipoles (FP32/BF16 modes)

    // workspace, grown on demand
    int64_t cap_n = -1;
    uint32_t* keys = nullptr;
    uint32_t* keys_sorted = nullptr;
    int32_t* idx = nullptr;
    int32_t* idx_sorted = nullptr;
    double4* P = nullptr;
    double4* F = nullptr;  // far field per sorted particle (phi, grad)
    int32_t* start = nullptr;
    void* sort_tmp = nullptr;
    size_t sort_tmp_bytes = 0;
    double* M = nullptr;
    double* L = nullptr;
    size_t lvl_off[CTFMM_DEPTH_MAX + 2] = {};
    int* err_flag = nullptr;
    bool have_result = false;

    // timing
    bool timing = false;
    hipEvent_t ev[NPHASE_EV] = {};
    ctfmm_stats_t st{};

    std::vector<void*> owned;  // every workspace allocation (released on destroy)
};

namespace {

ctfmm_status fail(ctfmm_ctx* c, ctfmm_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

thread_local std::string g_create_err;

#define HIPCHK(ctx, call)                                                                             \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess)                                                                         \
            return fail(ctx, CTFMM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));       \
    } while (0)

void* dev_alloc(ctfmm_ctx* c, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    if (c->ualloc) {
        p = c->ualloc(bytes, c->uuser, (void*)c->stream);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) c->owned.push_back(p);
    return p;
}

void dev_free_all(ctfmm_ctx* c) {
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (void* p : c->owned) {
        if (c->ufree) c->ufree(p, c->uuser, (void*)c->stream);
        else (void)hipFree(p);
    }
    c->owned.clear();
}

template <class Tp>
size_t put(std::vector<unsigned char>& blob, const Tp* src, size_t count) {
    size_t off = (blob.size() + 255) & ~size_t(255);
    blob.resize(off + count * sizeof(Tp));
    std::memcpy(blob.data() + off, src, count * sizeof(Tp));
    return off;
}

ctfmm_status upload_tables(ctfmm_ctx* c) {
    std::vector<unsigned char> blob;
    std::vector<double> m2m_t((size_t)8 * NIND * NIND), l2l_t((size_t)8 * NIND * NIND);
    for (int o = 0; o < 8; ++o)
        for (int n = 0; n < NIND; ++n)
            for (int j = 0; j < NIND; ++j) {
                m2m_t[((size_t)o * NIND + j) * NIND + n] = GEN_M2M[o][n][j];
                l2l_t[((size_t)o * NIND + j) * NIND + n] = GEN_L2L[o][n][j];
            }
    const size_t o_ind = put(blob, &GEN_IND[0][0], (size_t)NIND * 3);
    const size_t o_full = put(blob, &GEN_FULL[0][0], (size_t)NFULL * 3);
    const size_t o_imf = put(blob, GEN_INV_MFACT, (size_t)NFULL);
    const size_t o_es = put(blob, GEN_EXP_START, sizeof(GEN_EXP_START) / sizeof(GEN_EXP_START[0]));
    const size_t o_esl = put(blob, GEN_EXP_SLOT, sizeof(GEN_EXP_SLOT));
    const size_t o_ec = put(blob, GEN_EXP_COEF, sizeof(GEN_EXP_COEF) / sizeof(GEN_EXP_COEF[0]));
    const size_t o_ps = put(blob, GEN_P2M_START, sizeof(GEN_P2M_START) / sizeof(GEN_P2M_START[0]));
    const size_t o_pc = put(blob, GEN_P2M_COEF, sizeof(GEN_P2M_COEF) / sizeof(GEN_P2M_COEF[0]));
    const size_t o_pe = put(blob, &GEN_P2M_EXP[0][0], sizeof(GEN_P2M_EXP));
    const size_t o_m2m = put(blob, m2m_t.data(), m2m_t.size());
    const size_t o_l2l = put(blob, l2l_t.data(), l2l_t.size());
    const size_t o_cs = put(blob, &GEN_C_START[0][0], (size_t)NIND * NIND);
    const size_t o_cn = put(blob, &GEN_C_COUNT[0][0], (size_t)NIND * NIND);
    const size_t o_csl = put(blob, GEN_C_SLOT, sizeof(GEN_C_SLOT));
    const size_t o_cc = put(blob, GEN_C_COEF, sizeof(GEN_C_COEF) / sizeof(GEN_C_COEF[0]));
    const size_t o_ds = put(blob, GEN_DET_START, sizeof(GEN_DET_START) / sizeof(GEN_DET_START[0]));
    const size_t o_df = put(blob, GEN_DET_FULL, sizeof(GEN_DET_FULL) / sizeof(GEN_DET_FULL[0]));
    const size_t o_dc = put(blob, GEN_DET_COEF, sizeof(GEN_DET_COEF) / sizeof(GEN_DET_COEF[0]));
    void* d = dev_alloc(c, blob.size());
    if (!d) return fail(c, CTFMM_ENOMEM, "table allocation failed");
    HIPCHK(c, hipMemcpyAsync(d, blob.data(), blob.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    auto* b = (unsigned char*)d;
    c->tab_blob = d;
    c->T.ind = (const int8_t*)(b + o_ind);
    c->T.full = (const int8_t*)(b + o_full);
    c->T.inv_mfact = (const double*)(b + o_imf);
    c->T.exp_start = (const int16_t*)(b + o_es);
    c->T.exp_slot = (const uint8_t*)(b + o_esl);
    c->T.exp_coef = (const int32_t*)(b + o_ec);
    c->T.p2m_start = (const int16_t*)(b + o_ps);
    c->T.p2m_coef = (const double*)(b + o_pc);
    c->T.p2m_exp = (const int8_t*)(b + o_pe);
    c->T.m2m_t = (const double*)(b + o_m2m);
    c->T.l2l_t = (const double*)(b + o_l2l);
    c->T.c_start = (const int32_t*)(b + o_cs);
    c->T.c_count = (const uint8_t*)(b + o_cn);
    c->T.c_slot = (const uint8_t*)(b + o_csl);
    c->T.c_coef = (const double*)(b + o_cc);
    c->T.det_start = (const int16_t*)(b + o_ds);
    c->T.det_full = (const int16_t*)(b + o_df);
    c->T.det_coef = (const double*)(b + o_dc);
    return CTFMM_OK;
}

ctfmm_status build_operators(ctfmm_ctx* c) {
    const int p = c->prm.order_p;
    const size_t nc = (size_t)(p + 1) * (p + 1);
    c->Dv = (double*)dev_alloc(c, (size_t)NOFF * NIND * sizeof(double));
    c->Kt = (double*)dev_alloc(c, (size_t)NOFF * nc * nc * sizeof(double));
    if (!c->Dv || !c->Kt) return fail(c, CTFMM_ENOMEM, "operator allocation failed");
    launch_offset_dtensors(c->stream, p, c->Dv);
    HIPCHK(c, hipGetLastError());
    launch_build_k(c->stream, p, c->Dv, c->T, c->Kt);
    HIPCHK(c, hipGetLastError());
    // MFMA fragments of every K_v in the M2L precision
    const int prec = c->prm.precision;
    int max_lds = 0;
    HIPCHK(c, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
    if (m2l_lds_bytes(p, prec) > (size_t)max_lds)
        return fail(c, CTFMM_EUNSUPPORTED, "device LDS per workgroup too small for the M2L tile");
    c->Kpk = (unsigned char*)dev_alloc(c, m2l_packed_bytes(p, prec));
    const size_t zbytes = std::max((size_t)ldm_of(p) * 8, (size_t)s32_of(p) * 4);
    c->zero_row = (unsigned char*)dev_alloc(c, zbytes);
    if (!c->Kpk || !c->zero_row) return fail(c, CTFMM_ENOMEM, "operator allocation failed");
    HIPCHK(c, hipMemsetAsync(c->zero_row, 0, zbytes, c->stream));
    launch_pack_k(c->stream, p, prec, c->Kt, c->Kpk);
    HIPCHK(c, hipGetLastError());
    // offsets v of the ws=1 list for a target in octant o: v_d in [-2-o_d, 3-o_d], max|v_d| >= 2
    std::vector<int16_t> off(8 * 189);
    for (int o = 0; o < 8; ++o) {
        int k = 0;
        const int ox = o & 1, oy = (o >> 1) & 1, oz = (o >> 2) & 1;
        for (int vz = -2 - oz; vz <= 3 - oz; ++vz)
            for (int vy = -2 - oy; vy <= 3 - oy; ++vy)
                for (int vx = -2 - ox; vx <= 3 - ox; ++vx) {
                    if (std::abs(vx) <= 1 && std::abs(vy) <= 1 && std::abs(vz) <= 1) continue;
                    off[o * 189 + k++] = (int16_t)((vx + 3) + 7 * (vy + 3) + 49 * (vz + 3));
                }
        if (k != 189) return fail(c, CTFMM_EDEVICE, "offset list construction");
    }
    if (prec == CTFMM_PREC_FP32) {
        // source-octant-major order for the halo kernel: entries (q << 5 | u), then the K slot of r = -v
        std::vector<int16_t> hl(2 * 8 * 189);
        for (int o = 0; o < 8; ++o) {
            int k = 0;
            for (int q = 0; q < 8; ++q)
                for (int u = 0; u < 27; ++u) {
                    const int vx = 2 * (u % 3 - 1) + (q & 1) - (o & 1);
                    const int vy = 2 * ((u / 3) % 3 - 1) + ((q >> 1) & 1) - ((o >> 1) & 1);
                    const int vz = 2 * (u / 9 - 1) + ((q >> 2) & 1) - ((o >> 2) & 1);
                    if (std::abs(vx) <= 1 && std::abs(vy) <= 1 && std::abs(vz) <= 1) continue;
                    if (k >= 189) return fail(c, CTFMM_EDEVICE, "halo offset list construction");
                    hl[o * 189 + k] = (int16_t)((q << 5) | u);
                    hl[8 * 189 + o * 189 + k] = (int16_t)((NOFF - 1) - ((vx + 3) + 7 * (vy + 3) + 49 * (vz + 3)));
                    ++k;
                }
            if (k != 189) return fail(c, CTFMM_EDEVICE, "halo offset list construction");
        }
        off = hl;
    }
    c->offlist = (int16_t*)dev_alloc(c, off.size() * sizeof(int16_t));
    if (!c->offlist) return fail(c, CTFMM_ENOMEM, "operator allocation failed");
    HIPCHK(c, hipMemcpyAsync(c->offlist, off.data(), off.size() * sizeof(int16_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return CTFMM_OK;
}

ctfmm_status ensure_workspace(ctfmm_ctx* c, int64_t n) {
    if (n <= c->cap_n) return CTFMM_OK;
    // release the previous particle workspace (tables and operators are kept)
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<void*> keep = {c->tab_blob, (void*)c->Dv, (void*)c->Kt, (void*)c->Kpk, (void*)c->offlist,
                               (void*)c->zero_row, (void*)c->err_flag};
    std::vector<void*> rest;
    for (void* p : c->owned) {
        bool k = false;
        for (void* q : keep) k |= (p == q);
        if (!k) {
            if (c->ufree) c->ufree(p, c->uuser, (void*)c->stream);
            else (void)hipFree(p);
        } else {
            rest.push_back(p);
        }
    }
    c->owned = rest;
    c->cap_n = -1;
    const int d = c->prm.depth;
    const int p = c->prm.order_p;
    const size_t nc = (size_t)(p + 1) * (p + 1);
    const size_t nleaves = (size_t)1 << (3 * d);
    const size_t nn = (size_t)(n > 0 ? n : 1);
    c->keys = (uint32_t*)dev_alloc(c, nn * 4);
    c->keys_sorted = (uint32_t*)dev_alloc(c, nn * 4);
    c->idx = (int32_t*)dev_alloc(c, nn * 4);
    c->idx_sorted = (int32_t*)dev_alloc(c, nn * 4);
    c->P = (double4*)dev_alloc(c, nn * sizeof(double4));
    c->F = (double4*)dev_alloc(c, nn * sizeof(double4));
    c->start = (int32_t*)dev_alloc(c, (nleaves + 1) * 4);
    size_t cells = 0;
    for (int l = 0; l <= d; ++l) {
        c->lvl_off[l] = cells;
        cells += (size_t)1 << (3 * l);
    }
    c->lvl_off[d + 1] = cells;
    c->M = (double*)dev_alloc(c, cells * (size_t)ldm_of(p) * sizeof(double));
    c->L = (double*)dev_alloc(c, cells * (size_t)ldm_of(p) * sizeof(double));
    c->M32 = nullptr;
    if (c->prm.precision != CTFMM_PREC_FP64 && d >= 2) {
        c->M32 = (float*)dev_alloc(c, nleaves * (size_t)s32_of(p) * sizeof(float));
        if (!c->M32) return fail(c, CTFMM_ENOMEM, "workspace allocation failed");
    }
    c->sort_tmp_bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, c->sort_tmp_bytes, c->keys, c->keys_sorted, c->idx,
                                             c->idx_sorted, (int)nn, 0, d > 0 ? 3 * d : 1, c->stream);
    c->sort_tmp = dev_alloc(c, c->sort_tmp_bytes);
    if (!c->keys || !c->keys_sorted || !c->idx || !c->idx_sorted || !c->P || !c->F || !c->start || !c->M || !c->L ||
        !c->sort_tmp)
        return fail(c, CTFMM_ENOMEM, "workspace allocation failed");
    c->cap_n = n;
    return CTFMM_OK;
}

inline void rec(ctfmm_ctx* c, int i) {
    if (c->timing) (void)hipEventRecord(c->ev[i], c->stream);
}

float elapsed(ctfmm_ctx* c, int a, int b) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, c->ev[a], c->ev[b]);
    return ms;
}

// pairs per level of the ws=1 list on a full 2^l grid (for statistics)
int64_t m2l_pairs_level(int l) {
    const int64_t n1 = 1ll << l;
    int64_t tot1 = 0;  // per dimension: pairs (t, s) with parents adjacent, and the |t-s|<=1 count
    int64_t near1 = 0;
    for (int64_t t = 0; t < n1; ++t)
        for (int64_t s = 0; s < n1; ++s) {
            if (std::llabs((t >> 1) - (s >> 1)) <= 1) ++tot1;
            if (std::llabs(t - s) <= 1) ++near1;
        }
    return tot1 * tot1 * tot1 - near1 * near1 * near1;
}

int64_t near_pairs(int d) {
    const int64_t n1 = 1ll << d;
    int64_t a = 0;
    for (int64_t t = 0; t < n1; ++t)
        for (int64_t s = 0; s < n1; ++s)
            if (std::llabs(t - s) <= 1) ++a;
    return a * a * a;
}

}  // namespace

extern "C" {

int ctfmm_version(void) { return CTFMM_ABI_VERSION; }

ctfmm_status ctfmm_default_params(ctfmm_params* prm) {
    if (!prm) return CTFMM_EINVAL;
    std::memset(prm, 0, sizeof(*prm));
    prm->order_p = 4;
    prm->tree = CTFMM_TREE_UNIFORM;
    prm->depth = 3;
    prm->ws = 1;
    prm->precision = CTFMM_PREC_FP64;
    prm->root_side = 1.0;
    return CTFMM_OK;
}

ctfmm_status ctfmm_create(const ctfmm_params* prm, void* hip_stream, ctfmm_ctx** out) {
    g_create_err.clear();
    if (!prm || !out) {
        g_create_err = "null argument";
        return CTFMM_EINVAL;
    }
    *out = nullptr;
    if (prm->order_p < 0 || prm->order_p > CTFMM_P_MAX || prm->depth < 0 || prm->depth > CTFMM_DEPTH_MAX ||
        prm->ws != 1 || !(prm->root_side > 0.0) || !std::isfinite(prm->root_side) ||
        !std::isfinite(prm->root_lo[0]) || !std::isfinite(prm->root_lo[1]) || !std::isfinite(prm->root_lo[2])) {
        g_create_err = "invalid parameters (p in 0..10, depth in 0..9, ws == 1, finite root box)";
        return CTFMM_EINVAL;
    }
    if (prm->tree != CTFMM_TREE_UNIFORM) {
        g_create_err = "only the uniform octree is implemented";
        return CTFMM_EUNSUPPORTED;
    }
    if (prm->precision != CTFMM_PREC_FP64 && prm->precision != CTFMM_PREC_FP32 &&
        prm->precision != CTFMM_PREC_BF16X3) {
        g_create_err = "unknown precision mode";
        return CTFMM_EUNSUPPORTED;
    }
    ctfmm_ctx* c = new (std::nothrow) ctfmm_ctx();
    if (!c) return CTFMM_ENOMEM;
    c->prm = *prm;
    c->stream = (hipStream_t)hip_stream;
    (void)hipGetDevice(&c->device);
    ctfmm_status s = upload_tables(c);
    if (s == CTFMM_OK) {
        c->err_flag = (int*)dev_alloc(c, sizeof(int));
        if (!c->err_flag) s = fail(c, CTFMM_ENOMEM, "allocation failed");
    }
    if (s == CTFMM_OK) s = build_operators(c);
    if (s == CTFMM_OK) {
        for (auto& e : c->ev)
            if (hipEventCreate(&e) != hipSuccess) {
                s = fail(c, CTFMM_EDEVICE, "hipEventCreate failed");
                break;
            }
    }
    if (s != CTFMM_OK) {
        g_create_err = c->err;
        ctfmm_destroy(c);
        return s;
    }
    *out = c;
    return CTFMM_OK;
}

ctfmm_status ctfmm_set_allocator(ctfmm_ctx* c, ctfmm_alloc_fn alloc, ctfmm_free_fn free_fn, void* user) {
    if (!c) return CTFMM_EINVAL;
    if (alloc && !free_fn) return fail(c, CTFMM_EINVAL, "allocator needs a free function");
    // move everything to the new allocator: release, then rebuild tables/operators
    dev_free_all(c);
    c->cap_n = -1;
    c->have_result = false;
    c->ualloc = alloc;
    c->ufree = alloc ? free_fn : nullptr;
    c->uuser = user;
    ctfmm_status s = upload_tables(c);
    if (s != CTFMM_OK) return s;
    c->err_flag = (int*)dev_alloc(c, sizeof(int));
    if (!c->err_flag) return fail(c, CTFMM_ENOMEM, "allocation failed");
    return build_operators(c);
}

ctfmm_status ctfmm_evaluate(ctfmm_ctx* c, int64_t n, const double* xyz, const double* q, double* phi,
                            double* grad) {
    if (!c) return CTFMM_EINVAL;
    c->err.clear();
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(c, CTFMM_EINVAL, "n out of range");
    if (n == 0) return CTFMM_OK;
    if (!xyz || !q) return fail(c, CTFMM_EINVAL, "null xyz or q");
    ctfmm_status s = ensure_workspace(c, n);
    if (s != CTFMM_OK) return s;
    const int d = c->prm.depth;
    const int p = c->prm.order_p;
    const size_t nc = (size_t)(p + 1) * (p + 1);
    const int nleaves = 1 << (3 * d);
    Box box{{c->prm.root_lo[0], c->prm.root_lo[1], c->prm.root_lo[2]}, c->prm.root_side, d};
    hipStream_t st = c->stream;
    const int ni = (int)n;

    rec(c, 0);
    HIPCHK(c, hipMemsetAsync(c->err_flag, 0, sizeof(int), st));
    launch_keys(st, ni, xyz, box, c->keys, c->idx, c->err_flag);
    size_t tmpb = c->sort_tmp_bytes;
    HIPCHK(c, hipcub::DeviceRadixSort::SortPairs(c->sort_tmp, tmpb, c->keys, c->keys_sorted, c->idx,
                                                 c->idx_sorted, ni, 0, d > 0 ? 3 * d : 1, st));
    launch_gather(st, ni, c->idx_sorted, xyz, q, c->P);
    launch_leaf_start(st, nleaves, c->keys_sorted, ni, c->start);
    HIPCHK(c, hipGetLastError());
    rec(c, 1);
    const size_t ldm = (size_t)ldm_of(p);
    auto Ml = [&](int l) { return c->M + c->lvl_off[l] * ldm; };
    auto Ll = [&](int l) { return c->L + c->lvl_off[l] * ldm; };
    int evi = 5;
    if (d >= 2) {
        launch_p2m(st, p, box, c->start, c->P, c->T, Ml(d));
        rec(c, 2);
        for (int l = d; l >= 3; --l) launch_m2m(st, p, l - 1, Ml(l), Ml(l - 1), c->T);
        rec(c, 3);
        for (int l = 2; l <= d; ++l) {
            rec(c, evi);
            const void* msrc = Ml(l);
            if (c->prm.precision != CTFMM_PREC_FP64) {
                launch_to_f32(st, p, 1ll << (3 * l), Ml(l), c->M32);
                msrc = c->M32;
            }
            rec(c, evi + 1);
            HIPCHK(c, launch_m2l(st, p, c->prm.precision, l, msrc, Ll(l), c->Kpk, c->offlist, c->zero_row));
            rec(c, evi + 2);
            if (l >= 3) launch_l2l(st, p, l - 1, Ll(l - 1), Ll(l), c->T);
            rec(c, evi + 3);
            evi += 4;
        }
        rec(c, 4);
        launch_l2p(st, p, ni, box, c->keys_sorted, c->P, Ll(d), c->F);
        launch_p2p(st, ni, box, c->keys_sorted, c->start, c->P, c->idx_sorted, c->F, phi, grad);
    } else {
        rec(c, 2);
        rec(c, 3);
        rec(c, 4);
        launch_p2p(st, ni, box, c->keys_sorted, c->start, c->P, c->idx_sorted, nullptr, phi, grad);
    }
    HIPCHK(c, hipGetLastError());
    const int ev_end = NPHASE_EV - 1;
    rec(c, ev_end);
    c->have_result = true;
    c->st.evaluations += 1;
    for (int l = 2; l <= d; ++l) {
        c->st.m2l_launches += 1;
        c->st.m2l_pairs += m2l_pairs_level(l);
    }
    c->st.p2p_leaf_pairs += near_pairs(d);
    if (c->timing) {
        HIPCHK(c, hipEventSynchronize(c->ev[ev_end]));
        c->st.ms_total += elapsed(c, 0, ev_end);
        c->st.ms_tree += elapsed(c, 0, 1);
        c->st.ms_p2m += elapsed(c, 1, 2);
        c->st.ms_m2m += elapsed(c, 2, 3);
        c->st.ms_near += elapsed(c, 4, ev_end);
        int e = 5;
        for (int l = 2; l <= d; ++l) {
            c->st.ms_convert += elapsed(c, e, e + 1);
            c->st.ms_m2l += elapsed(c, e + 1, e + 2);
            c->st.ms_l2l += elapsed(c, e + 2, e + 3);
            e += 4;
        }
    }
    return CTFMM_OK;
}

ctfmm_status ctfmm_copy_expansions(ctfmm_ctx* c, int32_t level, int32_t which, double* host_out, size_t cap) {
    if (!c || !host_out) return CTFMM_EINVAL;
    const int p = c->prm.order_p;
    const size_t nc = (size_t)(p + 1) * (p + 1);
    if (!c->have_result) return fail(c, CTFMM_EINVAL, "no evaluate yet");
    if (level < 2 || level > c->prm.depth || (which != 0 && which != 1))
        return fail(c, CTFMM_EINVAL, "level must be in 2..depth and which 0 or 1");
    const size_t cnt = ((size_t)1 << (3 * level)) * nc;
    if (cap < cnt) return fail(c, CTFMM_EINVAL, "host buffer too small");
    double* tmp = nullptr;
    HIPCHK(c, hipMalloc(&tmp, cnt * sizeof(double)));
    const double* X = (which == 0 ? c->M : c->L) + c->lvl_off[level] * (size_t)ldm_of(p);
    launch_unscale_copy(c->stream, p, level, which, c->prm.root_side, X, tmp);
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipMemcpyAsync(host_out, tmp, cnt * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    hipError_t e3 = hipStreamSynchronize(c->stream);
    (void)hipFree(tmp);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) return fail(c, CTFMM_EDEVICE, "copy failed");
    return CTFMM_OK;
}

ctfmm_status ctfmm_set_timing(ctfmm_ctx* c, int32_t on) {
    if (!c) return CTFMM_EINVAL;
    c->timing = on != 0;
    return CTFMM_OK;
}

ctfmm_status ctfmm_stats(ctfmm_ctx* c, ctfmm_stats_t* out) {
    if (!c || !out) return CTFMM_EINVAL;
    *out = c->st;
    return CTFMM_OK;
}

ctfmm_status ctfmm_reset_stats(ctfmm_ctx* c) {
    if (!c) return CTFMM_EINVAL;
    std::memset(&c->st, 0, sizeof(c->st));
    return CTFMM_OK;
}

ctfmm_status ctfmm_sync(ctfmm_ctx* c) {
    if (!c) return CTFMM_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->err_flag) {
        int h = 0;
        HIPCHK(c, hipMemcpy(&h, c->err_flag, sizeof(int), hipMemcpyDeviceToHost));
        if (h) {
            HIPCHK(c, hipMemset(c->err_flag, 0, sizeof(int)));
            return fail(c, CTFMM_EINVAL, "non-finite particle coordinate");
        }
    }
    return CTFMM_OK;
}

const char* ctfmm_last_error(const ctfmm_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

void ctfmm_destroy(ctfmm_ctx* c) {
    if (!c) return;
    dev_free_all(c);
    for (auto& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"
