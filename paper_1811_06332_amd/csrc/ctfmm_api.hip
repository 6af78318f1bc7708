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

constexpr int NPHASE_EV = 8 + 4 * (AMAX + 1);

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

    int16_t* alist = nullptr;      // [8][189] (q << 5 | u) per target octant, then [8][189] operator slots

    // adaptive tree workspace (every buffer grows on demand)
    ABox abox{};
    uint64_t* k64 = nullptr;
    uint64_t* k64s = nullptr;
    size_t k64_cap = 0, k64s_cap = 0;
    int32_t* a_idx = nullptr;
    int32_t* a_idxs = nullptr;
    int32_t* leaf_of = nullptr;
    size_t a_idx_cap = 0, a_idxs_cap = 0, leaf_of_cap = 0;
    double4* a_P = nullptr;
    double4* a_F = nullptr;  // far field per sorted particle
    size_t a_P_cap = 0, a_F_cap = 0;
    double* bbox = nullptr;  // [NBB][6] partial bounds, then lo[3], side
    ATree tr{};
    size_t ncap = 0;
    int nn = 0;
    int32_t* sflag = nullptr;
    int32_t* sincl = nullptr;
    int32_t* scstart = nullptr;
    size_t sflag_cap = 0, sincl_cap = 0, scstart_cap = 0;
    unsigned char* tmp = nullptr;
    size_t tmp_cap = 0;
    int32_t* lcnt = nullptr;  // [3][nn+1] U, W, X counts
    int32_t* loff = nullptr;  // [3][nn+1] exclusive scans
    size_t lcnt_cap = 0, loff_cap = 0;
    int32_t* ulist = nullptr;
    int32_t* wlist = nullptr;
    int32_t* xlist = nullptr;
    size_t ulist_cap = 0, wlist_cap = 0, xlist_cap = 0;
    uint32_t* lok = nullptr;
    uint32_t* loks = nullptr;
    int32_t* lov = nullptr;
    int32_t* lovs = nullptr;
    size_t lok_cap = 0, loks_cap = 0, lov_cap = 0, lovs_cap = 0;
    int32_t* bse = nullptr;  // [2][256] (level, octant) bucket bounds
    int4* tiles = nullptr;
    int32_t* tgt_tab = nullptr;
    int32_t* src_tab = nullptr;
    int32_t* vcount = nullptr;
    size_t tiles_cap = 0, tgt_cap = 0, src_cap = 0, vcount_cap = 0;
    int32_t* vsum = nullptr;
    double* aM = nullptr;
    double* aL = nullptr;
    double* aMh = nullptr;
    float* aM32 = nullptr;
    size_t aM_cap = 0, aL_cap = 0, aMh_cap = 0, aM32_cap = 0;
    std::vector<int> lev_first, lev_count, tile_first, tile_count;
    std::vector<int4> tiles_host;
    int64_t tot_u = 0, tot_w = 0, tot_x = 0, v_pairs = -1;
    long long* wcnt = nullptr;  // [nn+1] (target, W entry) pairs per node
    long long* wpoff = nullptr; // [nn+1] their exclusive scan
    double4* wbuf = nullptr;    // one contribution per pair
    size_t wcnt_cap = 0, wpoff_cap = 0, wbuf_cap = 0;
    long long wpairs = 0;

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

void dev_release(ctfmm_ctx* c, void* p) {
    if (!p) return;
    auto it = std::find(c->owned.begin(), c->owned.end(), p);
    if (it != c->owned.end()) c->owned.erase(it);
    if (c->ufree) {
        c->ufree(p, c->uuser, (void*)c->stream);  // stream-ordered
    } else {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(p);
    }
}

// grow a device array to at least `need` elements (by 1.5x or more); `keep`
// copies the old contents
template <class T>
bool grow(ctfmm_ctx* c, T*& ptr, size_t& cap, size_t need, bool keep) {
    if (ptr && need <= cap) return true;
    const size_t ncap = std::max<size_t>(std::max<size_t>(need, 1), cap + cap / 2);
    T* np = (T*)dev_alloc(c, ncap * sizeof(T));
    if (!np) return false;
    if (keep && ptr && cap) {
        if (hipMemcpyAsync(np, ptr, cap * sizeof(T), hipMemcpyDeviceToDevice, c->stream) != hipSuccess) return false;
    }
    dev_release(c, ptr);
    ptr = np;
    cap = ncap;
    return true;
}

void reset_adaptive(ctfmm_ctx* c) {
    // pointers only: the buffers themselves are released with the rest
    c->k64 = c->k64s = nullptr;
    c->k64_cap = c->k64s_cap = 0;
    c->a_idx = c->a_idxs = c->leaf_of = nullptr;
    c->a_idx_cap = c->a_idxs_cap = c->leaf_of_cap = 0;
    c->a_P = c->a_F = nullptr;
    c->a_P_cap = c->a_F_cap = 0;
    c->bbox = nullptr;
    c->tr = ATree{};
    c->ncap = 0;
    c->nn = 0;
    c->sflag = c->sincl = c->scstart = nullptr;
    c->sflag_cap = c->sincl_cap = c->scstart_cap = 0;
    c->tmp = nullptr;
    c->tmp_cap = 0;
    c->lcnt = c->loff = nullptr;
    c->lcnt_cap = c->loff_cap = 0;
    c->ulist = c->wlist = c->xlist = nullptr;
    c->ulist_cap = c->wlist_cap = c->xlist_cap = 0;
    c->lok = c->loks = nullptr;
    c->lov = c->lovs = nullptr;
    c->lok_cap = c->loks_cap = c->lov_cap = c->lovs_cap = 0;
    c->bse = nullptr;
    c->tiles = nullptr;
    c->tgt_tab = c->src_tab = c->vcount = nullptr;
    c->tiles_cap = c->tgt_cap = c->src_cap = c->vcount_cap = 0;
    c->vsum = nullptr;
    c->aM = c->aL = c->aMh = nullptr;
    c->aM32 = nullptr;
    c->aM_cap = c->aL_cap = c->aMh_cap = c->aM32_cap = 0;
    c->wcnt = c->wpoff = nullptr;
    c->wbuf = nullptr;
    c->wcnt_cap = c->wpoff_cap = c->wbuf_cap = 0;
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
    if (m2l_lds_bytes(p, prec) > (size_t)max_lds || m2l_tile_lds_bytes(p, prec) > (size_t)max_lds)
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
    {
        // source-octant-major order (the halo kernel, the adaptive tiles): entries (q << 5 | u), then the
        // operator slot of r = -v
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
        c->alist = (int16_t*)dev_alloc(c, hl.size() * sizeof(int16_t));
        if (!c->alist) return fail(c, CTFMM_ENOMEM, "operator allocation failed");
        HIPCHK(c, hipMemcpyAsync(c->alist, hl.data(), hl.size() * sizeof(int16_t), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (prec == CTFMM_PREC_FP32 && c->prm.tree == CTFMM_TREE_UNIFORM) off = hl;
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
                               (void*)c->alist, (void*)c->zero_row, (void*)c->err_flag};
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

// ------------------------------------------------------------------ adaptive tree

constexpr int NBB = 1024;  // blocks of the bounding-box reduction

bool grow_nodes(ctfmm_ctx* c, size_t need) {
    if (c->tr.key && need <= c->ncap) return true;
    const size_t ncap = std::max<size_t>(std::max<size_t>(need, 1024), c->ncap + c->ncap / 2);
    const size_t old = c->ncap;
    size_t k;
    k = old; if (!grow(c, c->tr.key, k, ncap, true)) return false;
    k = old; if (!grow(c, c->tr.pb, k, ncap, true)) return false;
    k = old; if (!grow(c, c->tr.pe, k, ncap, true)) return false;
    k = old; if (!grow(c, c->tr.par, k, ncap, true)) return false;
    k = old; if (!grow(c, c->tr.info, k, ncap, true)) return false;
    k = 8 * old; if (!grow(c, c->tr.child, k, 8 * ncap, true)) return false;
    k = 27 * old; if (!grow(c, c->tr.nb, k, 27 * ncap, true)) return false;
    c->ncap = ncap;
    return true;
}

// run a hipcub algorithm with the shared temporary buffer
template <class F>
ctfmm_status cub_run(ctfmm_ctx* c, F f) {
    size_t bytes = 0;
    HIPCHK(c, f(nullptr, bytes));
    if (!grow(c, c->tmp, c->tmp_cap, bytes, false)) return fail(c, CTFMM_ENOMEM, "workspace allocation failed");
    bytes = c->tmp_cap;
    HIPCHK(c, f((void*)c->tmp, bytes));
    return CTFMM_OK;
}

#define ACHK(expr)                                                                     \
    do {                                                                               \
        if (!(expr)) return fail(c, CTFMM_ENOMEM, "workspace allocation failed");      \
    } while (0)
#define SCHK(expr)                          \
    do {                                    \
        ctfmm_status s_ = (expr);           \
        if (s_ != CTFMM_OK) return s_;      \
    } while (0)

// keys, sort, the tree level by level, neighbour tables, U/W/X lists and the
// M2L tile tables.  Waits for the stream once per tree level and a few
// times more (sizes decide the next launches).
ctfmm_status build_adaptive(ctfmm_ctx* c, int n, const double* xyz, const double* q) {
    hipStream_t st = c->stream;
    const size_t nn_ = (size_t)n;
    ACHK(grow(c, c->k64, c->k64_cap, nn_, false));
    ACHK(grow(c, c->k64s, c->k64s_cap, nn_, false));
    ACHK(grow(c, c->a_idx, c->a_idx_cap, nn_, false));
    ACHK(grow(c, c->a_idxs, c->a_idxs_cap, nn_, false));
    ACHK(grow(c, c->leaf_of, c->leaf_of_cap, nn_, false));
    ACHK(grow(c, c->a_P, c->a_P_cap, nn_, false));
    ACHK(grow(c, c->a_F, c->a_F_cap, nn_, false));
    if (!c->bbox) {
        size_t cap = 0;
        ACHK(grow(c, c->bbox, cap, 6 * NBB + 4, false));
    }
    if (!c->bse) {
        size_t cap = 0;
        ACHK(grow(c, c->bse, cap, 512, false));
    }
    if (!c->vsum) {
        size_t cap = 0;
        ACHK(grow(c, c->vsum, cap, 1, false));
    }
    // root cube
    if (c->prm.root_side > 0.0) {
        c->abox = ABox{{c->prm.root_lo[0], c->prm.root_lo[1], c->prm.root_lo[2]}, c->prm.root_side};
    } else {
        const int nparts = std::min(NBB, std::max(1, (n + 255) / 256));
        launch_bbox(st, n, xyz, c->bbox, nparts, c->bbox + 6 * NBB);
        double hb[4];
        HIPCHK(c, hipMemcpyAsync(hb, c->bbox + 6 * NBB, sizeof(hb), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        if (!std::isfinite(hb[0]) || !std::isfinite(hb[1]) || !std::isfinite(hb[2]) || !std::isfinite(hb[3]))
            return fail(c, CTFMM_EINVAL, "non-finite particle coordinate");
        c->abox = ABox{{hb[0], hb[1], hb[2]}, hb[3]};
    }
    launch_keys64(st, n, xyz, c->abox, c->k64, c->a_idx, c->err_flag);
    SCHK(cub_run(c, [&](void* t, size_t& b) {
        return hipcub::DeviceRadixSort::SortPairs(t, b, c->k64, c->k64s, c->a_idx, c->a_idxs, n, 0, 3 * AMAX, st);
    }));
    launch_gather(st, n, c->a_idxs, xyz, q, c->a_P);
    HIPCHK(c, hipGetLastError());

    // tree, level by level
    ACHK(grow_nodes(c, 1));
    launch_root(st, n, c->tr);
    c->lev_first.assign(1, 0);
    c->lev_count.assign(1, 1);
    int first = 0, count = 1, total = 1;
    for (int l = 0;; ++l) {
        const size_t m = 8 * (size_t)count;
        ACHK(grow(c, c->sflag, c->sflag_cap, m, false));
        ACHK(grow(c, c->sincl, c->sincl_cap, m, false));
        ACHK(grow(c, c->scstart, c->scstart_cap, m, false));
        launch_split(st, l, first, count, c->prm.leaf_max, c->k64s, c->tr, c->sflag, c->scstart);
        SCHK(cub_run(c, [&](void* t, size_t& b) {
            return hipcub::DeviceScan::InclusiveSum(t, b, c->sflag, c->sincl, (int)m, st);
        }));
        int nnext = 0;
        HIPCHK(c, hipMemcpyAsync(&nnext, c->sincl + m - 1, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        if (nnext == 0) break;
        ACHK(grow_nodes(c, (size_t)total + nnext));
        launch_emit(st, l, first, count, total, c->sflag, c->sincl, c->scstart, c->tr);
        first = total;
        count = nnext;
        total += nnext;
        c->lev_first.push_back(first);
        c->lev_count.push_back(count);
    }
    HIPCHK(c, hipGetLastError());
    const int nn = total;
    c->nn = nn;
    const int maxlev = (int)c->lev_first.size() - 1;
    for (int l = 1; l <= maxlev; ++l) launch_nb(st, c->lev_first[l], c->lev_count[l], c->tr);
    launch_leaf_of(st, nn, c->tr, c->leaf_of);

    // U, W, X lists: count, scan, fill
    const size_t n1 = (size_t)nn + 1;
    ACHK(grow(c, c->lcnt, c->lcnt_cap, 3 * n1, false));
    ACHK(grow(c, c->loff, c->loff_cap, 3 * n1, false));
    int32_t *uc = c->lcnt, *wc = c->lcnt + n1, *xc = c->lcnt + 2 * n1;
    int32_t *uo = c->loff, *wo = c->loff + n1, *xo = c->loff + 2 * n1;
    HIPCHK(c, hipMemsetAsync(c->lcnt, 0, 3 * n1 * sizeof(int32_t), st));
    launch_lists(st, false, nn, c->tr, uc, wc, xc, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    for (int k = 0; k < 3; ++k) {
        int32_t* in = c->lcnt + k * n1;
        int32_t* out = c->loff + k * n1;
        SCHK(cub_run(c, [&](void* t, size_t& b) { return hipcub::DeviceScan::ExclusiveSum(t, b, in, out, (int)n1, st); }));
    }
    int tot[3];
    for (int k = 0; k < 3; ++k)
        HIPCHK(c, hipMemcpyAsync(&tot[k], c->loff + k * n1 + nn, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    c->tot_u = tot[0];
    c->tot_w = tot[1];
    c->tot_x = tot[2];
    ACHK(grow(c, c->ulist, c->ulist_cap, (size_t)tot[0], false));
    ACHK(grow(c, c->wlist, c->wlist_cap, (size_t)tot[1], false));
    ACHK(grow(c, c->xlist, c->xlist_cap, (size_t)tot[2], false));
    launch_lists(st, true, nn, c->tr, uc, wc, xc, uo, wo, xo, c->ulist, c->wlist, c->xlist);
    // (target particle, W entry) pairs of the multipole evaluations
    c->wpairs = 0;
    if (c->tot_w > 0) {
        ACHK(grow(c, c->wcnt, c->wcnt_cap, n1, false));
        ACHK(grow(c, c->wpoff, c->wpoff_cap, n1, false));
        HIPCHK(c, hipMemsetAsync(c->wcnt + nn, 0, sizeof(long long), st));
        launch_wpairs_count(st, nn, c->tr, wo, c->wcnt);
        SCHK(cub_run(c, [&](void* t, size_t& b) {
            return hipcub::DeviceScan::ExclusiveSum(t, b, c->wcnt, c->wpoff, (int)n1, st);
        }));
        long long wp = 0;
        HIPCHK(c, hipMemcpyAsync(&wp, c->wpoff + nn, sizeof(long long), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        c->wpairs = wp;
        ACHK(grow(c, c->wbuf, c->wbuf_cap, (size_t)wp, false));
    }

    // M2L tiles: nodes grouped by (level, octant), Morton order inside, 64 per tile
    ACHK(grow(c, c->lok, c->lok_cap, (size_t)nn, false));
    ACHK(grow(c, c->loks, c->loks_cap, (size_t)nn, false));
    ACHK(grow(c, c->lov, c->lov_cap, (size_t)nn, false));
    ACHK(grow(c, c->lovs, c->lovs_cap, (size_t)nn, false));
    launch_lvloct(st, nn, c->tr, c->lok, c->lov);
    SCHK(cub_run(c, [&](void* t, size_t& b) {
        return hipcub::DeviceRadixSort::SortPairs(t, b, c->lok, c->loks, c->lov, c->lovs, nn, 0, 8, st);
    }));
    launch_buckets(st, nn, c->loks, c->bse, c->bse + 256);
    int hb[512];
    HIPCHK(c, hipMemcpyAsync(hb, c->bse, sizeof(hb), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    c->tiles_host.clear();
    c->tile_first.assign(maxlev + 1, 0);
    c->tile_count.assign(maxlev + 1, 0);
    for (int l = 2; l <= maxlev; ++l) {
        c->tile_first[l] = (int)c->tiles_host.size();
        for (int o = 0; o < 8; ++o) {
            const int k = (l << 3) | o;
            const int b = hb[k], e = hb[256 + k];
            for (int s0 = b; s0 < e; s0 += 64) c->tiles_host.push_back(make_int4(o, s0, std::min(64, e - s0), l));
        }
        c->tile_count[l] = (int)c->tiles_host.size() - c->tile_first[l];
    }
    const size_t ntiles = c->tiles_host.size();
    if (ntiles) {
        ACHK(grow(c, c->tiles, c->tiles_cap, ntiles, false));
        ACHK(grow(c, c->tgt_tab, c->tgt_cap, 64 * ntiles, false));
        ACHK(grow(c, c->src_tab, c->src_cap, 189 * 64 * ntiles, false));
        ACHK(grow(c, c->vcount, c->vcount_cap, 189 * ntiles, false));
        HIPCHK(c, hipMemcpyAsync(c->tiles, c->tiles_host.data(), ntiles * sizeof(int4), hipMemcpyHostToDevice, st));
        launch_m2l_tables(st, (int)ntiles, c->tiles, c->lovs, c->tr, c->alist, c->tgt_tab, c->src_tab, c->vcount);
    }
    HIPCHK(c, hipGetLastError());
    c->v_pairs = -1;
    return CTFMM_OK;
}

// (target, source) pairs of the M2L tiles built last (waits for the stream)
ctfmm_status count_v_pairs(ctfmm_ctx* c) {
    if (c->v_pairs >= 0) return CTFMM_OK;
    const int m = 189 * (int)c->tiles_host.size();
    int v = 0;
    if (m > 0) {
        SCHK(cub_run(c, [&](void* t, size_t& b) {
            return hipcub::DeviceReduce::Sum(t, b, c->vcount, c->vsum, m, c->stream);
        }));
        HIPCHK(c, hipMemcpyAsync(&v, c->vsum, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    c->v_pairs = v;
    return CTFMM_OK;
}

ctfmm_status evaluate_adaptive(ctfmm_ctx* c, int n, const double* xyz, const double* q, double* phi,
                               double* grad) {
    hipStream_t st = c->stream;
    const int p = c->prm.order_p;
    const int prec = c->prm.precision;
    const size_t ldm = (size_t)ldm_of(p);
    // events: 0 start, 1 tree built, 2 P2M, 3 M2M, 4 conversions, 6-9 M2L / P2L / L2L, 5 before the near field
    rec(c, 0);
    HIPCHK(c, hipMemsetAsync(c->err_flag, 0, sizeof(int), st));
    SCHK(build_adaptive(c, n, xyz, q));
    rec(c, 1);
    const int nn = c->nn;
    const int maxlev = (int)c->lev_first.size() - 1;
    ACHK(grow(c, c->aM, c->aM_cap, (size_t)nn * ldm, false));
    ACHK(grow(c, c->aL, c->aL_cap, (size_t)nn * ldm, false));
    const ABox box = c->abox;
    launch_p2m_nodes(st, p, 0, nn, box, c->tr, c->a_P, c->T, c->aM);
    rec(c, 2);
    for (int l = maxlev - 1; l >= 2; --l) launch_m2m_nodes(st, p, c->lev_first[l], c->lev_count[l], c->tr, c->aM, c->T);
    rec(c, 3);
    const void* msrc = c->aM;
    if (maxlev >= 2) {
        const int f2 = c->lev_first[2];
        if (c->tot_w > 0) {
            ACHK(grow(c, c->aMh, c->aMh_cap, (size_t)nn * ldm, false));
            launch_mhat(st, p, f2, nn - f2, c->aM, c->aMh);
        }
        if (prec != CTFMM_PREC_FP64) {
            ACHK(grow(c, c->aM32, c->aM32_cap, (size_t)nn * s32_of(p), false));
            launch_to_f32(st, p, nn, c->aM, c->aM32);
            msrc = c->aM32;
        }
    }
    rec(c, 4);
    // downward: L(B) = M2L(V) + P2L(X) + L2L(parent).  M2L over the tiles of
    // every level at once (it reads only M), then the X lists, then L2L top-down.
    rec(c, 6);
    if (!c->tiles_host.empty()) {
        const AdaptM2L ad{c->tiles, c->tgt_tab, c->src_tab, c->alist + 8 * 189, 0};
        HIPCHK(c, launch_m2l_tables(st, p, prec, (int)c->tiles_host.size(), ad, msrc, c->aL, c->Kpk, c->zero_row));
    }
    rec(c, 7);
    if (c->tot_x > 0) launch_p2l(st, p, nn, box, c->tr, c->loff + 2 * ((size_t)nn + 1), c->xlist, c->a_P, c->aL);
    rec(c, 8);
    for (int l = 3; l <= maxlev; ++l)
        launch_l2l_nodes(st, p, c->lev_first[l - 1], c->lev_count[l - 1], c->tr, c->aL, c->T);
    rec(c, 9);
    rec(c, 5);
    const size_t n1 = (size_t)nn + 1;
    launch_near_adaptive(st, p, n, nn, c->wpairs, box, c->tr, c->leaf_of, c->a_P, c->aL, c->aMh, c->loff + n1,
                         c->wlist, c->wpoff, c->wbuf, c->loff, c->ulist, c->a_idxs, c->a_F, phi, grad);
    HIPCHK(c, hipGetLastError());
    const int ev_end = NPHASE_EV - 1;
    rec(c, ev_end);
    c->have_result = true;
    c->st.evaluations += 1;
    c->st.m2l_launches += c->tiles_host.empty() ? 0 : 1;
    c->st.p2p_leaf_pairs += c->tot_u;
    if (c->timing) {
        SCHK(count_v_pairs(c));
        c->st.m2l_pairs += c->v_pairs;
        HIPCHK(c, hipEventSynchronize(c->ev[ev_end]));
        c->st.ms_total += elapsed(c, 0, ev_end);
        c->st.ms_tree += elapsed(c, 0, 1);
        c->st.ms_p2m += elapsed(c, 1, 2);
        c->st.ms_m2m += elapsed(c, 2, 3);
        c->st.ms_convert += elapsed(c, 3, 4);
        c->st.ms_near += elapsed(c, 5, ev_end);
        c->st.ms_m2l += elapsed(c, 6, 7);
        c->st.ms_p2l += elapsed(c, 7, 8);
        c->st.ms_l2l += elapsed(c, 8, 9);
    }
    return CTFMM_OK;
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
    prm->leaf_max = 64;
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
    if (prm->tree != CTFMM_TREE_UNIFORM && prm->tree != CTFMM_TREE_ADAPTIVE) {
        g_create_err = "unknown tree type";
        return CTFMM_EUNSUPPORTED;
    }
    const bool adaptive = prm->tree == CTFMM_TREE_ADAPTIVE;
    const bool box_ok = std::isfinite(prm->root_side) && std::isfinite(prm->root_lo[0]) &&
                        std::isfinite(prm->root_lo[1]) && std::isfinite(prm->root_lo[2]) &&
                        (adaptive || prm->root_side > 0.0);
    if (prm->order_p < 0 || prm->order_p > CTFMM_P_MAX || prm->ws != 1 || !box_ok ||
        (!adaptive && (prm->depth < 0 || prm->depth > CTFMM_DEPTH_MAX)) || (adaptive && prm->leaf_max < 1)) {
        g_create_err = "invalid parameters (p in 0..10, ws == 1, finite root box; uniform: depth in 0..9, "
                       "root_side > 0; adaptive: leaf_max >= 1)";
        return CTFMM_EINVAL;
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
    reset_adaptive(c);
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
    if (c->prm.tree == CTFMM_TREE_ADAPTIVE) return evaluate_adaptive(c, (int)n, xyz, q, phi, grad);
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
    if (c->prm.tree != CTFMM_TREE_UNIFORM) return fail(c, CTFMM_EUNSUPPORTED, "expansion copies need the uniform tree");
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

ctfmm_status ctfmm_tree_stats(ctfmm_ctx* c, ctfmm_tree_stats_t* out) {
    if (!c || !out) return CTFMM_EINVAL;
    if (!c->have_result) return fail(c, CTFMM_EINVAL, "no evaluate yet");
    std::memset(out, 0, sizeof(*out));
    if (c->prm.tree == CTFMM_TREE_UNIFORM) {
        const int d = c->prm.depth;
        for (int l = 0; l <= d; ++l) out->nodes += 1ll << (3 * l);
        out->leaves = 1ll << (3 * d);
        out->max_level = d;
        for (int l = 2; l <= d; ++l) out->v_pairs += m2l_pairs_level(l);
        out->u_pairs = near_pairs(d);
        for (int k = 0; k < 3; ++k) out->root_lo[k] = c->prm.root_lo[k];
        out->root_side = c->prm.root_side;
        return CTFMM_OK;
    }
    ctfmm_status s = count_v_pairs(c);
    if (s != CTFMM_OK) return s;
    std::vector<int32_t> info((size_t)c->nn);
    HIPCHK(c, hipMemcpyAsync(info.data(), c->tr.info, info.size() * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int32_t v : info) out->leaves += (v >> 8) & 1;
    out->nodes = c->nn;
    out->max_level = (int64_t)c->lev_first.size() - 1;
    out->v_pairs = c->v_pairs;
    out->u_pairs = c->tot_u;
    out->w_pairs = c->tot_w;
    out->x_pairs = c->tot_x;
    for (int k = 0; k < 3; ++k) out->root_lo[k] = c->abox.lo[k];
    out->root_side = c->abox.side;
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
