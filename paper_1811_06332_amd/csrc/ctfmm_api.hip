// Host side of libctfmm: context, workspace, operator tables and the C ABI
// declared in include/ctfmm.h.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <chrono>
#include <climits>
#include <cstring>
#include <new>
#include <string>
#include <array>
#include <vector>

#include "ctfmm.h"
#include "ctfmm_internal.h"

using namespace ctfmm;

namespace {

constexpr int NPHASE_EV = 8 + 4 * (AMAX + 1);

}  // namespace

// Operators of one expansion order in the context's M2L precision; Kmix
// (built when orders per pair are first used) holds the operators of every
// order q <= p in the order-p fragment layout, one set after the other.
struct OpSet {
    int p = -1;
    double* Dv = nullptr;
    double* Kt = nullptr;
    unsigned char* Kpk = nullptr;
    unsigned char* Kmix = nullptr;
};

// Workspace of one forest of adaptive trees (all systems of one order p);
// every device buffer grows on demand.
struct Forest {
    int p = 0;
    int nsys = 0;
    int n = 0;
    std::vector<int32_t> goff_h, gbase_h;
    int32_t* goff = nullptr;
    int32_t* gbase = nullptr;
    size_t goff_cap = 0, gbase_cap = 0;
    ABox* boxes = nullptr;
    size_t boxes_cap = 0;
    uint64_t* k64 = nullptr;
    uint64_t* k64s = nullptr;
    size_t k64_cap = 0, k64s_cap = 0;
    uint32_t* k32 = nullptr;   // top 32 key bits
    uint32_t* k32s = nullptr;
    int32_t* deep = nullptr;   // set when the tree goes deeper than the 32-bit sort orders
    size_t k32_cap = 0, k32s_cap = 0, deep_cap = 0;
    int32_t* a_idx = nullptr;
    int32_t* a_idxs = nullptr;
    int32_t* leaf_of = nullptr;
    size_t a_idx_cap = 0, a_idxs_cap = 0, leaf_of_cap = 0;
    double4* a_P = nullptr;
    double4* a_F = nullptr;   // far field per sorted particle
    double4* a_Fn = nullptr;  // near field per sorted particle
    size_t a_P_cap = 0, a_F_cap = 0, a_Fn_cap = 0;
    double* bbox = nullptr;  // [NBB][6] partial bounds, then lo[3], side
    size_t bbox_cap = 0;
    ATree tr{};
    size_t ncap = 0;
    int nn = 0;
    int32_t* sflag = nullptr;
    int32_t* sincl = nullptr;
    int32_t* scstart = nullptr;
    size_t sflag_cap = 0, sincl_cap = 0, scstart_cap = 0;
    int32_t* lcnt = nullptr;  // [7][nn+1]: own U, W, X, finer U counts, U totals, fill cursors
    int32_t* lsort = nullptr;  // sort output of the transposed list entries
    size_t lsort_cap = 0;
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
    size_t bse_cap = 0;
    int4* tiles = nullptr;
    int4* tiles_tmp = nullptr;   // tiles in bucket order, before the sort
    uint64_t* tkey = nullptr;    // [2][ntiles] tile sort keys
    int32_t* tidx = nullptr;     // [2][ntiles] tile sort values
    size_t tiles_tmp_cap = 0, tkey_cap = 0, tidx_cap = 0;
    int32_t* tgt_tab = nullptr;
    int32_t* src_tab = nullptr;
    int32_t* vcount = nullptr;
    size_t tiles_cap = 0, tgt_cap = 0, src_cap = 0, vcount_cap = 0;
    int32_t* vsum = nullptr;
    size_t vsum_cap = 0;
    double* aM = nullptr;
    double* aL = nullptr;
    double* aWc = nullptr;  // W-list polynomial coefficients [node][m2p_coef_ld(p)]
    float* aM32 = nullptr;
    size_t aM_cap = 0, aL_cap = 0, aWc_cap = 0, aM32_cap = 0;
    std::vector<int> lev_first, lev_count;
    std::vector<int4> tiles_host;
    int64_t tot_u = 0, tot_w = 0, tot_x = 0, v_pairs = -1;
    const unsigned char* Kpk = nullptr;  // operators of order p
    int tt = 64;                         // targets per M2L tile
    int hb[512] = {};                    // (level, octant) bucket bounds on the host
    // active offsets of every M2L tile: [ntiles][189] offsets and their
    // orders, [ntiles] counts
    int16_t* ivl = nullptr;
    int8_t* ivo = nullptr;
    int32_t* ivc = nullptr;
    size_t ivl_cap = 0, ivo_cap = 0, ivc_cap = 0;
    // M2L orders per pair
    int8_t* ordn = nullptr;      // [nn][15] order per (source node, distance class)
    int8_t* tq = nullptr;        // [ntiles][189] order of every (tile, offset), -1 = no pair
    int32_t* ocnt = nullptr;     // [11][ntiles * 189] pairs per order
    float* mx = nullptr;         // network inputs of (node, class)
    float* my = nullptr;         // network outputs
    size_t ordn_cap = 0, tq_cap = 0, ocnt_cap = 0, mx_cap = 0, my_cap = 0;
    const unsigned char* Kmix = nullptr;  // operators of every order <= p (order-p layout)
    int nchunk = 1;              // M2L workgroups per tile (offset chunks)
    bool up_early = false;       // P2M and M2M already launched by the tree build
    double* part = nullptr;      // [nchunk][nn][ldm] partial local expansions
    size_t part_cap = 0;
    // dual-tree traversal: centres and radii, round counters, frontiers, the
    // M2L and direct-pair keys (unsorted, sorted), their CSR forms
    double4* zr = nullptr;
    double4* zsum = nullptr;  // charge sums per node (charge-weighted centres)
    size_t zsum_cap = 0;
    int* dcnt = nullptr;
    int2* front[2] = {};
    uint64_t *mk = nullptr, *mks = nullptr, *pk = nullptr, *pks = nullptr;
    int32_t *moff = nullptr, *msrc = nullptr, *poff = nullptr, *psrc = nullptr;
    size_t zr_cap = 0, dcnt_cap = 0, front_cap[2] = {}, mk_cap = 0, mks_cap = 0, pk_cap = 0, pks_cap = 0;
    size_t moff_cap = 0, msrc_cap = 0, poff_cap = 0, psrc_cap = 0;
    size_t cap_f = 0, cap_m = 0, cap_p = 0;  // entries the traversal may write
    int n_m2l = 0, n_p2p = 0, dual_sh = 0;
};

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
    float* Kq = nullptr;           // FP32: the same, four chunks of a lane side by side
    unsigned char* Kmix = nullptr; // the operators of every order <= p (per-pair orders)
    int16_t* offlist = nullptr;    // [8][189] offset slots of each target octant
    unsigned char* zero_row = nullptr;  // a zero source row (out-of-domain sources)
    int* pinned = nullptr;              // pinned host words for small device-to-host reads
    int* pinned_dev = nullptr;          // their address for kernels
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

    // adaptive trees: operators of further orders, forests (one per order in a
    // batch; [0] for a single system), the shared hipcub scratch buffer and the
    // graph of the batched numeric passes
    std::vector<OpSet> opsets;
    std::vector<Forest> forests;
    int nforests = 0;
    unsigned char* tmp = nullptr;
    size_t tmp_cap = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream the graph is captured on
    hipStream_t side[2] = {};  // the near field (P2P) and the X lists (P2L) beside the expansion passes
    hipEvent_t side_ev[7] = {};
    // M2L order per pair (adaptive tree): 0 = the fixed order p, 1 = a table
    // by |v|^2, 2 = the network's decision per (source cell, distance class),
    // 3 = a reproducible hash of (source cell, distance class)
    int order_mode = 0;
    unsigned long long order_seed = 0;
    int order_pmin = 0;
    // dual-tree traversal: acceptance parameter and expansion centres
    double theta = 0.5;
    int centre = CTFMM_CENTRE_GEOMETRIC;
    int32_t* order_tab = nullptr;  // device [28]
    float* model = nullptr;        // device [MLP_NPARAM + 24]: parameters, input mean, input std
    float order_thr = 0.f;         // log10(target error) - margin
    // network training scratch
    float* mlp_act = nullptr;
    float* mlp_err = nullptr;
    float* mlp_grad = nullptr;
    float* mlp_m = nullptr;
    float* mlp_v = nullptr;
    float* mlp_loss = nullptr;
    size_t mlp_act_cap = 0, mlp_err_cap = 0, mlp_grad_cap = 0, mlp_m_cap = 0, mlp_v_cap = 0, mlp_loss_cap = 0;
    int32_t* mlp_sel = nullptr;
    int32_t* mlp_vs = nullptr;
    size_t mlp_sel_cap = 0, mlp_vs_cap = 0;
    int tile_forced[CTFMM_P_MAX + 1] = {};  // M2L targets per tile set by the caller (0 = tune)
    int tile_tuned[CTFMM_P_MAX + 1] = {};   // ... chosen by the tuner (0 = not yet)
    int chunk_tuned[CTFMM_P_MAX + 1] = {};  // M2L workgroups per tile chosen by the tuner (0 = the default rule)
    hipEvent_t tev[2] = {};                 // events of the tuner
    std::vector<long long> gsig;

    // timing
    bool timing = false;
    // phase events, two sets: an adaptive evaluation with fixed orders leaves
    // its timings pending in one set while the next evaluation records the other
    hipEvent_t evs[2][NPHASE_EV] = {};
    hipEvent_t* ev = evs[0];
    struct Pending {
        bool on = false;
        hipEvent_t* ev = nullptr;  // the event set of the pending evaluation
        int word = 0;              // pinned word with its M2L pair count
    } pend;
    ctfmm_stats_t st{};

    // point dipoles in sorted order (uniform tree, ctfmm_evaluate_dipoles)
    double4* Pd = nullptr;
    size_t Pd_cap = 0;
    // FP64 copies of the caller's arrays for the FP32 entry points: xyz, q, phi, grad
    double* io[4] = {};
    size_t io_cap[4] = {};

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
    c->opsets.clear();
    c->Kmix = nullptr;
    for (int k = 0; k < 4; ++k) {
        c->io[k] = nullptr;
        c->io_cap[k] = 0;
    }
    c->forests.clear();
    c->nforests = 0;
    c->tmp = nullptr;
    c->tmp_cap = 0;
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->gsig.clear();
    c->order_mode = 0;
    c->order_tab = nullptr;
    c->model = nullptr;
    c->mlp_act = c->mlp_err = c->mlp_grad = c->mlp_m = c->mlp_v = c->mlp_loss = nullptr;
    c->mlp_act_cap = c->mlp_err_cap = c->mlp_grad_cap = c->mlp_m_cap = c->mlp_v_cap = c->mlp_loss_cap = 0;
    c->mlp_sel = c->mlp_vs = nullptr;
    c->mlp_sel_cap = c->mlp_vs_cap = 0;
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
    if (m2l_lds_bytes(p, prec) > (size_t)max_lds || m2l_tile_lds_bytes(p, prec, 32) > (size_t)max_lds)
        return fail(c, CTFMM_EUNSUPPORTED, "device LDS per workgroup too small for the M2L tile");
    c->Kpk = (unsigned char*)dev_alloc(c, m2l_packed_bytes(p, prec));
    const size_t zbytes = std::max((size_t)ldm_of(PMAX) * 8, (size_t)s32_of(PMAX) * 4);
    c->zero_row = (unsigned char*)dev_alloc(c, zbytes);
    if (!c->Kpk || !c->zero_row) return fail(c, CTFMM_ENOMEM, "operator allocation failed");
    HIPCHK(c, hipMemsetAsync(c->zero_row, 0, zbytes, c->stream));
    launch_pack_k(c->stream, p, prec, c->Kt, c->Kpk, p);
    if (prec == CTFMM_PREC_FP32) {
        c->Kq = (float*)dev_alloc(c, m2l_quad_bytes(p));
        if (!c->Kq) return fail(c, CTFMM_ENOMEM, "operator allocation failed");
        launch_quad_k(c->stream, p, c->Kpk, c->Kq);
    }
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
    std::vector<void*> keep = {c->tab_blob,      (void*)c->Dv,       (void*)c->Kt,       (void*)c->Kpk,
                               (void*)c->offlist, (void*)c->alist,    (void*)c->zero_row, (void*)c->err_flag,
                               (void*)c->io[0],   (void*)c->io[1],    (void*)c->io[2],    (void*)c->io[3],
                               (void*)c->Kq};
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
    c->Pd = nullptr;  // released above with the particle workspace
    c->Pd_cap = 0;
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

float elapsed_in(hipEvent_t* ev, int a, int b) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[a], ev[b]);
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

bool grow_nodes(ctfmm_ctx* c, Forest& f, size_t need) {
    if (f.tr.key && need <= f.ncap) return true;
    const size_t ncap = std::max<size_t>(std::max<size_t>(need, 1024), f.ncap + f.ncap / 2);
    const size_t old = f.ncap;
    size_t k;
    k = old; if (!grow(c, f.tr.key, k, ncap, true)) return false;
    k = old; if (!grow(c, f.tr.pb, k, ncap, true)) return false;
    k = old; if (!grow(c, f.tr.pe, k, ncap, true)) return false;
    k = old; if (!grow(c, f.tr.par, k, ncap, true)) return false;
    k = old; if (!grow(c, f.tr.info, k, ncap, true)) return false;
    k = old; if (!grow(c, f.tr.sys, k, ncap, true)) return false;
    k = 8 * old; if (!grow(c, f.tr.child, k, 8 * ncap, true)) return false;
    k = 27 * old; if (!grow(c, f.tr.nb, k, 27 * ncap, true)) return false;
    k = old; if (!grow(c, f.tr.geo, k, ncap, true)) return false;
    f.ncap = ncap;
    return true;
}

// the pinned host words (at least 1024), allocated on first use
int* pinned_words(ctfmm_ctx* c) {
    if (!c->pinned) {
        if (hipHostMalloc((void**)&c->pinned, 1024 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
            c->pinned = nullptr;
        } else if (hipHostGetDevicePointer((void**)&c->pinned_dev, c->pinned, 0) != hipSuccess) {
            (void)hipHostFree(c->pinned);
            c->pinned = nullptr;
            c->pinned_dev = nullptr;
        }
    }
    return c->pinned;
}

// Small device-to-host reads of non-negative words.  arm() sets the first
// count pinned words to a sentinel before the copies into them are enqueued;
// wait_words() then spins until the copies have written every word, which
// comes back sooner than a stream synchronisation.  After a bounded spin it
// falls back to the synchronisation (which also returns any device error).
constexpr int WORD_UNSET = INT_MIN;
void arm_words(int* pw, int count) {
    for (int k = 0; k < count; ++k) reinterpret_cast<volatile int*>(pw)[k] = WORD_UNSET;
}
ctfmm_status wait_words(ctfmm_ctx* c, const int* pw, int count) {
    const volatile int* v = pw;
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        int k = 0;
        while (k < count && v[k] != WORD_UNSET) ++k;
        if (k == count) return CTFMM_OK;
        if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(200)) break;
        __builtin_ia32_pause();
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < count; ++k)
        if (v[k] == WORD_UNSET) return fail(c, CTFMM_EDEVICE, "device-to-host read did not arrive");
    return CTFMM_OK;
}

// run a hipcub algorithm with the shared temporary buffer
template <class F>
ctfmm_status cub_run(ctfmm_ctx* c, F fn) {
    size_t bytes = 0;
    HIPCHK(c, fn(nullptr, bytes));
    if (!grow(c, c->tmp, c->tmp_cap, bytes, false)) return fail(c, CTFMM_ENOMEM, "workspace allocation failed");
    bytes = c->tmp_cap;
    HIPCHK(c, fn((void*)c->tmp, bytes));
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

// operators of order p in the context's precision (built on first use)
ctfmm_status get_ops(ctfmm_ctx* c, int p, const unsigned char** kpk) {
    if (p == c->prm.order_p) {
        *kpk = c->Kpk;
        return CTFMM_OK;
    }
    for (const OpSet& o : c->opsets)
        if (o.p == p) {
            *kpk = o.Kpk;
            return CTFMM_OK;
        }
    const int prec = c->prm.precision;
    int max_lds = 0;
    HIPCHK(c, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
    if (m2l_tile_lds_bytes(p, prec, 32) > (size_t)max_lds)
        return fail(c, CTFMM_EUNSUPPORTED, "device LDS per workgroup too small for the M2L tile");
    const size_t nc = (size_t)(p + 1) * (p + 1);
    OpSet o;
    o.p = p;
    o.Dv = (double*)dev_alloc(c, (size_t)NOFF * NIND * sizeof(double));
    o.Kt = (double*)dev_alloc(c, (size_t)NOFF * nc * nc * sizeof(double));
    o.Kpk = (unsigned char*)dev_alloc(c, m2l_packed_bytes(p, prec));
    if (!o.Dv || !o.Kt || !o.Kpk) return fail(c, CTFMM_ENOMEM, "operator allocation failed");
    launch_offset_dtensors(c->stream, p, o.Dv);
    launch_build_k(c->stream, p, o.Dv, c->T, o.Kt);
    launch_pack_k(c->stream, p, prec, o.Kt, o.Kpk, p);
    HIPCHK(c, hipGetLastError());
    c->opsets.push_back(o);
    *kpk = o.Kpk;
    return CTFMM_OK;
}

// operators of every order q <= p in the order-p layout (built on first use)
ctfmm_status get_mixed_ops(ctfmm_ctx* c, int p, const unsigned char** kmix) {
    const unsigned char* dummy = nullptr;
    SCHK(get_ops(c, p, &dummy));
    const double* Kt = nullptr;
    unsigned char** slot = nullptr;
    if (p == c->prm.order_p) {
        Kt = c->Kt;
        slot = &c->Kmix;
    } else {
        for (OpSet& o : c->opsets)
            if (o.p == p) {
                Kt = o.Kt;
                slot = &o.Kmix;
            }
    }
    if (!Kt || !slot) return fail(c, CTFMM_EDEVICE, "operator set missing");
    if (!*slot) {
        const size_t per = m2l_packed_bytes(p, c->prm.precision);
        *slot = (unsigned char*)dev_alloc(c, per * (size_t)(p + 1));
        if (!*slot) return fail(c, CTFMM_ENOMEM, "operator allocation failed");
        for (int q = 0; q <= p; ++q) launch_pack_k(c->stream, p, c->prm.precision, Kt, *slot + per * q, q);
        HIPCHK(c, hipGetLastError());
    }
    *kmix = *slot;
    return CTFMM_OK;
}

// The M2L order rule of a forest: per-pair orders (table or network) apply
// to the forests of the context's own order; other forests keep their order.
int order_mode_of(const ctfmm_ctx* c, const Forest& f) { return f.p == c->prm.order_p ? c->order_mode : 0; }

// FP32 M2L runs the kernel that loads the source rows into registers
// (k_m2l_rb), from k-quad-major FP32 rows; the other precisions the tile
// kernel that stages them in LDS.
bool rb_m2l(const ctfmm_ctx* c) { return c->prm.precision == CTFMM_PREC_FP32; }

// M2L arguments of the forest's tiles over their active offsets; with
// orders, each active offset at the order of its (tile, offset)
AdaptM2L m2l_args(ctfmm_ctx* c, const Forest& f, bool orders) {
    AdaptM2L ad{f.tiles, f.tgt_tab, f.src_tab, c->alist + 8 * 189, 0};
    ad.ivlist = f.ivl;
    ad.ivcnt = f.ivc;
    if (orders) {
        ad.ivord = f.ivo;
        ad.kord_stride = m2l_packed_bytes(f.p, c->prm.precision);
    }
    return ad;
}

hipError_t m2l_adaptive(ctfmm_ctx* c, const Forest& f, hipStream_t st, const AdaptM2L& ad, const void* msrc,
                        double* out) {
    const int nt = (int)f.tiles_host.size();
    // the FP32 kernel truncates the order-p operators per offset itself
    const unsigned char* K = (ad.ivord && !rb_m2l(c)) ? f.Kmix : f.Kpk;
    if (rb_m2l(c)) return launch_m2l_rb(st, f.p, f.tt, nt, ad, static_cast<const float*>(msrc), out, K, c->zero_row);
    return launch_m2l_tables(st, f.p, c->prm.precision, f.tt, nt, ad, msrc, out, K, c->zero_row);
}

// Workgroups per M2L tile: the 189 offsets of a tile are split into chunks
// until there are about 2048 workgroups (8 per CU), at most 8 per tile.
int chunks_for(size_t ntiles) {
    if (ntiles == 0) return 1;
    const size_t want = (2048 + ntiles - 1) / ntiles;
    return (int)std::min<size_t>(8, std::max<size_t>(1, want));
}

// offset chunks per M2L tile, and the partial-sum slots they need (one per
// chunk, and one for the X lists)
ctfmm_status set_chunks(ctfmm_ctx* c, Forest& f, int nchunk) {
    f.nchunk = nchunk;
    if (!f.tiles_host.empty())
        ACHK(grow(c, f.part, f.part_cap, (size_t)(f.nchunk + 1) * f.nn * ldm_of(f.p), false));
    return CTFMM_OK;
}

// M2L tiles of tt targets from the (level, octant) buckets, and their tables
ctfmm_status make_tiles(ctfmm_ctx* c, Forest& f, int tt) {
    const int maxlev = (int)f.lev_first.size() - 1;
    f.tiles_host.clear();
    for (int l = 2; l <= maxlev; ++l)
        for (int o = 0; o < 8; ++o) {
            const int k = (l << 3) | o;
            const int b = f.hb[k], e = f.hb[256 + k];
            for (int s0 = b; s0 < e; s0 += tt) f.tiles_host.push_back(make_int4(o, s0, std::min(tt, e - s0), l));
        }
    f.tt = tt;
    const size_t ntiles = f.tiles_host.size();
    SCHK(set_chunks(c, f, c->chunk_tuned[f.p] ? c->chunk_tuned[f.p] : chunks_for(ntiles)));
    if (!ntiles) return CTFMM_OK;
    ACHK(grow(c, f.tiles, f.tiles_cap, ntiles, false));
    ACHK(grow(c, f.tgt_tab, f.tgt_cap, (size_t)tt * ntiles, false));
    ACHK(grow(c, f.src_tab, f.src_cap, (size_t)189 * tt * ntiles, false));
    ACHK(grow(c, f.vcount, f.vcount_cap, 189 * ntiles, false));
    ACHK(grow(c, f.tiles_tmp, f.tiles_tmp_cap, ntiles, false));
    ACHK(grow(c, f.tkey, f.tkey_cap, 2 * ntiles, false));
    ACHK(grow(c, f.tidx, f.tidx_cap, 2 * ntiles, false));
    ACHK(grow(c, f.ivl, f.ivl_cap, 189 * ntiles, false));
    ACHK(grow(c, f.ivo, f.ivo_cap, 189 * ntiles, false));
    ACHK(grow(c, f.ivc, f.ivc_cap, ntiles, false));
    HIPCHK(c, hipMemcpyAsync(f.tiles_tmp, f.tiles_host.data(), ntiles * sizeof(int4), hipMemcpyHostToDevice,
                             c->stream));
    // Tiles in the order of their first target's parent: the workgroups that
    // run together on one XCD then share their source rows in its L2.
    const int nt = (int)ntiles;
    int kbits = 3;
    while (kbits < 64 && (1ll << (kbits - 3)) < (long long)f.nn) ++kbits;
    launch_tile_keys(c->stream, nt, f.tiles_tmp, f.lovs, f.tr, f.tkey, f.tidx);
    SCHK(cub_run(c, [&](void* t, size_t& b) {
        return hipcub::DeviceRadixSort::SortPairs(t, b, f.tkey, f.tkey + nt, f.tidx, f.tidx + nt, nt, 0, kbits,
                                                  c->stream);
    }));
    launch_gather_int4(c->stream, nt, f.tidx + nt, f.tiles_tmp, f.tiles);
    launch_m2l_tables(c->stream, tt, (int)ntiles, f.tiles, f.lovs, f.tr, c->alist, f.tgt_tab, f.src_tab, f.vcount);
    // the offsets with at least one source, at the forest's order (per-pair
    // orders rewrite these lists in the numeric pass)
    launch_active_offsets(c->stream, nt, f.p, nullptr, f.vcount, f.ivl, f.ivo, f.ivc);
    HIPCHK(c, hipGetLastError());
    return CTFMM_OK;
}

// The tile-shape tuner: for every tile size the device's LDS admits (on this
// forest's own tables) and every split of a tile's offsets over 1 to 4
// workgroups, times three runs (after a warm-up run) of the M2L launch (at
// the forest's order) with the clear and the sum of its partial-sum slots.
// It returns the smallest tile within 5% of the fastest time (the fastest
// split for it): the trial launches run alone, while in an evaluation M2L
// shares the GPU with the near field and the X and W lists, where smaller
// workgroups fit beside them (Plummer 2^20, p=8: 32 targets 3.66-3.69 ms
// per step, 64 targets 3.82, with the same time alone).  The multipole
// buffer's contents do not matter for the timing; what it writes is
// overwritten by the real pass.
ctfmm_status tune_tile(ctfmm_ctx* c, Forest& f, int* best, int* best_chunks) {
    const int prec = c->prm.precision;
    int max_lds = 0;
    HIPCHK(c, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
    for (auto& e : c->tev)
        if (!e) HIPCHK(c, hipEventCreate(&e));
    const void* msrc = prec == CTFMM_PREC_FP64 ? (const void*)f.aM : (const void*)f.aM32;
    const size_t lsz = (size_t)f.nn * ldm_of(f.p);
    std::vector<std::array<float, 3>> trials;  // (tile, chunks, ms)
    *best = 32;  // fits wherever the context could be created
    *best_chunks = 0;
    for (int tt : {32, 64, 128}) {
        if (m2l_tile_lds_bytes(f.p, prec, tt) > (size_t)max_lds) continue;
        SCHK(make_tiles(c, f, tt));
        for (int nchunk = 1; nchunk <= 4; ++nchunk) {
            SCHK(set_chunks(c, f, nchunk));
            const int slots = nchunk + (f.tot_x > 0 ? 1 : 0);
            AdaptM2L ad = m2l_args(c, f, false);
            double* out = f.aL;
            if (slots > 1) {
                ad.acc = true;
                ad.nchunk = nchunk;
                ad.chunk_stride = lsz;
                out = f.part;
            }
            auto run = [&]() -> ctfmm_status {
                // only the X-list slot is added into; the M2L chunks write theirs
                if (slots > nchunk) launch_fill0(c->stream, (long long)lsz, f.part + (size_t)nchunk * lsz);
                HIPCHK(c, m2l_adaptive(c, f, c->stream, ad, msrc, out));
                if (slots > 1)
                    launch_sum_chunks(c->stream, slots, lsz, f.part, f.aL, (f.p + 1) * (f.p + 1), ldm_of(f.p),
                                      f.lev_first.size() > 2 ? f.lev_first[2] : 0);
                return CTFMM_OK;
            };
            SCHK(run());
            float ms = 0.f;
            for (int rep = 0; rep < 3; ++rep) {  // the fastest of three timed runs
                HIPCHK(c, hipEventRecord(c->tev[0], c->stream));
                SCHK(run());
                HIPCHK(c, hipEventRecord(c->tev[1], c->stream));
                HIPCHK(c, hipEventSynchronize(c->tev[1]));
                float t = 0.f;
                HIPCHK(c, hipEventElapsedTime(&t, c->tev[0], c->tev[1]));
                ms = rep == 0 ? t : std::min(ms, t);
            }
            trials.push_back({(float)tt, (float)nchunk, ms});
        }
    }
    float tmin = 0.f;
    for (const auto& t : trials)
        if (tmin == 0.f || t[2] < tmin) tmin = t[2];
    float tsel = 0.f;
    for (const auto& t : trials) {
        if (t[2] > 1.05f * tmin) continue;
        const int tt = (int)t[0];
        if (*best_chunks == 0 || tt < *best || (tt == *best && t[2] < tsel)) {
            *best = tt;
            *best_chunks = (int)t[1];
            tsel = t[2];
        }
    }
    return CTFMM_OK;
}

// Keys, sort, the trees level by level, neighbour tables, U/W/X lists, the
// (particle, W entry) pairs and the M2L tile tables of one forest.  Waits for
// the stream once per tree level and a few times more (sizes decide the next
// launches).  f.p, f.nsys, f.goff_h and f.gbase_h are set by the caller.
ctfmm_status build_forest(ctfmm_ctx* c, Forest& f, const double* xyz, const double* q, bool explicit_box,
                          bool early_up = false, bool tree_only = false) {
    hipStream_t st = c->stream;
    const int n = f.n;
    const size_t nn_ = (size_t)std::max(n, 1);
    SCHK(get_ops(c, f.p, &f.Kpk));
    ACHK(grow(c, f.k64, f.k64_cap, nn_, false));
    ACHK(grow(c, f.k64s, f.k64s_cap, nn_, false));
    ACHK(grow(c, f.k32, f.k32_cap, nn_, false));
    ACHK(grow(c, f.k32s, f.k32s_cap, nn_, false));
    ACHK(grow(c, f.deep, f.deep_cap, 1, false));
    ACHK(grow(c, f.a_idx, f.a_idx_cap, nn_, false));
    ACHK(grow(c, f.a_idxs, f.a_idxs_cap, nn_, false));
    ACHK(grow(c, f.leaf_of, f.leaf_of_cap, nn_, false));
    ACHK(grow(c, f.a_P, f.a_P_cap, nn_, false));
    ACHK(grow(c, f.a_F, f.a_F_cap, nn_, false));
    ACHK(grow(c, f.a_Fn, f.a_Fn_cap, nn_, false));
    ACHK(grow(c, f.bbox, f.bbox_cap, 6 * NBB + 4, false));
    ACHK(grow(c, f.bse, f.bse_cap, 512, false));
    ACHK(grow(c, f.vsum, f.vsum_cap, 1, false));
    ACHK(grow(c, f.boxes, f.boxes_cap, (size_t)f.nsys, false));
    ACHK(grow(c, f.goff, f.goff_cap, (size_t)f.nsys + 1, false));
    ACHK(grow(c, f.gbase, f.gbase_cap, (size_t)f.nsys, false));
    HIPCHK(c, hipMemcpyAsync(f.goff, f.goff_h.data(), (f.nsys + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(f.gbase, f.gbase_h.data(), f.nsys * sizeof(int32_t), hipMemcpyHostToDevice, st));
    const ASys sy{f.nsys, f.goff, f.gbase};
    // root cubes
    if (explicit_box) {
        const ABox b{{c->prm.root_lo[0], c->prm.root_lo[1], c->prm.root_lo[2]}, c->prm.root_side};
        HIPCHK(c, hipMemcpyAsync(f.boxes, &b, sizeof(ABox), hipMemcpyHostToDevice, st));
        HIPCHK(c, hipStreamSynchronize(st));
    } else if (f.nsys == 1) {
        const int nparts = std::min(NBB, std::max(1, (n + 255) / 256));
        launch_bbox(st, n, xyz + 3 * (size_t)f.gbase_h[0], f.bbox, nparts, f.bbox + 6 * NBB);
        HIPCHK(c, hipMemcpyAsync(f.boxes, f.bbox + 6 * NBB, sizeof(ABox), hipMemcpyDeviceToDevice, st));
    } else {
        launch_bbox_systems(st, sy, xyz, f.boxes);
    }
    launch_keys64(st, n, sy, xyz, f.boxes, f.k64, f.k32, f.a_idx, c->err_flag, f.nsys > 1);
    // The particles are sorted by the top 32 key bits (4 radix passes instead
    // of 8), which orders every cell down to level 10, and the full keys are
    // recomputed in sorted order.  Several systems are sorted at once on the
    // system index above those bits (one radix sort over all particles: a
    // segmented sort gives each system, up to 500 k particles, to one
    // workgroup).  A tree that goes deeper (some level-10 cell holds more
    // than leaf_max particles) is detected with the first level's count; the
    // particles are then sorted on all 63 bits and the tree built again.
    if (f.nsys == 1) {
        SCHK(cub_run(c, [&](void* t, size_t& b) {
            return hipcub::DeviceRadixSort::SortPairs(t, b, f.k32, f.k32s, f.a_idx, f.a_idxs, n, 0, 32, st);
        }));
    } else {
        int sbits = 1;
        while ((1 << sbits) < f.nsys) ++sbits;
        SCHK(cub_run(c, [&](void* t, size_t& b) {
            return hipcub::DeviceRadixSort::SortPairs(t, b, f.k64, f.k64s, f.a_idx, f.a_idxs, n, 0, 32 + sbits, st);
        }));
        launch_low32(st, n, f.k64s, f.k32s);
    }
    launch_gather_keyed(st, n, sy, f.a_idxs, xyz, q, f.boxes, f.a_P, f.k64s);
    launch_deep_check(st, n, sy, f.k32s, c->prm.leaf_max, f.deep);
    HIPCHK(c, hipGetLastError());
    auto full_sort = [&]() -> ctfmm_status {
        if (f.nsys == 1) {
            SCHK(cub_run(c, [&](void* t, size_t& b) {
                return hipcub::DeviceRadixSort::SortPairs(t, b, f.k64, f.k64s, f.a_idx, f.a_idxs, n, 0, 3 * AMAX, st);
            }));
        } else {
            // the full keys again (the first sort's keys held the system index)
            launch_keys64(st, n, sy, xyz, f.boxes, f.k64, f.k32, f.a_idx, c->err_flag, false);
            SCHK(cub_run(c, [&](void* t, size_t& b) {
                return hipcub::DeviceSegmentedRadixSort::SortPairs(t, b, f.k64, f.k64s, f.a_idx, f.a_idxs, n,
                                                                    f.nsys, f.goff, f.goff + 1, 0, 3 * AMAX, st);
            }));
        }
        launch_gather(st, n, f.a_idxs, xyz, q, f.a_P);
        HIPCHK(c, hipGetLastError());
        return CTFMM_OK;
    };
    bool sorted_full = false;

    // trees, level by level (level 0 holds one root per system)
    ACHK(grow_nodes(c, f, (size_t)f.nsys));
tree_again:
    launch_roots(st, sy, f.tr);
    f.lev_first.assign(1, 0);
    f.lev_count.assign(1, f.nsys);
    int first = 0, count = f.nsys, total = f.nsys;
    for (int l = 0;; ++l) {
        const size_t m = 8 * (size_t)count;
        ACHK(grow(c, f.sflag, f.sflag_cap, m, false));
        ACHK(grow(c, f.sincl, f.sincl_cap, m, false));
        ACHK(grow(c, f.scstart, f.scstart_cap, m, false));
        launch_split(st, l, first, count, c->prm.leaf_max, f.k64s, f.tr, f.sflag, f.scstart);
        SCHK(cub_run(c, [&](void* t, size_t& b) {
            return hipcub::DeviceScan::InclusiveSum(t, b, f.sflag, f.sincl, (int)m, st);
        }));
        // the children go to [total, total + nnext) with nnext <= m: they are
        // emitted before the host learns nnext
        ACHK(grow_nodes(c, f, (size_t)total + m));
        int* pw = pinned_words(c);
        if (!pw) return fail(c, CTFMM_ENOMEM, "pinned host allocation failed");
        const int nw = (l == 0 && !sorted_full) ? 2 : 1;  // level 0 also reads the depth check
        arm_words(pw, nw);
        // k_emit writes the count (and the depth check) into the pinned words
        launch_emit(st, l, first, count, total, f.sflag, f.sincl, f.scstart, f.tr, c->pinned_dev,
                    nw == 2 ? f.deep : nullptr);
        SCHK(wait_words(c, pw, nw));
        if (nw == 2 && pw[1] != 0) {
            SCHK(full_sort());
            sorted_full = true;
            goto tree_again;
        }
        const int nnext = pw[0];
        if (nnext == 0) break;
        first = total;
        count = nnext;
        total += nnext;
        f.lev_first.push_back(first);
        f.lev_count.push_back(count);
    }
    HIPCHK(c, hipGetLastError());
    const int nn = total;
    f.nn = nn;
    const int maxlev = (int)f.lev_first.size() - 1;
    launch_node_geo(st, nn, f.boxes, f.tr);
    for (int l = 1; l <= maxlev; ++l) launch_nb(st, f.lev_first[l], f.lev_count[l], f.tr);
    launch_leaf_of(st, nn, f.tr, f.leaf_of);
    for (auto& x : c->side)
        if (!x) HIPCHK(c, hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    for (auto& e : c->side_ev)
        if (!e) HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (tree_only) return CTFMM_OK;
    // P2M and M2M need only the nodes: with early_up they start here on a side
    // stream, beside the list and M2L-table construction, and the numeric
    // pass joins them
    f.up_early = early_up;
    if (early_up) {
        ACHK(grow(c, f.aM, f.aM_cap, (size_t)nn * ldm_of(f.p), false));
        HIPCHK(c, hipEventRecord(c->side_ev[5], st));
        HIPCHK(c, hipStreamWaitEvent(c->side[1], c->side_ev[5], 0));
        launch_p2m_nodes(c->side[1], f.p, 0, nn, f.boxes, f.tr, f.a_P, c->T, f.aM);
        for (int l = maxlev - 1; l >= 2; --l)
            launch_m2m_nodes(c->side[1], f.p, f.lev_first[l], f.lev_count[l], f.tr, f.aM, c->T);
        HIPCHK(c, hipEventRecord(c->side_ev[6], c->side[1]));
    }

    // U, W, X lists: count, scan, fill, order the transposed entries
    const size_t n1 = (size_t)nn + 1;
    ACHK(grow(c, f.lcnt, f.lcnt_cap, 7 * n1, false));
    ACHK(grow(c, f.loff, f.loff_cap, 3 * n1, false));
    int32_t *uc = f.lcnt, *wc = f.lcnt + n1, *xc = f.lcnt + 2 * n1, *ufc = f.lcnt + 3 * n1;
    int32_t *ut = f.lcnt + 4 * n1, *wfl = f.lcnt + 5 * n1, *ufl = f.lcnt + 6 * n1;
    int32_t *uo = f.loff, *wo = f.loff + n1, *xo = f.loff + 2 * n1;
    HIPCHK(c, hipMemsetAsync(f.lcnt, 0, 7 * n1 * sizeof(int32_t), st));
    launch_lists(st, false, nn, f.tr, uc, wc, xc, ufc, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                 nullptr);
    launch_add_i32(st, (int)n1, uc, ufc, ut);
    for (int k = 0; k < 3; ++k) {
        int32_t* in = k == 0 ? ut : f.lcnt + k * n1;
        int32_t* out = f.loff + k * n1;
        SCHK(cub_run(c, [&](void* t, size_t& b) { return hipcub::DeviceScan::ExclusiveSum(t, b, in, out, (int)n1, st); }));
    }
    int tot[3];
    int* pw = pinned_words(c);
    if (!pw) return fail(c, CTFMM_ENOMEM, "pinned host allocation failed");
    arm_words(pw, 3);
    for (int k = 0; k < 3; ++k)
        HIPCHK(c, hipMemcpyAsync(pw + k, f.loff + k * n1 + nn, sizeof(int), hipMemcpyDeviceToHost, st));
    SCHK(wait_words(c, pw, 3));
    for (int k = 0; k < 3; ++k) tot[k] = pw[k];
    f.tot_u = tot[0];
    f.tot_w = tot[1];
    f.tot_x = tot[2];
    ACHK(grow(c, f.ulist, f.ulist_cap, (size_t)tot[0], false));
    ACHK(grow(c, f.wlist, f.wlist_cap, (size_t)tot[1], false));
    ACHK(grow(c, f.xlist, f.xlist_cap, (size_t)tot[2], false));
    launch_lists(st, true, nn, f.tr, uc, wc, xc, ufc, uo, wo, xo, f.ulist, f.wlist, f.xlist, wfl, ufl);
    // the transposed entries in ascending node order: segment sorts of the W
    // lists and of the finer part of each U list ([uoff + own, uoff'))
    {
        ACHK(grow(c, f.lsort, f.lsort_cap, (size_t)std::max(tot[0], tot[1]) + 1, false));
        int32_t* ubeg = ut;  // the U totals are no longer needed
        launch_add_i32(st, nn, uo, uc, ubeg);
        if (tot[0] > 0) {
            HIPCHK(c, hipMemcpyAsync(f.lsort, f.ulist, (size_t)tot[0] * 4, hipMemcpyDeviceToDevice, st));
            launch_rank_sort(st, nn, ubeg, uo + 1, f.ulist, f.lsort);
            HIPCHK(c, hipMemcpyAsync(f.ulist, f.lsort, (size_t)tot[0] * 4, hipMemcpyDeviceToDevice, st));
        }
        if (tot[1] > 0) {
            launch_rank_sort(st, nn, wo, wo + 1, f.wlist, f.lsort);
            HIPCHK(c, hipMemcpyAsync(f.wlist, f.lsort, (size_t)tot[1] * 4, hipMemcpyDeviceToDevice, st));
        }
    }
    // expansion buffers
    const size_t ldm = (size_t)ldm_of(f.p);
    ACHK(grow(c, f.aM, f.aM_cap, (size_t)nn * ldm, false));
    ACHK(grow(c, f.aL, f.aL_cap, (size_t)nn * ldm, false));
    if (f.tot_w > 0) ACHK(grow(c, f.aWc, f.aWc_cap, (size_t)nn * m2p_coef_ld(f.p), false));
    if (c->prm.precision != CTFMM_PREC_FP64) ACHK(grow(c, f.aM32, f.aM32_cap, (size_t)nn * s32_of(f.p), false));

    // M2L tiles: nodes grouped by (level, octant), Morton order inside
    ACHK(grow(c, f.lok, f.lok_cap, (size_t)nn, false));
    ACHK(grow(c, f.loks, f.loks_cap, (size_t)nn, false));
    ACHK(grow(c, f.lov, f.lov_cap, (size_t)nn, false));
    ACHK(grow(c, f.lovs, f.lovs_cap, (size_t)nn, false));
    launch_lvloct(st, nn, f.tr, f.lok, f.lov);
    SCHK(cub_run(c, [&](void* t, size_t& b) {
        return hipcub::DeviceRadixSort::SortPairs(t, b, f.lok, f.loks, f.lov, f.lovs, nn, 0, 8, st);
    }));
    launch_buckets(st, nn, f.loks, f.bse, f.bse + 256);
    static_assert(sizeof(f.hb) <= 1024 * sizeof(int), "pinned words too few");
    arm_words(pw, 512);
    HIPCHK(c, hipMemcpyAsync(pw, f.bse, sizeof(f.hb), hipMemcpyDeviceToHost, st));
    SCHK(wait_words(c, pw, 512));
    std::memcpy(f.hb, pw, sizeof(f.hb));
    int tt = c->tile_forced[f.p] ? c->tile_forced[f.p] : c->tile_tuned[f.p];
    if (tt == 0 && maxlev >= 2) {
        int nc = 0;
        SCHK(tune_tile(c, f, &tt, &nc));
        c->tile_tuned[f.p] = tt;
        c->chunk_tuned[f.p] = nc;
    }
    SCHK(make_tiles(c, f, tt ? tt : 64));
    if (order_mode_of(c, f) != 0 && !f.tiles_host.empty()) {
        const size_t nt = f.tiles_host.size();
        if (!rb_m2l(c)) SCHK(get_mixed_ops(c, f.p, &f.Kmix));  // FP32 truncates the order-p set itself
        ACHK(grow(c, f.ordn, f.ordn_cap, (size_t)nn * NCLASS, false));
        ACHK(grow(c, f.tq, f.tq_cap, 189 * nt, false));
        ACHK(grow(c, f.ocnt, f.ocnt_cap, (size_t)11 * 189 * nt, false));
        if (order_mode_of(c, f) == 2) {
            ACHK(grow(c, f.mx, f.mx_cap, (size_t)nn * NCLASS * MLP_NIN, false));
            ACHK(grow(c, f.my, f.my_cap, (size_t)nn * NCLASS * MLP_NOUT, false));
        }
    }
    HIPCHK(c, hipGetLastError());
    f.v_pairs = -1;
    return CTFMM_OK;
}

// (target, source) pairs of the M2L tiles built last (waits for the stream)
ctfmm_status count_v_pairs(ctfmm_ctx* c, Forest& f) {
    if (f.v_pairs >= 0) return CTFMM_OK;
    const int m = 189 * (int)f.tiles_host.size();
    int v = 0;
    if (m > 0) {
        SCHK(cub_run(c, [&](void* t, size_t& b) {
            return hipcub::DeviceReduce::Sum(t, b, f.vcount, f.vsum, m, c->stream);
        }));
        HIPCHK(c, hipMemcpyAsync(&v, f.vsum, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    f.v_pairs = v;
    return CTFMM_OK;
}

// The numeric passes of one forest (no host waits, no memsets: graph-capturable).
// The near field (P2P) runs on a side stream from the start, followed there
// by the W lists once their coefficients are formed, and the X lists (P2L) on
// another beside M2L; the main stream joins them before the sum of the M2L
// slots and before the final sum of far and near field.  ev >= 0 records the
// phase events ev.. on the main stream (0 start, 1 P2M, 2 M2M, 3 conversions,
// 4 M2L with the X lists beside it and the order choice, 5 the rest of the
// X lists, 6 L2L, 7 far field and the join with the near field; 8 and 9
// around the M2L launch itself).  to_F leaves the results in sorted order in
// f.a_F (for launch_scatter_out) instead of writing phi and grad.
ctfmm_status numeric_forest(ctfmm_ctx* c, Forest& f, double* phi, double* grad, int ev, bool to_F = false) {
    hipStream_t st = c->stream;
    const int p = f.p;
    const int prec = c->prm.precision;
    const int nn = f.nn;
    const int maxlev = (int)f.lev_first.size() - 1;
    auto mark = [&](int k) {
        if (ev >= 0) rec(c, ev + k);
    };
    mark(0);
    // the near field needs only the particles and the U lists: it runs on a
    // side stream beside everything up to the final sum
    const size_t n1 = (size_t)nn + 1;
    HIPCHK(c, hipEventRecord(c->side_ev[0], st));
    HIPCHK(c, hipStreamWaitEvent(c->side[0], c->side_ev[0], 0));
    launch_p2p_near(c->side[0], f.n, nn, f.tr, f.a_P, f.loff, f.ulist, f.a_Fn);
    // the X lists need only the particles too: they start on a second side
    // stream into the last partial-sum slot of M2L (all slots cleared first)
    const size_t lsz = (size_t)nn * ldm_of(p);
    const bool x_early = !f.tiles_host.empty() && f.tot_x > 0;
    if (x_early) {
        launch_fill0(st, (long long)lsz, f.part + (size_t)f.nchunk * lsz);
        HIPCHK(c, hipEventRecord(c->side_ev[2], st));
        HIPCHK(c, hipStreamWaitEvent(c->side[1], c->side_ev[2], 0));
        launch_p2l(c->side[1], p, nn, f.boxes, f.tr, f.loff + 2 * n1, f.xlist, f.a_P, c->T,
                   f.part + (size_t)f.nchunk * lsz);
        HIPCHK(c, hipEventRecord(c->side_ev[3], c->side[1]));
    }
    if (f.up_early) {
        HIPCHK(c, hipStreamWaitEvent(st, c->side_ev[6], 0));
        mark(1);
    } else {
        launch_p2m_nodes(st, p, 0, nn, f.boxes, f.tr, f.a_P, c->T, f.aM);
        mark(1);
        for (int l = maxlev - 1; l >= 2; --l)
            launch_m2m_nodes(st, p, f.lev_first[l], f.lev_count[l], f.tr, f.aM, c->T);
    }
    mark(2);
    const void* msrc = f.aM;
    if (maxlev >= 2) {
        const int f2 = f.lev_first[2];
        if (f.tot_w > 0) {
            // the W lists need only the multipoles: they follow P2P on its side
            // stream, adding into the near field
            launch_m2p_coef(st, p, f2, nn - f2, f.aM, c->T, f.aWc);
            HIPCHK(c, hipEventRecord(c->side_ev[4], st));
            HIPCHK(c, hipStreamWaitEvent(c->side[0], c->side_ev[4], 0));
            launch_wlist_adaptive(c->side[0], p, nn, f.boxes, f.tr, f.a_P, f.aWc, f.loff + n1, f.wlist, f.a_Fn);
        }
        if (prec != CTFMM_PREC_FP64) {
            if (rb_m2l(c)) launch_to_f32_kq(st, p, nn, f.aM, f.aM32);
            else launch_to_f32(st, p, nn, f.aM, f.aM32);
            msrc = f.aM32;
        }
    }
    mark(3);
    // downward: L(B) = M2L(V) + P2L(X) + L2L(parent).  M2L over the tiles of
    // every level at once (it reads only M), the X lists beside it, then L2L
    // top-down.
    const int omode = order_mode_of(c, f);
    bool x_done = false;
    if (!f.tiles_host.empty()) {
        const int nt = (int)f.tiles_host.size();
        if (omode != 0) {
            // orders per (source cell, distance class), then per (tile,
            // offset) the largest its pairs ask for; the active-offset lists
            // are rewritten with those orders
            const int f2 = f.lev_first[2];
            if (omode == 1) {
                launch_order_table(st, nn, c->order_tab, f.ordn);
            } else if (omode == 3) {
                launch_order_hash(st, nn, f.tr, c->order_seed, c->order_pmin, p, f.ordn);
            } else {
                const long long rows = (long long)(nn - f2) * NCLASS;
                launch_mlp_node_features(st, f2, nn - f2, f.aM, ldm_of(p), f.mx);
                launch_mlp_forward16(st, rows, f.mx, c->model, c->model + MLP_NPARAM, f.my);
                launch_mlp_decide(st, f2, nn - f2, f.my, c->order_thr, f.ordn);
            }
            launch_m2l_orders(st, f.tt, nt, f.tiles, f.src_tab, c->alist + 8 * 189, f.ordn, f.tq, f.ocnt);
            launch_active_offsets(st, nt, p, f.tq, nullptr, f.ivl, f.ivo, f.ivc);
        }
        // M2L chunks into slots 0 .. nchunk-1 of part; the X lists (P2L, on a
        // side stream beside M2L) into slot nchunk; then the slots are summed
        AdaptM2L ad = m2l_args(c, f, omode != 0);
        const bool xs = f.tot_x > 0;
        const int slots = f.nchunk + (xs ? 1 : 0);
        if (slots == 1) {
            mark(8);
            HIPCHK(c, m2l_adaptive(c, f, st, ad, msrc, f.aL));
            mark(9);
        } else {
            if (xs && !x_early) launch_fill0(st, (long long)lsz, f.part + (size_t)f.nchunk * lsz);
            if (xs && !x_early) {
                HIPCHK(c, hipEventRecord(c->side_ev[2], st));
                HIPCHK(c, hipStreamWaitEvent(c->side[1], c->side_ev[2], 0));
                launch_p2l(c->side[1], p, nn, f.boxes, f.tr, f.loff + 2 * n1, f.xlist, f.a_P, c->T,
                           f.part + (size_t)f.nchunk * lsz);
                HIPCHK(c, hipEventRecord(c->side_ev[3], c->side[1]));
            }
            ad.acc = true;
            ad.nchunk = f.nchunk;
            ad.chunk_stride = lsz;
            mark(8);
            HIPCHK(c, m2l_adaptive(c, f, st, ad, msrc, f.part));
            mark(9);
            if (xs) HIPCHK(c, hipStreamWaitEvent(st, c->side_ev[3], 0));
            launch_sum_chunks(st, slots, lsz, f.part, f.aL, (p + 1) * (p + 1), ldm_of(p), f.lev_first[2]);
        }
        x_done = true;
    } else {
        mark(8);
        mark(9);
    }
    mark(4);
    if (f.tot_x > 0 && !x_done) launch_p2l(st, p, nn, f.boxes, f.tr, f.loff + 2 * n1, f.xlist, f.a_P, c->T, f.aL);
    mark(5);
    for (int l = 3; l <= maxlev; ++l) launch_l2l_nodes(st, p, f.lev_first[l - 1], f.lev_count[l - 1], f.tr, f.aL, c->T);
    mark(6);
    HIPCHK(c, hipEventRecord(c->side_ev[1], c->side[0]));  // P2P and the W lists are done
    HIPCHK(c, hipStreamWaitEvent(st, c->side_ev[1], 0));
    launch_far_adaptive(st, p, f.n, nn, false, f.boxes, f.tr, f.leaf_of, f.a_P, f.aL, f.aWc, f.loff + n1, f.wlist,
                        f.a_F, f.a_Fn, f.a_idxs, to_F, phi, grad);
    mark(7);
    HIPCHK(c, hipGetLastError());
    return CTFMM_OK;
}

// pairs per M2L order of the last numeric pass of f (waits for the stream)
ctfmm_status add_order_hist(ctfmm_ctx* c, Forest& f) {
    const int m = 189 * (int)f.tiles_host.size();
    if (m == 0) return CTFMM_OK;
    if (order_mode_of(c, f) == 0) {
        SCHK(count_v_pairs(c, f));
        c->st.m2l_order_pairs[f.p] += f.v_pairs;
        return CTFMM_OK;
    }
    for (int o = 0; o <= f.p; ++o) {
        int v = 0;
        const int32_t* in = f.ocnt + (size_t)o * m;
        SCHK(cub_run(c, [&](void* t, size_t& b) { return hipcub::DeviceReduce::Sum(t, b, in, f.vsum, m, c->stream); }));
        HIPCHK(c, hipMemcpyAsync(&v, f.vsum, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->st.m2l_order_pairs[o] += v;
    }
    return CTFMM_OK;
}

// phase times of one adaptive evaluation from its event set
void add_adaptive_times(ctfmm_ctx* c, hipEvent_t* ev) {
    const int ev_end = NPHASE_EV - 1;
    c->st.ms_total += elapsed_in(ev, 0, ev_end);
    c->st.ms_tree += elapsed_in(ev, 0, 1);
    c->st.ms_p2m += elapsed_in(ev, 2, 3);
    c->st.ms_m2m += elapsed_in(ev, 3, 4);
    c->st.ms_convert += elapsed_in(ev, 4, 5);
    const double m2l = elapsed_in(ev, 10, 11);
    c->st.ms_m2l += m2l;
    c->st.ms_p2l += elapsed_in(ev, 5, 7) - m2l;
    c->st.ms_l2l += elapsed_in(ev, 7, 8);
    c->st.ms_near += elapsed_in(ev, 8, 9);
}

// adds the timings and pair count left pending by an adaptive evaluation
// (waits for that evaluation to finish)
ctfmm_status finish_pending(ctfmm_ctx* c) {
    if (!c->pend.on) return CTFMM_OK;
    c->pend.on = false;
    HIPCHK(c, hipEventSynchronize(c->pend.ev[NPHASE_EV - 1]));
    int* pw = pinned_words(c);
    SCHK(wait_words(c, pw + c->pend.word, 1));
    c->st.m2l_pairs += pw[c->pend.word];
    add_adaptive_times(c, c->pend.ev);
    return CTFMM_OK;
}

void add_forest_stats(ctfmm_ctx* c, Forest& f) {
    c->st.m2l_launches += f.tiles_host.empty() ? 0 : 1;
    c->st.p2p_leaf_pairs += f.tot_u;
}

ctfmm_status evaluate_adaptive(ctfmm_ctx* c, int n, const double* xyz, const double* q, double* phi,
                               double* grad) {
    if (c->forests.empty()) c->forests.resize(1);
    Forest& f = c->forests[0];
    c->nforests = 1;
    f.p = c->prm.order_p;
    f.nsys = 1;
    f.n = n;
    f.goff_h = {0, n};
    f.gbase_h = {0};
    // events: 0 start, 1 tree built, 2.. the numeric phases, then the end
    rec(c, 0);
    HIPCHK(c, hipMemsetAsync(c->err_flag, 0, sizeof(int), c->stream));
    SCHK(build_forest(c, f, xyz, q, c->prm.root_side > 0.0, true));
    rec(c, 1);
    SCHK(numeric_forest(c, f, phi, grad, 2));
    const int ev_end = NPHASE_EV - 1;
    rec(c, ev_end);
    c->have_result = true;
    c->st.evaluations += 1;
    add_forest_stats(c, f);
    if (c->timing) {
        // The previous evaluation's timings are complete by now (this one's
        // tree build waited on the stream behind it): add them.  This one's
        // stay pending, with its pair count on its way to a pinned word, so
        // that the call returns without waiting for the GPU.
        SCHK(finish_pending(c));
        if (order_mode_of(c, f) == 0) {
            const int m = 189 * (int)f.tiles_host.size();
            int* pw = pinned_words(c);
            if (!pw) return fail(c, CTFMM_ENOMEM, "pinned host allocation failed");
            const int word = c->ev == c->evs[0] ? 1000 : 1001;
            arm_words(pw + word, 1);
            if (m > 0) {
                SCHK(cub_run(c, [&](void* t, size_t& b) {
                    return hipcub::DeviceReduce::Sum(t, b, f.vcount, f.vsum, m, c->stream);
                }));
                HIPCHK(c, hipMemcpyAsync(pw + word, f.vsum, sizeof(int), hipMemcpyDeviceToHost, c->stream));
            } else {
                pw[word] = 0;
            }
            c->pend.on = true;
            c->pend.ev = c->ev;
            c->pend.word = word;
            c->ev = c->ev == c->evs[0] ? c->evs[1] : c->evs[0];
        } else {
            SCHK(count_v_pairs(c, f));
            c->st.m2l_pairs += f.v_pairs;
            SCHK(add_order_hist(c, f));
            HIPCHK(c, hipEventSynchronize(c->ev[ev_end]));
            add_adaptive_times(c, c->ev);
        }
    }
    return CTFMM_OK;
}

// ------------------------------------------------------------------ dual-tree evaluation

// The traversal in rounds (ctfmm_dual.hip).  Each round opens one node of a
// pair (both halves of a self pair), so the level sum of a pair grows by at
// least one per round and no pair is left after round 2 maxlev + 1.  The
// host reads the round counts once: entries past a buffer's capacity were
// counted but not written, and the traversal then runs again with larger
// buffers (they are kept for the next evaluation).  Then both entry lists
// are sorted and put in CSR form by target (leaf).
ctfmm_status dual_traverse(ctfmm_ctx* c, Forest& f, int maxlev) {
    hipStream_t st = c->stream;
    const int nn = f.nn;
    const int nr = 2 * maxlev + 2;
    int sh = 1;
    while ((1ll << sh) < (long long)nn) ++sh;
    f.dual_sh = sh;
    ACHK(grow(c, f.dcnt, f.dcnt_cap, (size_t)nr + 3, false));
    if (f.cap_f == 0) {
        f.cap_f = std::max<size_t>(4096, 16 * (size_t)nn);
        f.cap_m = std::max<size_t>(4096, 128 * (size_t)nn);
        f.cap_p = std::max<size_t>(4096, 32 * (size_t)nn);
    }
    int* pw = pinned_words(c);
    if (!pw) return fail(c, CTFMM_ENOMEM, "pinned host allocation failed");
    const int nw = nr + 4;
    for (int attempt = 0;; ++attempt) {
        ACHK(grow(c, f.front[0], f.front_cap[0], f.cap_f, false));
        ACHK(grow(c, f.front[1], f.front_cap[1], f.cap_f, false));
        ACHK(grow(c, f.mk, f.mk_cap, f.cap_m, false));
        ACHK(grow(c, f.pk, f.pk_cap, f.cap_p, false));
        launch_dual_init(st, nr, f.dcnt, f.front[0]);
        for (int r = 0; r < nr; ++r)
            launch_dual_round(st, r, nr, f.front[r & 1], f.front[(r + 1) & 1], (int)f.cap_f, f.mk, (int)f.cap_m, f.pk,
                              (int)f.cap_p, sh, f.dcnt, f.tr, f.zr, c->theta);
        HIPCHK(c, hipGetLastError());
        arm_words(pw, nw);
        HIPCHK(c, hipMemcpyAsync(pw, f.dcnt, (size_t)(nr + 3) * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipMemcpyAsync(pw + nr + 3, c->err_flag, sizeof(int), hipMemcpyDeviceToHost, st));
        SCHK(wait_words(c, pw, nw));
        const int err = pw[nr + 3];
        if (err) {
            HIPCHK(c, hipMemsetAsync(c->err_flag, 0, sizeof(int), st));
            return fail(c, CTFMM_EINVAL, (err & 1) ? "non-finite particle coordinate"
                                                   : "the AP variant needs positive charges");
        }
        size_t maxf = 0;
        for (int r = 1; r <= nr; ++r) maxf = std::max<size_t>(maxf, (size_t)pw[r]);
        const size_t nm = (size_t)pw[nr + 1], np = (size_t)pw[nr + 2];
        if (maxf <= f.cap_f && nm <= f.cap_m && np <= f.cap_p) {
            if (pw[nr] != 0) return fail(c, CTFMM_EDEVICE, "dual-tree traversal did not finish");
            f.n_m2l = (int)nm;
            f.n_p2p = (int)np;
            break;
        }
        if (attempt >= 16 || nm > (size_t)INT_MAX / 2 || np > (size_t)INT_MAX / 2 || maxf > (size_t)INT_MAX / 2)
            return fail(c, CTFMM_ENOMEM, "dual-tree traversal lists too long");
        f.cap_f = std::max(2 * f.cap_f, maxf + maxf / 4);
        f.cap_m = std::max(f.cap_m, nm + nm / 4 + 64);
        f.cap_p = std::max(f.cap_p, np + np / 4 + 64);
    }
    ACHK(grow(c, f.mks, f.mks_cap, std::max<size_t>(f.n_m2l, 1), false));
    ACHK(grow(c, f.pks, f.pks_cap, std::max<size_t>(f.n_p2p, 1), false));
    ACHK(grow(c, f.msrc, f.msrc_cap, std::max<size_t>(f.n_m2l, 1), false));
    ACHK(grow(c, f.psrc, f.psrc_cap, std::max<size_t>(f.n_p2p, 1), false));
    const int nm = f.n_m2l, np = f.n_p2p;
    if (nm > 0)
        SCHK(cub_run(c, [&](void* t, size_t& b) {
            return hipcub::DeviceRadixSort::SortKeys(t, b, f.mk, f.mks, nm, 0, 2 * sh, st);
        }));
    SCHK(cub_run(c, [&](void* t, size_t& b) {
        return hipcub::DeviceRadixSort::SortKeys(t, b, f.pk, f.pks, np, 0, 2 * sh, st);
    }));
    launch_dual_csr(st, nn, f.mks, f.dcnt + nr + 1, (int)f.cap_m, sh, f.moff, f.msrc);
    launch_dual_csr(st, nn, f.pks, f.dcnt + nr + 2, (int)f.cap_p, sh, f.poff, f.psrc);
    HIPCHK(c, hipGetLastError());
    return CTFMM_OK;
}

// events: 0 start, 1 tree and centres, 2 traversal and lists, 3 upward pass
// joined, 4 M2L, 5 L2L, last: L2P and the near field joined
void add_dual_times(ctfmm_ctx* c) {
    const int e = NPHASE_EV - 1;
    c->st.ms_total += elapsed(c, 0, e);
    c->st.ms_tree += elapsed(c, 0, 2);
    c->st.ms_m2l += elapsed(c, 3, 4);
    c->st.ms_l2l += elapsed(c, 4, 5);
    c->st.ms_near += elapsed(c, 5, e);
}

ctfmm_status evaluate_dual(ctfmm_ctx* c, int n, const double* xyz, const double* q, double* phi, double* grad) {
    if (c->forests.empty()) c->forests.resize(1);
    Forest& f = c->forests[0];
    c->nforests = 1;
    f.p = c->prm.order_p;
    f.nsys = 1;
    f.n = n;
    f.goff_h = {0, n};
    f.gbase_h = {0};
    const bool ap = c->centre == CTFMM_CENTRE_AP;
    hipStream_t st = c->stream;
    rec(c, 0);
    HIPCHK(c, hipMemsetAsync(c->err_flag, 0, sizeof(int), st));
    SCHK(build_forest(c, f, xyz, q, c->prm.root_side > 0.0, false, true));
    const int nn = f.nn, p = f.p, maxlev = (int)f.lev_first.size() - 1;
    const size_t ldm = (size_t)ldm_of(p);
    ACHK(grow(c, f.zr, f.zr_cap, (size_t)nn, false));
    ACHK(grow(c, f.aM, f.aM_cap, (size_t)nn * ldm, false));
    ACHK(grow(c, f.aL, f.aL_cap, (size_t)nn * ldm, false));
    ACHK(grow(c, f.moff, f.moff_cap, (size_t)nn + 1, false));
    ACHK(grow(c, f.poff, f.poff_cap, (size_t)nn + 1, false));
    ACHK(grow(c, f.zsum, f.zsum_cap, (size_t)nn, false));
    launch_dual_centres(st, n, nn, f.lev_first, f.lev_count, f.tr, f.boxes, f.leaf_of, f.a_P, c->centre, f.zsum, f.zr,
                        c->err_flag);
    rec(c, 1);
    // the upward pass needs the centres only: it runs on a side stream beside
    // the traversal
    HIPCHK(c, hipEventRecord(c->side_ev[0], st));
    HIPCHK(c, hipStreamWaitEvent(c->side[1], c->side_ev[0], 0));
    launch_dual_p2m(c->side[1], p, nn, f.tr, f.zr, f.a_P, c->T, f.aM);
    for (int l = maxlev - 1; l >= 0; --l)
        launch_dual_m2m(c->side[1], p, f.lev_first[l], f.lev_count[l], f.tr, f.zr, c->T, f.aM);
    HIPCHK(c, hipEventRecord(c->side_ev[1], c->side[1]));
    SCHK(dual_traverse(c, f, maxlev));
    rec(c, 2);
    // the near field beside the expansions
    HIPCHK(c, hipEventRecord(c->side_ev[2], st));
    HIPCHK(c, hipStreamWaitEvent(c->side[0], c->side_ev[2], 0));
    launch_p2p_near(c->side[0], n, nn, f.tr, f.a_P, f.poff, f.psrc, f.a_Fn);
    HIPCHK(c, hipEventRecord(c->side_ev[3], c->side[0]));
    HIPCHK(c, hipStreamWaitEvent(st, c->side_ev[1], 0));
    rec(c, 3);
    launch_dual_m2l(st, p, ap, nn, f.tr, f.zr, f.moff, f.msrc, f.aM, f.aL);
    rec(c, 4);
    for (int l = 1; l <= maxlev; ++l) launch_dual_l2l(st, p, f.lev_first[l], f.lev_count[l], f.tr, f.zr, c->T, f.aL);
    rec(c, 5);
    HIPCHK(c, hipStreamWaitEvent(st, c->side_ev[3], 0));
    launch_dual_l2p(st, p, ap, n, f.tr, f.leaf_of, f.zr, f.a_P, f.aL, f.a_Fn, f.a_idxs, phi, grad);
    HIPCHK(c, hipGetLastError());
    rec(c, NPHASE_EV - 1);
    c->have_result = true;
    c->st.evaluations += 1;
    c->st.m2l_launches += 1;
    c->st.m2l_pairs += f.n_m2l;
    c->st.p2p_leaf_pairs += f.n_p2p;
    if (c->timing) {
        HIPCHK(c, hipEventSynchronize(c->ev[NPHASE_EV - 1]));
        add_dual_times(c);
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
    if (prm->tree != CTFMM_TREE_UNIFORM && prm->tree != CTFMM_TREE_ADAPTIVE && prm->tree != CTFMM_TREE_DUAL) {
        g_create_err = "unknown tree type";
        return CTFMM_EUNSUPPORTED;
    }
    if (prm->order_p > CTFMM_P_MAX) {
        g_create_err = "expansion order above the compiled maximum (10)";
        return CTFMM_EUNSUPPORTED;
    }
    const bool adaptive = prm->tree != CTFMM_TREE_UNIFORM;  // the adaptive octree (lists or dual traversal)
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
    if (prm->tree == CTFMM_TREE_DUAL && prm->precision != CTFMM_PREC_FP64) {
        g_create_err = "the dual-tree traversal is FP64 only";
        return CTFMM_EUNSUPPORTED;
    }
    ctfmm_ctx* c = new (std::nothrow) ctfmm_ctx();
    if (!c) return CTFMM_ENOMEM;
    c->prm = *prm;
    c->stream = (hipStream_t)hip_stream;
    (void)hipGetDevice(&c->device);
    ctfmm_status s = upload_tables(c);
    if (s == CTFMM_OK && mlp_noalloc_setup(c->device) != hipSuccess)
        s = fail(c, CTFMM_EDEVICE, "device address of the backward-pass scratch array");
    if (s == CTFMM_OK) {
        c->err_flag = (int*)dev_alloc(c, sizeof(int));
        if (!c->err_flag) s = fail(c, CTFMM_ENOMEM, "allocation failed");
        else if (hipMemsetAsync(c->err_flag, 0, sizeof(int), c->stream) != hipSuccess)
            s = fail(c, CTFMM_EDEVICE, "clearing the error flag failed");
    }
    if (s == CTFMM_OK) s = build_operators(c);
    if (s == CTFMM_OK) {
        for (auto& set : c->evs)
            for (auto& e : set)
                if (s == CTFMM_OK && hipEventCreate(&e) != hipSuccess) s = fail(c, CTFMM_EDEVICE, "hipEventCreate failed");
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
    HIPCHK(c, hipMemsetAsync(c->err_flag, 0, sizeof(int), c->stream));  // workspace is never assumed zero
    return build_operators(c);
}

namespace {

// The uniform-tree evaluation; dip (may be null): point dipoles [n][3]
ctfmm_status evaluate_uniform(ctfmm_ctx* c, int64_t n, const double* xyz, const double* q, const double* dip,
                              double* phi, double* grad) {
    ctfmm_status s = ensure_workspace(c, n);
    if (s != CTFMM_OK) return s;
    if (dip && !grow(c, c->Pd, c->Pd_cap, (size_t)n, false)) return fail(c, CTFMM_ENOMEM, "workspace allocation failed");
    const double4* Pd = dip ? c->Pd : nullptr;
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
    if (dip) launch_gather_dip(st, ni, c->idx_sorted, dip, c->Pd);
    launch_leaf_start(st, nleaves, c->keys_sorted, ni, c->start);
    HIPCHK(c, hipGetLastError());
    rec(c, 1);
    const size_t ldm = (size_t)ldm_of(p);
    auto Ml = [&](int l) { return c->M + c->lvl_off[l] * ldm; };
    auto Ll = [&](int l) { return c->L + c->lvl_off[l] * ldm; };
    int evi = 5;
    if (d >= 2) {
        launch_p2m(st, p, box, c->start, c->P, c->T, Ml(d), Pd);
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
            // FP32: the M2L kernel adds the L2L from the parents itself
            const bool fused = c->prm.precision == CTFMM_PREC_FP32 && l >= 3;
            HIPCHK(c, launch_m2l(st, p, c->prm.precision, l, msrc, Ll(l), c->Kpk, c->offlist, c->zero_row, c->Kq,
                                 fused ? Ll(l - 1) : nullptr, c->T.l2l_t));
            rec(c, evi + 2);
            if (l >= 3 && !fused) launch_l2l(st, p, l - 1, Ll(l - 1), Ll(l), c->T);
            rec(c, evi + 3);
            evi += 4;
        }
        rec(c, 4);
        launch_l2p(st, p, ni, box, c->start, c->keys_sorted, c->P, Ll(d), c->F);
        if (Pd) launch_p2p(st, ni, box, c->keys_sorted, c->start, c->P, c->idx_sorted, c->F, phi, grad, Pd);
        else launch_p2p_leaves(st, box, c->start, c->P, c->idx_sorted, c->F, phi, grad);
    } else {
        rec(c, 2);
        rec(c, 3);
        rec(c, 4);
        if (Pd) launch_p2p(st, ni, box, c->keys_sorted, c->start, c->P, c->idx_sorted, nullptr, phi, grad, Pd);
        else launch_p2p_leaves(st, box, c->start, c->P, c->idx_sorted, nullptr, phi, grad);
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

}  // namespace

ctfmm_status ctfmm_evaluate(ctfmm_ctx* c, int64_t n, const double* xyz, const double* q, double* phi,
                            double* grad) {
    if (!c) return CTFMM_EINVAL;
    c->err.clear();
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(c, CTFMM_EINVAL, "n out of range");
    if (n == 0) return CTFMM_OK;
    if (!xyz || !q) return fail(c, CTFMM_EINVAL, "null xyz or q");
    if (c->prm.tree == CTFMM_TREE_ADAPTIVE) return evaluate_adaptive(c, (int)n, xyz, q, phi, grad);
    if (c->prm.tree == CTFMM_TREE_DUAL) {
        if (c->centre == CTFMM_CENTRE_AP && phi)
            return fail(c, CTFMM_EINVAL, "the AP variant gives the gradient only (phi must be NULL)");
        return evaluate_dual(c, (int)n, xyz, q, phi, grad);
    }
    return evaluate_uniform(c, n, xyz, q, nullptr, phi, grad);
}

ctfmm_status ctfmm_evaluate_dipoles(ctfmm_ctx* c, int64_t n, const double* xyz, const double* q, const double* dip,
                                    double* phi, double* grad) {
    if (!c) return CTFMM_EINVAL;
    c->err.clear();
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(c, CTFMM_EINVAL, "n out of range");
    if (n == 0) return CTFMM_OK;
    if (!xyz || !q || !dip) return fail(c, CTFMM_EINVAL, "null xyz, q or dip");
    if (c->prm.tree != CTFMM_TREE_UNIFORM) return fail(c, CTFMM_EUNSUPPORTED, "point dipoles need the uniform tree");
    return evaluate_uniform(c, n, xyz, q, dip, phi, grad);
}

ctfmm_status ctfmm_evaluate_batched(ctfmm_ctx* c, int32_t nsys, const int64_t* offsets, const int32_t* orders,
                                    const double* xyz, const double* q, double* phi, double* grad) {
    if (!c) return CTFMM_EINVAL;
    c->err.clear();
    if (c->prm.tree != CTFMM_TREE_ADAPTIVE) return fail(c, CTFMM_EUNSUPPORTED, "batched evaluation needs the adaptive tree");
    if (nsys < 1 || !offsets || !orders) return fail(c, CTFMM_EINVAL, "nsys >= 1 and host offsets/orders required");
    if (offsets[0] != 0) return fail(c, CTFMM_EINVAL, "offsets[0] must be 0");
    for (int s = 0; s < nsys; ++s) {
        if (offsets[s + 1] < offsets[s]) return fail(c, CTFMM_EINVAL, "offsets must not decrease");
        if (orders[s] < 0) return fail(c, CTFMM_EINVAL, "negative order");
        if (orders[s] > CTFMM_P_MAX) return fail(c, CTFMM_EUNSUPPORTED, "order above the compiled maximum (10)");
    }
    const int64_t total = offsets[nsys];
    if (total >= (int64_t(1) << 31)) return fail(c, CTFMM_EINVAL, "total particle count must be < 2^31");
    if (total == 0) return CTFMM_OK;
    if (!xyz || !q) return fail(c, CTFMM_EINVAL, "null xyz or q");
    // one forest per order, systems in input order inside it
    std::vector<int> ps(orders, orders + nsys);
    std::sort(ps.begin(), ps.end());
    ps.erase(std::unique(ps.begin(), ps.end()), ps.end());
    if (c->forests.size() < ps.size()) c->forests.resize(ps.size());
    c->nforests = (int)ps.size();
    for (int k = 0; k < c->nforests; ++k) {
        Forest& f = c->forests[k];
        f.p = ps[k];
        f.goff_h.assign(1, 0);
        f.gbase_h.clear();
        for (int s = 0; s < nsys; ++s)
            if (orders[s] == f.p) {
                f.gbase_h.push_back((int32_t)offsets[s]);
                f.goff_h.push_back(f.goff_h.back() + (int32_t)(offsets[s + 1] - offsets[s]));
            }
        f.nsys = (int)f.gbase_h.size();
        f.n = f.goff_h.back();
    }
    rec(c, 0);
    HIPCHK(c, hipMemsetAsync(c->err_flag, 0, sizeof(int), c->stream));
    for (int k = 0; k < c->nforests; ++k) SCHK(build_forest(c, c->forests[k], xyz, q, false));
    rec(c, 1);
    // every value the numeric launches depend on
    // (the outputs are not among them: the graph leaves results in sorted order)
    std::vector<long long> sig = {c->nforests, c->order_mode};
    for (int k = 0; k < c->nforests; ++k) {
        const Forest& f = c->forests[k];
        const void* ptrs[] = {f.boxes, f.tr.key, f.tr.pb, f.tr.pe, f.tr.par, f.tr.info, f.tr.child, f.tr.nb, f.tr.sys, f.tr.geo,
                              f.a_P, f.a_F, f.a_Fn, f.aM, f.aL, f.aWc, f.aM32, f.loff, f.xlist, f.wlist, f.ulist,
                              f.a_idxs, f.leaf_of, f.tiles, f.tgt_tab, f.src_tab, f.Kpk, f.Kmix, f.ordn,
                              f.tq, f.ocnt, f.ivl, f.ivo, f.ivc, f.mx, f.my, c->order_tab, c->model, f.part};
        for (const void* q2 : ptrs) sig.push_back((long long)(uintptr_t)q2);
        sig.insert(sig.end(), {f.p, f.n, f.nn, (long long)f.tiles_host.size(), f.tot_w, f.tot_x, f.tt,
                               f.nchunk});
        sig.insert(sig.end(), f.lev_first.begin(), f.lev_first.end());
        sig.insert(sig.end(), f.lev_count.begin(), f.lev_count.end());
    }
    if (sig != c->gsig) {
        // new shapes: run eagerly (also sets kernel attributes) and capture on the next call
        if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
        if (c->graph) (void)hipGraphDestroy(c->graph);
        c->gexec = nullptr;
        c->graph = nullptr;
        for (int k = 0; k < c->nforests; ++k) SCHK(numeric_forest(c, c->forests[k], nullptr, nullptr, -1, true));
        c->gsig = sig;
    } else {
        if (!c->gexec) {
            if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
            hipStream_t user = c->stream;
            c->stream = c->cap_stream;
            ctfmm_status cs = CTFMM_OK;
            hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                for (int k = 0; k < c->nforests && cs == CTFMM_OK; ++k)
                    cs = numeric_forest(c, c->forests[k], nullptr, nullptr, -1, true);
                hipGraph_t g = nullptr;
                const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
                if (e2 == hipSuccess && cs == CTFMM_OK) c->graph = g;
                else if (g) (void)hipGraphDestroy(g);
                if (e2 != hipSuccess && cs == CTFMM_OK) cs = fail(c, CTFMM_EDEVICE, "hipStreamEndCapture failed");
            } else {
                cs = fail(c, CTFMM_EDEVICE, "hipStreamBeginCapture failed");
            }
            c->stream = user;
            if (cs != CTFMM_OK) return cs;
            HIPCHK(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
        }
        HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
        c->st.graph_launches += 1;
    }
    for (int k = 0; k < c->nforests; ++k) {
        const Forest& f = c->forests[k];
        launch_scatter_out(c->stream, f.n, f.a_idxs, f.a_F, phi, grad);
    }
    HIPCHK(c, hipGetLastError());
    const int ev_end = NPHASE_EV - 1;
    rec(c, ev_end);
    c->have_result = true;
    c->st.evaluations += 1;
    for (int k = 0; k < c->nforests; ++k) add_forest_stats(c, c->forests[k]);
    if (c->timing) {
        for (int k = 0; k < c->nforests; ++k) {
            SCHK(count_v_pairs(c, c->forests[k]));
            c->st.m2l_pairs += c->forests[k].v_pairs;
            SCHK(add_order_hist(c, c->forests[k]));
        }
        HIPCHK(c, hipEventSynchronize(c->ev[ev_end]));
        c->st.ms_total += elapsed(c, 0, ev_end);
        c->st.ms_tree += elapsed(c, 0, 1);
        c->st.ms_numeric += elapsed(c, 1, ev_end);
    }
    return CTFMM_OK;
}

namespace {

// FP64 copies of FP32 inputs (and room for the outputs) for the FP32 entry points
ctfmm_status widen_inputs(ctfmm_ctx* c, int64_t n, const float* xyz, const float* q) {
    const size_t want[4] = {(size_t)3 * n, (size_t)n, (size_t)n, (size_t)3 * n};
    for (int k = 0; k < 4; ++k)
        if (!grow(c, c->io[k], c->io_cap[k], want[k], false)) return fail(c, CTFMM_ENOMEM, "workspace allocation failed");
    launch_widen(c->stream, 3 * n, xyz, c->io[0]);
    launch_widen(c->stream, n, q, c->io[1]);
    HIPCHK(c, hipGetLastError());
    return CTFMM_OK;
}

ctfmm_status narrow_outputs(ctfmm_ctx* c, int64_t n, float* phi, float* grad) {
    if (phi) launch_narrow(c->stream, n, c->io[2], phi);
    if (grad) launch_narrow(c->stream, 3 * n, c->io[3], grad);
    HIPCHK(c, hipGetLastError());
    return CTFMM_OK;
}

}  // namespace

ctfmm_status ctfmm_evaluate_f32(ctfmm_ctx* c, int64_t n, const float* xyz, const float* q, float* phi, float* grad) {
    if (!c) return CTFMM_EINVAL;
    c->err.clear();
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(c, CTFMM_EINVAL, "n out of range");
    if (n == 0) return CTFMM_OK;
    if (!xyz || !q) return fail(c, CTFMM_EINVAL, "null xyz or q");
    SCHK(widen_inputs(c, n, xyz, q));
    SCHK(ctfmm_evaluate(c, n, c->io[0], c->io[1], phi ? c->io[2] : nullptr, grad ? c->io[3] : nullptr));
    return narrow_outputs(c, n, phi, grad);
}

ctfmm_status ctfmm_evaluate_batched_f32(ctfmm_ctx* c, int32_t nsys, const int64_t* offsets, const int32_t* orders,
                                        const float* xyz, const float* q, float* phi, float* grad) {
    if (!c) return CTFMM_EINVAL;
    c->err.clear();
    if (nsys < 1 || !offsets || !orders) return fail(c, CTFMM_EINVAL, "nsys >= 1 and host offsets/orders required");
    const int64_t n = offsets[nsys];
    if (offsets[0] != 0 || n < 0 || n >= (int64_t(1) << 31)) return fail(c, CTFMM_EINVAL, "bad offsets");
    if (n == 0) return CTFMM_OK;
    if (!xyz || !q) return fail(c, CTFMM_EINVAL, "null xyz or q");
    SCHK(widen_inputs(c, n, xyz, q));
    SCHK(ctfmm_evaluate_batched(c, nsys, offsets, orders, c->io[0], c->io[1], phi ? c->io[2] : nullptr,
                                grad ? c->io[3] : nullptr));
    return narrow_outputs(c, n, phi, grad);
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
    double* tmp = (double*)dev_alloc(c, cnt * sizeof(double));
    if (!tmp) return fail(c, CTFMM_ENOMEM, "workspace allocation failed");
    const double* X = (which == 0 ? c->M : c->L) + c->lvl_off[level] * (size_t)ldm_of(p);
    launch_unscale_copy(c->stream, p, level, which, c->prm.root_side, X, tmp);
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipMemcpyAsync(host_out, tmp, cnt * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    hipError_t e3 = hipStreamSynchronize(c->stream);
    dev_release(c, tmp);
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
    for (int k = 0; k < c->nforests; ++k) {
        Forest& f = c->forests[k];
        ctfmm_status s = count_v_pairs(c, f);
        if (s != CTFMM_OK) return s;
        std::vector<int32_t> info((size_t)f.nn);
        HIPCHK(c, hipMemcpyAsync(info.data(), f.tr.info, info.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int32_t v : info) out->leaves += (v >> 8) & 1;
        out->nodes += f.nn;
        out->max_level = std::max<int64_t>(out->max_level, (int64_t)f.lev_first.size() - 1);
        const bool dual = c->prm.tree == CTFMM_TREE_DUAL;
        out->v_pairs += dual ? f.n_m2l : f.v_pairs;
        out->u_pairs += dual ? f.n_p2p : f.tot_u;
        out->w_pairs += f.tot_w;
        out->x_pairs += f.tot_x;
    }
    if (c->nforests > 0) {
        ABox b{};
        HIPCHK(c, hipMemcpy(&b, c->forests[0].boxes, sizeof(ABox), hipMemcpyDeviceToHost));
        for (int k = 0; k < 3; ++k) out->root_lo[k] = b.lo[k];
        out->root_side = b.side;
    }
    return CTFMM_OK;
}

ctfmm_status ctfmm_copy_tree(ctfmm_ctx* c, ctfmm_tree_copy_t* io) {
    if (!c || !io) return CTFMM_EINVAL;
    if (c->prm.tree == CTFMM_TREE_UNIFORM) return fail(c, CTFMM_EUNSUPPORTED, "tree copies need the adaptive tree");
    if (!c->have_result || c->nforests < 1) return fail(c, CTFMM_EINVAL, "no evaluate yet");
    Forest& f = c->forests[0];
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const bool lists = c->prm.tree == CTFMM_TREE_ADAPTIVE;
    const size_t nn = (size_t)f.nn, n1 = nn + 1, nt = f.tiles_host.size(), tt = (size_t)f.tt;
    std::vector<int32_t> tgt, src;
    if (nt > 0 && io->v_pairs) {
        tgt.resize(tt * nt);
        src.resize(189 * tt * nt);
        HIPCHK(c, hipMemcpy(tgt.data(), f.tgt_tab, tgt.size() * 4, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(src.data(), f.src_tab, src.size() * 4, hipMemcpyDeviceToHost));
    }
    SCHK(count_v_pairs(c, f));
    io->nodes = (int64_t)nn;
    io->particles = f.n;
    io->u_len = f.tot_u;
    io->w_len = f.tot_w;
    io->x_len = f.tot_x;
    io->v_len = f.v_pairs;
    auto get = [&](void* dst, const void* from, size_t bytes) -> ctfmm_status {
        if (dst && bytes) HIPCHK(c, hipMemcpy(dst, from, bytes, hipMemcpyDeviceToHost));
        return CTFMM_OK;
    };
    SCHK(get(io->key, f.tr.key, nn * 8));
    SCHK(get(io->parent, f.tr.par, nn * 4));
    SCHK(get(io->pb, f.tr.pb, nn * 4));
    SCHK(get(io->pe, f.tr.pe, nn * 4));
    SCHK(get(io->perm, f.a_idxs, (size_t)f.n * 4));
    if (lists) {
        SCHK(get(io->u_off, f.loff, n1 * 4));
        SCHK(get(io->w_off, f.loff + n1, n1 * 4));
        SCHK(get(io->x_off, f.loff + 2 * n1, n1 * 4));
        SCHK(get(io->u_list, f.ulist, (size_t)f.tot_u * 4));
        SCHK(get(io->w_list, f.wlist, (size_t)f.tot_w * 4));
        SCHK(get(io->x_list, f.xlist, (size_t)f.tot_x * 4));
    } else {
        for (int32_t* o : {io->u_off, io->w_off, io->x_off})
            if (o) std::memset(o, 0, n1 * 4);
    }
    if (io->level || io->leaf) {
        std::vector<int32_t> info(nn);
        SCHK(get(info.data(), f.tr.info, nn * 4));
        for (size_t i = 0; i < nn; ++i) {
            if (io->level) io->level[i] = info[i] & 0xff;
            if (io->leaf) io->leaf[i] = (info[i] >> 8) & 1;
        }
    }
    if (io->v_pairs) {
        int64_t k = 0;
        for (size_t t = 0; t < nt; ++t)
            for (size_t iv = 0; iv < 189; ++iv)
                for (size_t r = 0; r < tt; ++r) {
                    const int32_t a = tgt[t * tt + r], b = src[(189 * t + iv) * tt + r];
                    if (a < 0 || b < 0) continue;
                    if (k >= f.v_pairs) return fail(c, CTFMM_EDEVICE, "M2L tables hold more pairs than counted");
                    io->v_pairs[2 * k] = a;
                    io->v_pairs[2 * k + 1] = b;
                    ++k;
                }
        if (k != f.v_pairs) return fail(c, CTFMM_EDEVICE, "M2L tables hold fewer pairs than counted");
    }
    return CTFMM_OK;
}

ctfmm_status ctfmm_set_order_table(ctfmm_ctx* c, const int32_t* order_r2) {
    if (!c) return CTFMM_EINVAL;
    if (c->prm.tree != CTFMM_TREE_ADAPTIVE) return fail(c, CTFMM_EUNSUPPORTED, "per-pair orders need the adaptive tree");
    if (!order_r2) {
        c->order_mode = 0;
        return CTFMM_OK;
    }
    for (int k = 4; k <= 27; ++k)
        if (order_r2[k] < 0 || order_r2[k] > c->prm.order_p)
            return fail(c, CTFMM_EINVAL, "orders must lie in 0..p for |v|^2 in 4..27");
    if (!c->order_tab) {
        size_t cap = 0;
        if (!grow(c, c->order_tab, cap, 28, false)) return fail(c, CTFMM_ENOMEM, "allocation failed");
    }
    int32_t tab[28];
    std::memcpy(tab, order_r2, sizeof(tab));
    HIPCHK(c, hipMemcpyAsync(c->order_tab, tab, sizeof(tab), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->order_mode = 1;
    return CTFMM_OK;
}

ctfmm_status ctfmm_set_order_hash(ctfmm_ctx* c, uint64_t seed, int32_t pmin) {
    if (!c) return CTFMM_EINVAL;
    if (c->prm.tree != CTFMM_TREE_ADAPTIVE) return fail(c, CTFMM_EUNSUPPORTED, "per-pair orders need the adaptive tree");
    if (pmin < 0 || pmin > c->prm.order_p) return fail(c, CTFMM_EINVAL, "pmin must lie in 0..p");
    c->order_seed = seed;
    c->order_pmin = pmin;
    c->order_mode = 3;
    return CTFMM_OK;
}

ctfmm_status ctfmm_set_mac(ctfmm_ctx* c, double theta, int32_t centre) {
    if (!c) return CTFMM_EINVAL;
    c->err.clear();
    if (c->prm.tree != CTFMM_TREE_DUAL) return fail(c, CTFMM_EUNSUPPORTED, "the MAC belongs to the dual tree");
    if (!(theta >= 0.0 && theta <= 1.0)) return fail(c, CTFMM_EINVAL, "theta outside [0, 1]");
    if (centre < CTFMM_CENTRE_GEOMETRIC || centre > CTFMM_CENTRE_AP) return fail(c, CTFMM_EINVAL, "unknown centre");
    c->theta = theta;
    c->centre = centre;
    return CTFMM_OK;
}

ctfmm_status ctfmm_copy_dual(ctfmm_ctx* c, ctfmm_dual_copy_t* io) {
    if (!c || !io) return CTFMM_EINVAL;
    c->err.clear();
    if (c->prm.tree != CTFMM_TREE_DUAL) return fail(c, CTFMM_EUNSUPPORTED, "traversal copies need the dual tree");
    if (!c->have_result || c->nforests < 1) return fail(c, CTFMM_EINVAL, "no evaluate yet");
    Forest& f = c->forests[0];
    HIPCHK(c, hipStreamSynchronize(c->stream));
    io->nodes = f.nn;
    io->m2l = f.n_m2l;
    io->p2p = f.n_p2p;
    if (io->zr) HIPCHK(c, hipMemcpy(io->zr, f.zr, (size_t)f.nn * sizeof(double4), hipMemcpyDeviceToHost));
    const uint64_t mask = (1ull << f.dual_sh) - 1;
    for (int w = 0; w < 2; ++w) {
        int32_t* out = w == 0 ? io->m2l_pairs : io->p2p_pairs;
        const size_t cnt = w == 0 ? (size_t)f.n_m2l : (size_t)f.n_p2p;
        if (!out || cnt == 0) continue;
        std::vector<uint64_t> k(cnt);
        HIPCHK(c, hipMemcpy(k.data(), w == 0 ? f.mks : f.pks, cnt * 8, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < cnt; ++i) {
            out[2 * i] = (int32_t)(k[i] >> f.dual_sh);
            out[2 * i + 1] = (int32_t)(k[i] & mask);
        }
    }
    return CTFMM_OK;
}

ctfmm_status ctfmm_set_order_model(ctfmm_ctx* c, const float* params, const float* norm, double target_rel_err,
                                   double margin) {
    if (!c) return CTFMM_EINVAL;
    if (c->prm.tree != CTFMM_TREE_ADAPTIVE) return fail(c, CTFMM_EUNSUPPORTED, "per-pair orders need the adaptive tree");
    if (!params) {
        c->order_mode = 0;
        return CTFMM_OK;
    }
    if (c->prm.order_p != 10) return fail(c, CTFMM_EUNSUPPORTED, "the network chooses orders 2..10: use p = 10");
    if (!norm || !(target_rel_err > 0.0) || !std::isfinite(margin)) return fail(c, CTFMM_EINVAL, "bad model arguments");
    for (int k = 0; k < MLP_NIN; ++k)
        if (!(norm[MLP_NIN + k] > 0.f)) return fail(c, CTFMM_EINVAL, "input scales must be positive");
    if (!c->model) {
        size_t cap = 0;
        if (!grow(c, c->model, cap, MLP_NPARAM + 2 * MLP_NIN, false)) return fail(c, CTFMM_ENOMEM, "allocation failed");
    }
    std::vector<float> buf(MLP_NPARAM + 2 * MLP_NIN);
    std::memcpy(buf.data(), params, MLP_NPARAM * sizeof(float));
    std::memcpy(buf.data() + MLP_NPARAM, norm, 2 * MLP_NIN * sizeof(float));
    HIPCHK(c, hipMemcpyAsync(c->model, buf.data(), buf.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->order_thr = (float)(std::log10(target_rel_err) - margin);
    c->order_mode = 2;
    return CTFMM_OK;
}

ctfmm_status ctfmm_mlp_forward(ctfmm_ctx* c, int64_t n, const float* x, const float* params, int32_t precision,
                               float* y) {
    if (!c) return CTFMM_EINVAL;
    if (n < 0 || (n > 0 && (!x || !params || !y)) || (precision != 0 && precision != 1))
        return fail(c, CTFMM_EINVAL, "n >= 0, device x, params, y and precision 0 (FP32) or 1 (FP16)");
    if (precision == 0) launch_mlp_forward32(c->stream, n, x, params, y);
    else launch_mlp_forward16(c->stream, n, x, params, nullptr, y);
    HIPCHK(c, hipGetLastError());
    return CTFMM_OK;
}

ctfmm_status ctfmm_mlp_backward(ctfmm_ctx* c, int64_t n, const float* x, const float* t, const float* params,
                                float* grad, float* loss) {
    if (!c) return CTFMM_EINVAL;
    if (n < 1 || !x || !t || !params || !grad || !loss) return fail(c, CTFMM_EINVAL, "n >= 1 and device pointers");
    if (!grow(c, c->mlp_act, c->mlp_act_cap, (size_t)n * 5 * MLP_NH + mlp_backward_part_floats(n), false) ||
        !grow(c, c->mlp_err, c->mlp_err_cap, (size_t)n, false))
        return fail(c, CTFMM_ENOMEM, "allocation failed");
    launch_mlp_backward(c->stream, n, x, t, params, c->mlp_act, c->mlp_err, grad, loss);
    HIPCHK(c, hipGetLastError());
    return CTFMM_OK;
}

ctfmm_status ctfmm_mlp_backward_noalloc(ctfmm_ctx* c, int64_t n, const float* x, const float* t, const float* params,
                                       float* grad, float* loss) {
    if (!c) return CTFMM_EINVAL;
    if (n < 1 || !x || !t || !params || !grad || !loss) return fail(c, CTFMM_EINVAL, "n >= 1 and device pointers");
    if (n > mlp_noalloc_max())
        return fail(c, CTFMM_EINVAL, "n above the scratch capacity of the allocation-free backward pass (" +
                                         std::to_string(mlp_noalloc_max()) + " samples)");
    HIPCHK(c, launch_mlp_backward_noalloc(c->stream, c->device, n, x, t, params, grad, loss));
    return CTFMM_OK;
}

ctfmm_status ctfmm_mlp_train(ctfmm_ctx* c, int64_t n, const float* x, const float* t, float* params, int32_t steps,
                             int32_t batch, float lr, float* loss_host) {
    if (!c) return CTFMM_EINVAL;
    if (!x || !t || !params || steps < 1 || batch < 1 || batch > n || !(lr > 0.f))
        return fail(c, CTFMM_EINVAL, "1 <= batch <= n, steps >= 1, lr > 0 and device pointers");
    if (!grow(c, c->mlp_act, c->mlp_act_cap, (size_t)batch * 5 * MLP_NH + mlp_backward_part_floats(batch), false) ||
        !grow(c, c->mlp_err, c->mlp_err_cap, (size_t)batch, false) ||
        !grow(c, c->mlp_grad, c->mlp_grad_cap, MLP_NPARAM, false) ||
        !grow(c, c->mlp_m, c->mlp_m_cap, MLP_NPARAM, false) || !grow(c, c->mlp_v, c->mlp_v_cap, MLP_NPARAM, false) ||
        !grow(c, c->mlp_loss, c->mlp_loss_cap, (size_t)steps, false))
        return fail(c, CTFMM_ENOMEM, "allocation failed");
    HIPCHK(c, hipMemsetAsync(c->mlp_m, 0, MLP_NPARAM * sizeof(float), c->stream));
    HIPCHK(c, hipMemsetAsync(c->mlp_v, 0, MLP_NPARAM * sizeof(float), c->stream));
    const int64_t windows = n / batch;
    for (int step = 1; step <= steps; ++step) {
        const int64_t start = ((step - 1) % windows) * batch;
        launch_mlp_backward(c->stream, batch, x + start * MLP_NIN, t + start * MLP_NOUT, params, c->mlp_act,
                            c->mlp_err, c->mlp_grad, c->mlp_loss + (step - 1));
        launch_adam(c->stream, step, lr, params, c->mlp_grad, c->mlp_m, c->mlp_v);
    }
    HIPCHK(c, hipGetLastError());
    if (loss_host) {
        HIPCHK(c, hipMemcpyAsync(loss_host, c->mlp_loss, steps * sizeof(float), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return CTFMM_OK;
}

namespace {

// offset slot of v (2 <= |v|_inf <= 3), or -1
int far_slot(const int32_t* v) {
    const int a = std::abs(v[0]), b = std::abs(v[1]), d = std::abs(v[2]);
    const int m = std::max(a, std::max(b, d));
    if (m < 2 || m > 3) return -1;
    return (v[0] + 3) + 7 * (v[1] + 3) + 49 * (v[2] + 3);
}

}  // namespace

ctfmm_status ctfmm_mlp_labels(ctfmm_ctx* c, int64_t n, const double* M, const int32_t* v_host, float* x, float* y) {
    if (!c) return CTFMM_EINVAL;
    if (c->prm.order_p != 10) return fail(c, CTFMM_EUNSUPPORTED, "training data needs a context of order 10");
    if (n < 0 || (n > 0 && (!M || !v_host || !x || !y))) return fail(c, CTFMM_EINVAL, "bad arguments");
    if (n == 0) return CTFMM_OK;
    std::vector<int32_t> slots((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        slots[i] = far_slot(v_host + 3 * i);
        if (slots[i] < 0) return fail(c, CTFMM_EINVAL, "offsets need 2 <= |v|_inf <= 3");
    }
    if (!grow(c, c->mlp_vs, c->mlp_vs_cap, (size_t)n, false)) return fail(c, CTFMM_ENOMEM, "allocation failed");
    HIPCHK(c, hipMemcpyAsync(c->mlp_vs, slots.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    launch_mlp_labels(c->stream, n, M, 121, nullptr, c->mlp_vs, c->Kt, x, y);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return CTFMM_OK;
}

ctfmm_status ctfmm_mlp_samples(ctfmm_ctx* c, int64_t npart, const double* xyz, const double* q, int64_t nsamp,
                               uint64_t seed, float* x, float* y) {
    if (!c) return CTFMM_EINVAL;
    c->err.clear();
    if (c->prm.tree != CTFMM_TREE_ADAPTIVE || c->prm.order_p != 10)
        return fail(c, CTFMM_EUNSUPPORTED, "training data needs an adaptive context of order 10");
    if (npart < 1 || npart >= (int64_t(1) << 31) || nsamp < 0 || !xyz || !q || (nsamp > 0 && (!x || !y)))
        return fail(c, CTFMM_EINVAL, "bad arguments");
    if (c->forests.empty()) c->forests.resize(1);
    Forest& f = c->forests[0];
    c->nforests = 1;
    f.p = 10;
    f.nsys = 1;
    f.n = (int)npart;
    f.goff_h = {0, (int)npart};
    f.gbase_h = {0};
    const int saved_mode = c->order_mode;
    c->order_mode = 0;
    ctfmm_status s = build_forest(c, f, xyz, q, c->prm.root_side > 0.0);
    c->order_mode = saved_mode;
    if (s != CTFMM_OK) return s;
    const int maxlev = (int)f.lev_first.size() - 1;
    if (maxlev < 2) return fail(c, CTFMM_EINVAL, "the tree has no cells below level 2 to sample");
    launch_p2m_nodes(c->stream, 10, 0, f.nn, f.boxes, f.tr, f.a_P, c->T, f.aM);
    for (int l = maxlev - 1; l >= 2; --l)
        launch_m2m_nodes(c->stream, 10, f.lev_first[l], f.lev_count[l], f.tr, f.aM, c->T);
    if (!grow(c, c->mlp_sel, c->mlp_sel_cap, (size_t)std::max<int64_t>(nsamp, 1), false) ||
        !grow(c, c->mlp_vs, c->mlp_vs_cap, (size_t)std::max<int64_t>(nsamp, 1), false))
        return fail(c, CTFMM_ENOMEM, "allocation failed");
    const int f2 = f.lev_first[2];
    launch_mlp_pick(c->stream, nsamp, seed, f2, f.nn - f2, c->mlp_sel, c->mlp_vs);
    launch_mlp_labels(c->stream, nsamp, f.aM, ldm_of(10), c->mlp_sel, c->mlp_vs, c->Kt, x, y);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->have_result = false;
    return CTFMM_OK;
}

ctfmm_status ctfmm_set_m2l_tile(ctfmm_ctx* c, int32_t p, int32_t targets) {
    if (!c) return CTFMM_EINVAL;
    if (p < 0 || p > CTFMM_P_MAX || (targets != 0 && targets != 32 && targets != 64 && targets != 128))
        return fail(c, CTFMM_EINVAL, "p in 0..10 and targets in {0, 32, 64, 128}");
    if (targets) {
        int max_lds = 0;
        HIPCHK(c, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
        if (m2l_tile_lds_bytes(p, c->prm.precision, targets) > (size_t)max_lds)
            return fail(c, CTFMM_EUNSUPPORTED, "this tile does not fit the device's LDS");
    }
    c->tile_forced[p] = targets;
    return CTFMM_OK;
}

ctfmm_status ctfmm_get_m2l_tile(ctfmm_ctx* c, int32_t p, int32_t* targets) {
    if (!c || !targets || p < 0 || p > CTFMM_P_MAX) return CTFMM_EINVAL;
    *targets = c->tile_forced[p] ? c->tile_forced[p] : c->tile_tuned[p];
    return CTFMM_OK;
}

ctfmm_status ctfmm_set_timing(ctfmm_ctx* c, int32_t on) {
    if (!c) return CTFMM_EINVAL;
    c->timing = on != 0;
    return CTFMM_OK;
}

ctfmm_status ctfmm_stats(ctfmm_ctx* c, ctfmm_stats_t* out) {
    if (!c || !out) return CTFMM_EINVAL;
    SCHK(finish_pending(c));
    *out = c->st;
    return CTFMM_OK;
}

ctfmm_status ctfmm_reset_stats(ctfmm_ctx* c) {
    if (!c) return CTFMM_EINVAL;
    if (c->pend.on) HIPCHK(c, hipEventSynchronize(c->pend.ev[NPHASE_EV - 1]));
    c->pend.on = false;  // an evaluation from before the reset is not counted
    std::memset(&c->st, 0, sizeof(c->st));
    return CTFMM_OK;
}

ctfmm_status ctfmm_sync(ctfmm_ctx* c) {
    if (!c) return CTFMM_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    SCHK(finish_pending(c));
    if (c->err_flag) {
        int h = 0;
        HIPCHK(c, hipMemcpy(&h, c->err_flag, sizeof(int), hipMemcpyDeviceToHost));
        if (h) {
            HIPCHK(c, hipMemset(c->err_flag, 0, sizeof(int)));
            return fail(c, CTFMM_EINVAL, (h & 1) ? "non-finite particle coordinate"
                                                 : "the AP variant needs positive charges");
        }
    }
    return CTFMM_OK;
}

const char* ctfmm_last_error(const ctfmm_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

void ctfmm_destroy(ctfmm_ctx* c) {
    if (!c) return;
    dev_free_all(c);
    reset_adaptive(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (auto& e : c->tev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : c->side_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& x : c->side)
        if (x) (void)hipStreamDestroy(x);
    for (auto& set : c->evs)
        for (auto& e : set)
            if (e) (void)hipEventDestroy(e);
    if (c->pinned) (void)hipHostFree(c->pinned);
    delete c;
}

}  // extern "C"
