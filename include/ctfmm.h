/*
 * ctfmm.h -- C ABI of libctfmm: the Cartesian traceless fast multipole
 * method (Coles & Bieri, "An Optimizing Symbolic Algebra Approach for
 * Generating Fast Multipole Method Operators", arXiv 1811.06332) on AMD
 * Instinct MI355X (gfx950).
 *
 * Problem (Appendix B, Eq. PhiAB; Sec. 2.1, Eq. L2P): given N particles with
 * positions x_a and weights q_a, compute for every particle b
 *     Phi(x_b)      = sum_{a != b} q_a / |x_b - x_a|
 *     grad Phi(x_b) = -sum_{a != b} q_a (x_b - x_a) / |x_b - x_a|^3
 * approximated by the FMM operators P2M, M2M, M2L, L2L, L2P (Sec. 2.1) with
 * a direct near field (Appendix C).  The potential is positive for positive
 * weights (Sec. 2.1); gravitational users negate Phi and grad Phi.  Free
 * space: no periodic images.  A pair at exactly zero distance contributes
 * nothing.  Accuracy is set by the expansion order p and the
 * well-separation rule (Appendix C): here a cell interacts through M2L with
 * the same-level cells that are not adjacent to it but whose parents are
 * adjacent to its parent (ws = 1); adjacent leaves are summed directly.
 *
 * Conventions for every function:
 *   - Pointers named "dev" are device (HIP) memory, "host" host memory.
 *   - The caller owns every buffer it passes; the library never frees them.
 *   - Work is asynchronous on the stream given to ctfmm_create; results are
 *     valid after ctfmm_sync or any later stream-ordered operation.
 *   - Every function returns a ctfmm_status; no exception crosses the ABI
 *     and nothing aborts.  ctfmm_last_error gives a message for the last
 *     failure on a context.
 *   - A context is not thread-safe: use one context per host thread/stream.
 */
#ifndef CTFMM_H
#define CTFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CTFMM_ABI_VERSION 4
/* largest expansion order compiled in */
#define CTFMM_P_MAX 10
/* deepest uniform octree (2^(3*depth) leaves) */
#define CTFMM_DEPTH_MAX 9
/* deepest level of the adaptive octree (63-bit Morton keys) */
#define CTFMM_ADAPTIVE_LEVEL_MAX 21

typedef struct ctfmm_ctx ctfmm_ctx;

typedef enum ctfmm_status {
    CTFMM_OK = 0,
    CTFMM_EINVAL = 1,       /* bad argument: null pointer, n < 0, p < 0, depth out of range,
                               non-finite coordinate (reported by ctfmm_sync) */
    CTFMM_ENOMEM = 2,       /* device allocation failed (or the allocator returned NULL) */
    CTFMM_EDEVICE = 3,      /* a HIP runtime call failed */
    CTFMM_EUNSUPPORTED = 4  /* valid request this build does not implement: p above
                               CTFMM_P_MAX, or a tree, precision or tile the build or
                               the device does not provide */
} ctfmm_status;

typedef enum ctfmm_tree {
    CTFMM_TREE_UNIFORM = 0,  /* uniform octree of the given depth over a cube */
    CTFMM_TREE_ADAPTIVE = 1, /* a node holding more than leaf_max particles is split
                                into its non-empty octants, down to level
                                CTFMM_ADAPTIVE_LEVEL_MAX (Appendix C: geometric
                                splits at the cell centre).  Interactions follow
                                the adaptive lists: V (same-level cells that are
                                not adjacent but whose parents are) by M2L;
                                U (adjacent leaves) by direct summation; W (finer
                                cells not adjacent to a leaf while their parent
                                is) by evaluating their multipole expansion at
                                the leaf's particles; X (the converse of W) by
                                forming the local expansion directly from the
                                coarse leaf's particles. */
    CTFMM_TREE_DUAL = 2      /* the same octree (leaf_max, root cube), driven by
                                the dual-tree traversal of Appendix C: node pairs
                                that satisfy the multipole acceptance criterion
                                theta |z_B - z_A| > r_A + r_B (z the expansion
                                centres, r the enclosing radii) interact by M2L
                                in both directions (Newton's third law holds to
                                rounding); otherwise the node of larger radius is
                                opened; leaf pairs that fail it are summed
                                directly.  theta and the centres are set with
                                ctfmm_set_mac (default 0.5, geometric centres).
                                FP64 only; no batches, no dipoles. */
} ctfmm_tree;

/* Arithmetic of the M2L translation.  Everything else (P2M, M2M, L2L, L2P,
 * P2P, the derivative tensors) is always FP64. */
typedef enum ctfmm_precision {
    CTFMM_PREC_FP64 = 0,        /* FP64 matrix cores, FP64 accumulation */
    CTFMM_PREC_FP32 = 1,        /* FP32 matrix cores, FP32 accumulation */
    CTFMM_PREC_BF16X3 = 2       /* operands split into three BF16 pieces, the six
                                   leading piece products on BF16 matrix cores,
                                   FP32 accumulation */
} ctfmm_precision;

typedef struct ctfmm_params {
    int32_t order_p;    /* expansion order p, 0..CTFMM_P_MAX */
    int32_t tree;       /* ctfmm_tree */
    int32_t depth;      /* leaf level of the uniform octree, 0..CTFMM_DEPTH_MAX
                           (ignored by the adaptive tree) */
    int32_t ws;         /* well-separation in cells; only 1 is supported */
    int32_t precision;  /* ctfmm_precision */
    int32_t leaf_max;   /* adaptive tree: most particles in a leaf (>= 1) */
    double root_lo[3];  /* lower corner of the root cube */
    double root_side;   /* side of the root cube; particles outside are clamped
                           into the boundary cells.  Adaptive tree only:
                           root_side <= 0 selects the automatic cube, centred on
                           the particles' bounding box with side = largest
                           extent * (1 + 2^-20) (1 if all particles coincide) */
} ctfmm_params;

typedef struct ctfmm_stats_t {
    /* accumulated over evaluate calls since the last ctfmm_reset_stats,
       measured with HIP events on the context stream when timing is on */
    double ms_total;        /* whole evaluate calls */
    double ms_tree;         /* keys, sort, leaf ranges (adaptive: also the tree, its lists
                               and the M2L tables) */
    double ms_p2m;
    double ms_m2m;
    double ms_m2l;          /* all M2L launches (adaptive tree: the M2L kernel itself) */
    double ms_l2l;
    double ms_near;         /* L2P + P2P (adaptive tree: L2P and the wait for the near field,
                               whose P2P and W-list multipole evaluations run on a side
                               stream beside the expansion passes) */
    double ms_convert;      /* FP32 copies of the multipoles for the FP32/BF16 M2L modes
                               (adaptive tree: also the weighted multipoles of the W list) */
    double ms_p2l;          /* adaptive tree: the rest of the downward M2L/X-list step (local
                               expansions formed from X-list particles, on a side stream
                               beside M2L where the orders are fixed, the partial-sum
                               clear and sum) */
    double ms_numeric;      /* batched evaluation: every numeric pass (one graph launch) */
    int64_t evaluations;
    int64_t m2l_launches;
    int64_t m2l_pairs;      /* cell pairs translated by M2L, summed over calls */
    int64_t p2p_leaf_pairs; /* leaf pairs of the near field, summed over calls */
    int64_t graph_launches; /* batched evaluations replayed from the captured graph */
    int64_t m2l_order_pairs[CTFMM_P_MAX + 1]; /* adaptive tree with timing on: M2L pairs per
                               order actually used (the chosen-order histogram) */
} ctfmm_stats_t;

/* Shape of the tree and interaction lists built by the last evaluate. */
typedef struct ctfmm_tree_stats_t {
    int64_t nodes;      /* tree nodes, root included */
    int64_t leaves;
    int64_t max_level;
    int64_t v_pairs;    /* M2L (target, source) cell pairs */
    int64_t u_pairs;    /* near-field (target leaf, source leaf) pairs, self included */
    int64_t w_pairs;    /* (target leaf, source cell) multipole evaluations */
    int64_t x_pairs;    /* (target cell, source leaf) direct local expansions */
    double root_lo[3];
    double root_side;
} ctfmm_tree_stats_t;

/* ABI version (CTFMM_ABI_VERSION). */
int ctfmm_version(void);

/* Fill *prm with defaults: p = 4, uniform tree, depth 3, ws = 1, FP64,
 * leaf_max 64, root cube [0,1)^3.  Returns CTFMM_EINVAL if prm is NULL. */
ctfmm_status ctfmm_default_params(ctfmm_params* prm);

/* Create a context on the current HIP device, bound to hip_stream (a
 * hipStream_t; NULL = the null stream).  Builds the per-offset M2L operator
 * matrices for the requested p and precision: for each integer offset v of
 * the ws = 1 lists, the linear map of Eq. M2L (Sec. 2.1) from the
 * independent multipole components to the independent local components,
 * with D(v) from Eq. traceless grad and Eq. Detracer3 (Appendix A).  *out
 * receives the context (owned by the library; release with ctfmm_destroy).
 * Errors: EINVAL (null prm/out, p < 0, depth or ws out of range, root_side
 * <= 0 or not finite), EUNSUPPORTED (p > CTFMM_P_MAX, tree or precision
 * unknown), ENOMEM, EDEVICE. */
ctfmm_status ctfmm_create(const ctfmm_params* prm, void* hip_stream, ctfmm_ctx** out);

/* Route every device workspace allocation through alloc/free (called with
 * the user pointer and the context stream; frees are stream-ordered on that
 * stream, so a caching allocator bound to it may hand the memory out again
 * to later work on the stream).  Buffers already held are released first
 * and the operator tables rebuilt through the new allocator.  NULL alloc
 * restores hipMalloc/hipFree.  An alloc returning NULL makes the call that
 * needed memory fail with ENOMEM (this one included: the tables are
 * rebuilt here).  The Python binding routes it to torch's caching
 * allocator. */
typedef void* (*ctfmm_alloc_fn)(size_t bytes, void* user, void* hip_stream);
typedef void (*ctfmm_free_fn)(void* ptr, void* user, void* hip_stream);
ctfmm_status ctfmm_set_allocator(ctfmm_ctx* ctx, ctfmm_alloc_fn alloc, ctfmm_free_fn free_fn, void* user);

/* Potential and gradient of n particles: Phi_b = sum_{a != b} q_a / |x_b -
 * x_a| and its gradient (Appendix B, Eq. PhiAB; Sec. 2.1, Eq. L2P), by the
 * FMM of Appendix C: P2M (Eq. P2M), M2M (Eq. M2M), M2L (Eq. M2L), L2L (Eq.
 * L2L), L2P (Eq. L2P) and the direct near field.  With the adaptive tree
 * the call builds the tree and its lists on the device and waits for the
 * stream a few times while doing so (the sizes of each level decide the
 * next launches); the numeric passes that follow are asynchronous.
 *   xyz  dev, n*3 doubles, row-major (x0,y0,z0,x1,...)
 *   q    dev, n doubles
 *   phi  dev, n doubles, may be NULL (not written)
 *   grad dev, n*3 doubles row-major, may be NULL
 * Outputs are in input order.  n = 0 is a no-op.  n must be < 2^31.
 * The workspace grows to fit n and is kept for later calls. */
ctfmm_status ctfmm_evaluate(ctfmm_ctx* ctx, int64_t n, const double* xyz, const double* q,
                            double* phi, double* grad);

/* ctfmm_evaluate with point dipoles beside the charges (uniform tree): the
 * potential and gradient at every particle of the charges q_a and dipoles
 * d_a of all the others,
 *     Phi(x_b) = sum_{a != b} [ q_a / |r| + d_a . r / |r|^3 ],  r = x_b - x_a,
 * a dipole being the limit of two opposite charges infinitely close
 * (Appendix B.1).  P2M forms each dipole's multipole as a pure dipole at
 * the particle moved to the cell centre by Eq. M2M; the near field adds the
 * dipole pair terms.
 *   dip  dev, n*3 doubles row-major (d_x, d_y, d_z per particle)
 * Other arguments as ctfmm_evaluate.  Errors as ctfmm_evaluate, and
 * EUNSUPPORTED (adaptive tree). */
ctfmm_status ctfmm_evaluate_dipoles(ctfmm_ctx* ctx, int64_t n, const double* xyz, const double* q,
                                    const double* dip, double* phi, double* grad);

/* ctfmm_evaluate with FP32 inputs and outputs (same layouts, float
 * instead of double).  The inputs are widened to FP64 on the device, the
 * method runs as in ctfmm_evaluate (its M2L in the context's precision),
 * and the outputs are rounded to FP32.  The FP64 copies (56 bytes per
 * particle) are workspace kept for later calls.  Errors as
 * ctfmm_evaluate. */
ctfmm_status ctfmm_evaluate_f32(ctfmm_ctx* ctx, int64_t n, const float* xyz, const float* q, float* phi,
                                float* grad);

/* Potential and gradient of nsys independent systems in one call (adaptive
 * tree only).  System s is particles offsets[s] .. offsets[s+1]-1 of the
 * concatenated arrays (same layouts as ctfmm_evaluate) and is expanded to
 * order orders[s] (0..CTFMM_P_MAX) in its own automatic root cube; systems
 * never interact.  Systems of one order share every launch: the trees of
 * all of them form one forest, built on the device (the call waits for the
 * stream once per tree level and a few times more), and one M2L launch
 * serves every level of every system of that order.  The numeric passes of
 * all forests are replayed from a captured HIP graph when the launch
 * signature (sizes and buffers) equals that of the previous call, and run
 * eagerly (then captured on the next call) when it changed.
 *   offsets  host, nsys+1 int64, offsets[0] = 0, non-decreasing, total < 2^31
 *   orders   host, nsys int32
 * Outputs are in input order.  Timing reports ms_total, ms_tree (keys,
 * trees, lists) and ms_numeric.  Errors: EINVAL (bad offsets or orders,
 * null pointers), EUNSUPPORTED (uniform tree), ENOMEM, EDEVICE. */
ctfmm_status ctfmm_evaluate_batched(ctfmm_ctx* ctx, int32_t nsys, const int64_t* offsets, const int32_t* orders,
                                    const double* xyz, const double* q, double* phi, double* grad);

/* ctfmm_evaluate_batched with FP32 inputs and outputs, widened and rounded
 * as in ctfmm_evaluate_f32.  Errors as ctfmm_evaluate_batched. */
ctfmm_status ctfmm_evaluate_batched_f32(ctfmm_ctx* ctx, int32_t nsys, const int64_t* offsets, const int32_t* orders,
                                        const float* xyz, const float* q, float* phi, float* grad);

/* Copy the expansions of one level of the last evaluate to host memory:
 * which = 0 for the multipoles M (Eq. P2M, Eq. M2M), 1 for the local
 * expansions L (Eq. M2L, Eq. L2L).  The
 * values are the physical (unscaled) traceless components M_n, L_n with
 * n_z in {0,1} ((p+1)^2 per cell, ordered by rank, then n_z, then n_x
 * descending); cells row-major with x fastest (index ix + 2^l (iy + 2^l iz)).
 * host_out must hold 8^level * (p+1)^2 doubles (cap, in doubles).
 * Synchronises the stream.  Errors: EINVAL (level outside 2..depth, cap too
 * small, no evaluate yet), EUNSUPPORTED (adaptive tree), EDEVICE. */
ctfmm_status ctfmm_copy_expansions(ctfmm_ctx* ctx, int32_t level, int32_t which, double* host_out,
                                   size_t cap);

/* Tree and list sizes of the last evaluate (synchronises the stream).
 * Errors: EINVAL (null argument, no evaluate yet), EDEVICE. */
ctfmm_status ctfmm_tree_stats(ctfmm_ctx* ctx, ctfmm_tree_stats_t* out);

/* The adaptive tree and its interaction lists as built by the last
 * evaluate (a batch: the forest of its first order), copied to host memory
 * so that they can be compared entry by entry (Appendix C builds the same
 * objects: the tree, and for every cell the cells it interacts with and
 * how).  Every call writes the six sizes; each array the caller sets (non
 * NULL) is filled and must hold the size it is documented with.  Nodes are
 * numbered level by level, in Morton order within a level.
 *   key[nodes]     Morton prefix of the node's cell at its level (3 * level
 *                  bits, x in the lowest bit of each triple)
 *   level, leaf, parent (-1 for roots), pb, pe [nodes]: the node's sorted
 *                  particle range [pb, pe)
 *   perm[particles] input index of the particle at sorted position s
 *   u_off, w_off, x_off [nodes+1] and u_list, w_list, x_list: the U, W and X
 *                  list of node i in L_list[L_off[i] .. L_off[i+1])
 *   v_pairs[v_len][2] (target, source) of every M2L pair
 * Synchronises the stream.  Errors: EINVAL (null io, no adaptive evaluate
 * yet), EUNSUPPORTED (uniform tree), ENOMEM, EDEVICE.  The dual tree has no
 * U/V/W/X lists (their lengths are 0). */
typedef struct ctfmm_tree_copy_t {
    int64_t nodes, particles, u_len, v_len, w_len, x_len;
    uint64_t* key;
    int32_t *level, *leaf, *parent, *pb, *pe;
    int32_t* perm;
    int32_t *u_off, *u_list, *w_off, *w_list, *x_off, *x_list;
    int32_t* v_pairs;
} ctfmm_tree_copy_t;
ctfmm_status ctfmm_copy_tree(ctfmm_ctx* ctx, ctfmm_tree_copy_t* io);

/* M2L tile shape of the adaptive tree for order p (a scheduling choice with
 * no counterpart in the paper; results do not depend on it beyond
 * rounding): targets per workgroup
 * tile, 32, 64 or 128 (one 16-target block per wavefront).  By default
 * (targets = 0) the first evaluation that needs order p times every shape
 * the device's LDS admits on its own tables and keeps the fastest for the
 * context's lifetime.  Errors: EINVAL (p or targets out of range),
 * EUNSUPPORTED (the tile does not fit the device's LDS). */
ctfmm_status ctfmm_set_m2l_tile(ctfmm_ctx* ctx, int32_t p, int32_t targets);

/* The tile shape in use for order p (0 if none has been chosen yet). */
ctfmm_status ctfmm_get_m2l_tile(ctfmm_ctx* ctx, int32_t p, int32_t* targets);

/* ---- M2L order per interaction (adaptive tree) ----
 *
 * By default every M2L (V-list) pair uses the context order p.  Two other
 * rules choose an order p' <= p per pair; M2L of a pair is then Eq. M2L
 * truncated at |n| + |m| <= p' (the order-p' operator acting on the order-p
 * expansions; the truncation rule is that of Sec. 2.1), and every other
 * operator keeps order p.  The M2L tile of a group of same-level targets
 * (one octant, up to 128 of them) at one offset runs at the largest order
 * chosen for its pairs, so no pair gets less than its rule asks for; one
 * M2L launch serves every order.  Per-pair orders apply to the systems
 * whose order is the context's (others of a batch keep their own order). */

/* Order by separation: order_r2 (host, 28 ints) gives the order of a pair
 * whose integer cell offset v has |v|^2 = k (4 <= k <= 27 occur); entries
 * must lie in 0..p.  NULL restores the fixed order.  Errors: EINVAL,
 * EUNSUPPORTED (uniform tree). */
ctfmm_status ctfmm_set_order_table(ctfmm_ctx* ctx, const int32_t* order_r2);

/* ---- dual-tree traversal (tree CTFMM_TREE_DUAL, Appendix C) ---- */

typedef enum ctfmm_centre {
    CTFMM_CENTRE_GEOMETRIC = 0,  /* expansions about each cube's centre */
    CTFMM_CENTRE_MASS = 1,       /* about the charge-weighted mean of the node's
                                    particles (the cube's centre where the node's
                                    total charge is not positive) */
    CTFMM_CENTRE_AP = 2          /* the AP variant (Sec. 4): about the centre of
                                    mass, the dipole (which vanishes there) left
                                    out of every M2L, the gradient only; every
                                    charge must be positive (else ctfmm_evaluate
                                    returns EINVAL) and phi must be NULL */
} ctfmm_centre;

/* The acceptance parameter theta (0 <= theta <= 1; 0 accepts no pair, which
 * is the direct sum) and the expansion centres (ctfmm_centre) of the
 * dual-tree traversal.  The enclosing radius of a node is the largest
 * distance from its centre to one of its particles.  Errors: EINVAL (theta
 * outside [0, 1], unknown centre), EUNSUPPORTED (other trees). */
ctfmm_status ctfmm_set_mac(ctfmm_ctx* ctx, double theta, int32_t centre);

/* The traversal's result of the last evaluation (host buffers, each may be
 * NULL; sizes are always written): zr [nodes][4] = centre and enclosing
 * radius per node (node numbers as ctfmm_copy_tree), m2l [m2l][2] the
 * directed M2L entries (target, source) in ascending order, p2p [p2p][2] the
 * ordered direct leaf pairs (leaf, partner; a leaf with itself once) in
 * ascending order.  Synchronises the stream.  Errors: EINVAL (null io, no
 * evaluation yet), EUNSUPPORTED (other trees), EDEVICE. */
typedef struct ctfmm_dual_copy_t {
    int64_t nodes, m2l, p2p;
    double* zr;
    int32_t* m2l_pairs;
    int32_t* p2p_pairs;
} ctfmm_dual_copy_t;
ctfmm_status ctfmm_copy_dual(ctfmm_ctx* ctx, ctfmm_dual_copy_t* io);

/* Orders from a reproducible map of (source cell, distance class), to check
 * the per-pair-order machinery (the per-tile maximum, the operators of
 * every order, the single M2L launch) against an independent
 * implementation with the same map: the order of source cell C (Morton
 * prefix key, level l, system s of a batch, 0 for a single system) in
 * distance class k (0..14, the occupied |v|^2 values 4, 5, 6, 8, 9, 10,
 * 11, 12, 13, 14, 17, 18, 19, 22, 27 in that order) is pmin + h mod (p -
 * pmin + 1), h = S(S(S(seed ^ key) ^ l) ^ (16 s + k)), S the SplitMix64
 * output function (increment 0x9E3779B97F4A7C15, then z ^= z >> 30,
 * z *= 0xBF58476D1CE4E5B9, z ^= z >> 27, z *= 0x94D049BB133111EB,
 * z ^= z >> 31).  Errors: EINVAL (pmin outside 0..p), EUNSUPPORTED
 * (uniform tree). */
ctfmm_status ctfmm_set_order_hash(ctfmm_ctx* ctx, uint64_t seed, int32_t pmin);

/* The expansion-order network: 12 inputs -> 64 -> 64 -> 9 outputs, ReLU
 * after both hidden layers.  Parameters are CTFMM_MLP_NPARAM floats in this
 * order: W1[64][12], b1[64], W2[64][64], b2[64], W3[9][64], b3[9]
 * (row-major, y = W x + b per layer).  Output k predicts log10 of the
 * relative field error of M2L truncated at order k + 2 for one (source
 * cell, separation) pair; the inputs are |v| / (sqrt(3)/2) and, for ranks
 * n = 0..10, log10 of the 2-norm of the source's rank-n multipole
 * components relative to the largest rank norm. */
#define CTFMM_MLP_NIN 12
#define CTFMM_MLP_NOUT 9
#define CTFMM_MLP_NPARAM 5577

/* Choose orders with the network (context order must be 10): for every
 * (source cell, |v|^2 class) the inputs are standardised with norm (host,
 * 24 floats: mean[12], then std[12] > 0), the network runs in FP16 on the
 * matrix cores, and the order is the smallest p' whose prediction is at
 * most log10(target_rel_err) - margin, else 10 (the fixed order is the
 * fallback).  params (host) NULL restores the fixed order.  Errors: EINVAL,
 * EUNSUPPORTED (uniform tree, or p != 10). */
ctfmm_status ctfmm_set_order_model(ctfmm_ctx* ctx, const float* params, const float* norm, double target_rel_err,
                                   double margin);

/* Network forward pass on n samples: x dev [n][12], params dev, y dev
 * [n][9]; precision 0 = FP32, 1 = FP16 operands with FP32 accumulation on
 * the matrix cores.  Asynchronous.  Errors: EINVAL. */
ctfmm_status ctfmm_mlp_forward(ctfmm_ctx* ctx, int64_t n, const float* x, const float* params, int32_t precision,
                               float* y);

/* Gradient of the mean squared error mean_{b,k} (y_bk - t_bk)^2 over n >= 1
 * samples (x dev [n][12], t dev [n][9]) with respect to params (dev): grad
 * dev [CTFMM_MLP_NPARAM], loss dev [1].  FP32, summed in a fixed order.
 * Asynchronous.  Errors: EINVAL, ENOMEM. */
ctfmm_status ctfmm_mlp_backward(ctfmm_ctx* ctx, int64_t n, const float* x, const float* t, const float* params,
                                float* grad, float* loss);

/* ctfmm_mlp_backward for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, with their scratch (activations and
 * per-chunk partial sums, about 5.6 MB) in a fixed device array of the
 * library, one per GPU, held until the process ends; no allocation of any
 * kind.  n may not exceed 4096.  Every call on one GPU uses that GPU's
 * array: calls that overlap in time on one GPU (other streams, other
 * contexts, other host threads) race and give wrong results.  The array's
 * address is looked up when a context is created on the device.
 * Asynchronous.  Errors: EINVAL (n < 1, n > 4096, null pointer), EDEVICE. */
ctfmm_status ctfmm_mlp_backward_noalloc(ctfmm_ctx* ctx, int64_t n, const float* x, const float* t,
                                       const float* params, float* grad, float* loss);

/* Adam training (beta 0.9, 0.999, eps 1e-8, step lr) of params (dev, in
 * place) for `steps` steps, step s using samples ((s-1) mod (n/batch)) *
 * batch .. + batch - 1 of x, t (dev).  loss_host (may be NULL) receives the
 * loss of every step.  Synchronises when loss_host is given.  Errors:
 * EINVAL, ENOMEM. */
ctfmm_status ctfmm_mlp_train(ctfmm_ctx* ctx, int64_t n, const float* x, const float* t, float* params, int32_t steps,
                             int32_t batch, float lr, float* loss_host);

/* Inputs and targets of the network for n given pairs (context order 10):
 * M dev [n][121] scaled order-10 multipoles of cells of side 1 (the
 * library's independent components), v_host [n][3] integer offsets target -
 * source with 2 <= |v|_inf <= 3.  x dev [n][12]; y dev [n][9] with
 * y_k = log10(max(e, 1e-15)), e the relative 2-norm difference of (phi,
 * grad phi) at the eight points (+-3/8)^3 of the target cell between M2L
 * truncated at order k + 2 and at order 10 (both evaluated by order-10 L2P).
 * Synchronises.  Errors: EINVAL, EUNSUPPORTED (p != 10). */
ctfmm_status ctfmm_mlp_labels(ctfmm_ctx* ctx, int64_t n, const double* M, const int32_t* v_host, float* x, float* y);

/* Training pairs drawn from a particle system (adaptive context of order
 * 10): builds its tree and multipoles, then sample i takes a cell of level
 * >= 2 and a far offset chosen by a counter-based hash of (seed, i), and
 * writes its inputs and targets as ctfmm_mlp_labels.  x, y dev.
 * Synchronises.  Errors: EINVAL (no cell below level 2), EUNSUPPORTED. */
ctfmm_status ctfmm_mlp_samples(ctfmm_ctx* ctx, int64_t npart, const double* xyz, const double* q, int64_t nsamp,
                               uint64_t seed, float* x, float* y);

/* Turn per-phase HIP-event timing on (1) or off (0; default).  The phases
 * are the operators of Sec. 2.1 and the tree and list construction. */
ctfmm_status ctfmm_set_timing(ctfmm_ctx* ctx, int32_t on);

/* Accumulated statistics (synchronises the stream when timing is on). */
ctfmm_status ctfmm_stats(ctfmm_ctx* ctx, ctfmm_stats_t* out);
ctfmm_status ctfmm_reset_stats(ctfmm_ctx* ctx);

/* Wait for the context stream; reports device-side argument errors (a
 * non-finite coordinate gives EINVAL) and HIP errors (EDEVICE). */
ctfmm_status ctfmm_sync(ctfmm_ctx* ctx);

/* Message of the last failure on ctx ("" if none); ctx may be NULL for
 * failures of ctfmm_create.  Valid until the next call on ctx. */
const char* ctfmm_last_error(const ctfmm_ctx* ctx);

/* Release the context and every buffer it allocated.  NULL is a no-op. */
void ctfmm_destroy(ctfmm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* CTFMM_H */
