/*
 * nif.h - C ABI of the MI355X neural visibility library (libnif.so).
 *
 * The library answers shadow-ray visibility queries with a Neural
 * Intersection Function (Fujieda, Kao, Harada, HPG 2023): for each
 * (ray, object) pair it clips the ray against the object's AABB (Sec. 2 end,
 * Sec. 3.1), encodes the entry point, exit point and direction with learned
 * multi-resolution grids (Sec. 3.1, Fig. 2), and evaluates a small MLP with a
 * sigmoid output giving the probability that the ray is NOT occluded by that
 * object (Sec. 3, Eq. (1); Sec. 5 "Architecture").  It also provides the
 * training step (Sec. 4.2, Sec. 5 "Training": joint optimisation of latents
 * and weights with Adam) and a plain BVH any-hit kernel for labels and for
 * the comparison the paper makes (Sec. 6 "Performance Evaluation").
 *
 * Conventions shared by every entry point:
 *  - Pointers marked (dev) are device memory owned by the caller; (host) are
 *    host memory read during the call only.  `stream` is a hipStream_t (NULL =
 *    the default stream).  Work is enqueued asynchronously on `stream`; the
 *    call returns before it completes.
 *  - Every call returns nif_status.  Argument errors (NULL pointer, n < 0,
 *    unsupported shape, workspace too small, unprepared context) are detected
 *    on the host before anything is enqueued; nif_last_error() then holds a
 *    thread-local message.  n == 0 is a successful no-op.
 *  - Per-query domain errors never fail a call: a non-finite origin or
 *    direction, a zero direction, t_max NaN or negative, or an object id
 *    outside [0, num_objects) give visibility = NaN.
 *  - The context owns host metadata and small device tables that it
 *    allocates itself (object table, packed weights per dtype, FP8 scales, the
 *    error word, box groups, training pointer tables and the binary32 weight
 *    images of the MLP being trained: kilobytes per object or MLP).  Grids,
 *    query images, master weights, gradients, optimiser state, inputs, outputs
 *    and workspaces are the caller's.  No C++ exception crosses this interface.
 */
#ifndef NIF_H
#define NIF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NIF_OK = 0,
    NIF_ERR_INVALID_ARG = -1, /* NULL pointer, negative size, id out of range */
    NIF_ERR_UNSUPPORTED = -2, /* model shape or dtype the kernels do not cover */
    NIF_ERR_WORKSPACE = -3,   /* workspace smaller than nif_workspace_bytes */
    NIF_ERR_HIP = -4,         /* a HIP runtime call failed */
    NIF_ERR_STATE = -5        /* context not prepared for the requested dtype */
} nif_status;

typedef enum { NIF_F32 = 0, NIF_F16 = 1, NIF_BF16 = 2, NIF_FP8_E4M3 = 3 } nif_dtype;

/* Model shape.  Grids: for each of the 3 encoded quantities (entry point,
 * exit point, direction) `levels` dense 3D tables; level l has
 * N_l = round(res_min * (res_max/res_min)^(l/(levels-1))) cells per axis and
 * (N_l+1)^3 vertices of `feats` latents, stored as grid_dtype (NIF_F32 or
 * NIF_F16; the paper keeps latents in half, Sec. 5 "Memory Footprint").
 * MLP: input 3*levels*feats, `hidden_layers` hidden layers of `width`, one
 * sigmoid output (Sec. 5 "Architecture").  The hidden activation is ReLU and
 * there are no biases: both are this library's choices for this network
 * family (the paper uses leaky ReLU, see nif_paper_*, and does not mention
 * biases).
 * Supported by the kernels: feats = 2, width = 64, levels in {4, 8},
 * 1 <= hidden_layers <= 8, res_max <= 1024. */
typedef struct {
    int32_t levels, res_min, res_max, feats;
    int32_t grid_dtype;
    int32_t hidden_layers, width;
} nif_model_desc;

typedef struct nif_ctx nif_ctx;

/* Create a context for `num_objects` objects sharing `num_mlps` MLPs
 * (num_mlps = 1 is the paper's single shared network, Sec. 4.1; one MLP per
 * object is the per-object variant).  *out receives the context. */
nif_status nif_create(const nif_model_desc* desc, int32_t num_objects, int32_t num_mlps, nif_ctx** out);
void nif_destroy(nif_ctx* ctx);

/* Parameter layout.  grid_elems: latents per object (one buffer per object,
 * tables in order entry/exit/direction x level, each vertex-major
 * ((z (N+1) + y) (N+1) + x) * feats + f).  table_offsets (host, 3*levels+1
 * entries, nullable): element offset of each table.  level_res (host, levels
 * entries, nullable).  mlp_params: weights per MLP, flat row-major
 * [W1 (width x din)][W2..WH (width x width)][w_out (width)]. */
nif_status nif_param_layout(const nif_ctx* ctx, int64_t* grid_elems, int64_t* table_offsets, int32_t* level_res,
                            int64_t* mlp_params);

/* Register object `obj`: its AABB (host, lo xyz then hi xyz; hi > lo on every
 * axis), its grid buffer (dev, grid_elems latents of grid_dtype) and the MLP
 * it uses.  Takes effect at the next nif_prepare.  grid may be NULL once the
 * object's query image is built (NIF_OPT_GRID_IMAGE 1 or 2, nif_build_image or
 * nif_prepare), else NIF_ERR_STATE: the object is then answered from its
 * image alone and its grid buffer may be freed, so that the images of many
 * objects fit where their grids and images together would not.  Such an
 * object keeps its image until a new grid, a new image buffer or another
 * image mode is set; training calls and nif_init_grid refuse a context with
 * such an object, and nif_encode and nif_calibrate_fp8 while its images are
 * not built (NIF_ERR_STATE). */
nif_status nif_set_object(nif_ctx* ctx, int32_t obj, const float* aabb, void* grid, int32_t mlp_index);

/* Register MLP `mlp`: binary32 master weights (dev, mlp_params floats).  The
 * binary32 path and the training step read them in place; reduced-precision
 * paths read the copy made by nif_prepare. */
nif_status nif_set_mlp(nif_ctx* ctx, int32_t mlp, float* weights);

/* FP8 E4M3 scales of MLP `mlp` (host, 2*hidden_layers floats): s_W for layers
 * 1..H, then s_x for the inputs of layers 1..H.  Layer j computes
 * s_W s_x (Q(W_j / s_W) . Q(h_{j-1} / s_x)) with Q = round to E4M3,
 * saturating at 448, accumulated in binary32. */
nif_status nif_set_fp8_scales(nif_ctx* ctx, int32_t mlp, const float* scales);

/* Scenes of several objects (Sec. 4.1: a top-level pass finds the objects
 * whose AABB a shadow ray meets; each such (ray, object) pair is one query; a
 * ray is visible iff all its pairs are, and a ray with no pair is visible).
 * nif_expand_pairs: for n_rays rays (dev, n x 6 floats) with t_max (dev),
 *   traverses a two-level box tree over the registered objects' AABBs (built
 *   by nif_prepare; 64-wide nodes, one wavefront per node, culled by the
 *   bounds of 64 consecutive rays, so rays given in a coherent order such as
 *   pixel order traverse fastest), decides every candidate box with the
 *   query's binary32 segment rule, and writes the pairs in ray order, objects
 *   ascending (the same pairs as testing every box for every ray): pair_rays (dev,
 *   max_pairs x 6 floats, a copy of the ray), pair_tmax, pair_ids (object),
 *   pair_ray (source ray index).  *pair_count (dev, int64) receives the number
 *   of pairs, also when it exceeds max_pairs (then only the first max_pairs
 *   are written: call again with more room).  Invalid rays (non-finite,
 *   zero direction, t_max NaN or negative) have no pairs.  n_rays <= 2^24 and
 *   n_rays x num_objects < 2^32 (else NIF_ERR_UNSUPPORTED).  Needs
 *   nif_prepare; ws: nif_pairs_workspace_bytes(ctx, n_rays) bytes (dev).
 * nif_combine_pairs: ray_visible (dev, n_rays bytes) = 0 iff some pair p of
 *   the ray (pair_ray[p], dev) has visibility[p] < 0.5 (dev), else 1. */
size_t nif_pairs_workspace_bytes(const nif_ctx* ctx, int64_t n_rays);
nif_status nif_expand_pairs(nif_ctx* ctx, const float* rays, const float* t_max, int64_t n_rays, int64_t max_pairs,
                            float* pair_rays, float* pair_tmax, int32_t* pair_ids, uint32_t* pair_ray,
                            int64_t* pair_count, void* ws, size_t ws_bytes, void* stream);
nif_status nif_combine_pairs(nif_ctx* ctx, const uint32_t* pair_ray, const float* visibility, int64_t n_pairs,
                             int64_t n_rays, uint8_t* ray_visible, void* stream);

/* The top-level pass of Sec. 4.1 feeding the query stage directly:
 * nif_expand_pairs_packed is nif_expand_pairs with the pairs written as the
 * query records that nif_query_packed reads:
 *   packed (dev, max_pairs x 8 floats, 16-byte aligned) row p = {ox, oy, oz,
 *   dx, dy, dz, t_max, object id (int32 bit pattern)}, pair_ray as in
 *   nif_expand_pairs, and keys (dev, max_pairs uint32, nullable) the
 *   ordering key of each pair: (object id, Morton code of the binary32 AABB
 *   entry point), the key nif_order and nif_order_packed compute for it;
 *   when the ordering reads only the object (NIF_OPT_ORDER_BITS 0, window
 *   sort off), its Morton part is left zero.
 *   Same pairs, order, counts, limits and workspace as nif_expand_pairs.
 * nif_order_keys: the ordering (as nif_order) of n queries from their keys
 *   (dev, n uint32, as written by nif_expand_pairs_packed), without reading
 *   the queries: perm (dev, n uint32); ws: nif_order_workspace_bytes(ctx, n).
 *   Keys must come from nif_expand_pairs_packed on the same context (the
 *   object count fixes their layout); NIF_OPT_WINDOW_SORT applies as for
 *   nif_order.
 * A scene step is then nif_expand_pairs_packed, nif_order_keys,
 * nif_query_packed and nif_combine_pairs, each pass reading what the one
 * before wrote once.
 * nif_expand_pairs_by_object: the same records, grouped by object as the
 *   top-level stage of Sec. 4.1 appends each object's inputs (objects
 *   ascending, rays ascending within an object), for at most 64 objects (else
 *   NIF_ERR_UNSUPPORTED): packed and pair_ray as in nif_expand_pairs_packed,
 *   obj_offsets (dev, num_objects + 1 int64, nullable) the first pair of each
 *   object and the total.  No ordering pass is needed: nif_query_packed reads
 *   the records with a NULL perm.  Counts, limits and workspace as
 *   nif_expand_pairs. */
nif_status nif_expand_pairs_packed(nif_ctx* ctx, const float* rays, const float* t_max, int64_t n_rays,
                                   int64_t max_pairs, float* packed, uint32_t* pair_ray, uint32_t* keys,
                                   int64_t* pair_count, void* ws, size_t ws_bytes, void* stream);
nif_status nif_order_keys(nif_ctx* ctx, const uint32_t* keys, int64_t n, uint32_t* perm, void* ws, size_t ws_bytes,
                          void* stream);
nif_status nif_expand_pairs_by_object(nif_ctx* ctx, const float* rays, const float* t_max, int64_t n_rays,
                                      int64_t max_pairs, float* packed, uint32_t* pair_ray, int64_t* pair_count,
                                      int64_t* obj_offsets, void* ws, size_t ws_bytes, void* stream);

/* The early-out form (Sec. 7: once one object is found to occlude a ray, its
 * other objects need not be queried), in two rounds over the same rays:
 * nif_expand_pairs_round with round = 1 writes each ray's first pair only, the
 *   box the ray enters first (smallest t_a, ties to the smaller object id);
 *   query them and combine with nif_combine_pairs.
 * round = 2 writes the other pairs of the rays whose ray_visible (dev, n_rays
 *   bytes, from round 1) is non-zero; query them and combine with
 *   nif_combine_pairs_and, which only clears ray_visible[r] for a pair below
 *   0.5 (no reset to 1).
 * The per-ray result equals nif_combine_pairs over all of nif_expand_pairs'
 * pairs.  Other arguments, order and limits as nif_expand_pairs. */
nif_status nif_expand_pairs_round(nif_ctx* ctx, const float* rays, const float* t_max, int64_t n_rays, int32_t round,
                                  const uint8_t* ray_visible, int64_t max_pairs, float* pair_rays, float* pair_tmax,
                                  int32_t* pair_ids, uint32_t* pair_ray, int64_t* pair_count, void* ws,
                                  size_t ws_bytes, void* stream);
nif_status nif_combine_pairs_and(nif_ctx* ctx, const uint32_t* pair_ray, const float* visibility, int64_t n_pairs,
                                 int64_t n_rays, uint8_t* ray_visible, void* stream);

/* Domain-error bits OR-ed together by every nif_query, nif_query_ordered,
 * nif_encode and plan launch of this context since the last clear: queries
 * whose output is NaN.  NIF_FLAG_INVALID_RAY: non-finite origin or direction,
 * zero direction, or t_max NaN or negative; NIF_FLAG_BAD_OBJECT: object id
 * outside [0, num_objects).  flags (host) receives the word; clear != 0 resets
 * it.  Synchronises `stream`. */
enum { NIF_FLAG_INVALID_RAY = 1, NIF_FLAG_BAD_OBJECT = 2 };
nif_status nif_get_error_flags(nif_ctx* ctx, uint32_t* flags, int32_t clear, void* stream);

/* FP8 calibration of MLP `mlp` (per-layer scaling for the E4M3 path, a
 * precision option of this library beyond the paper's binary32 and 16-bit
 * weights, Sec. 5): runs the
 * binary32 encoding and layers 1..H-1 over the n queries (dev arrays as
 * nif_query) whose object uses `mlp` and whose segment meets the AABB, and
 * sets s_W[j] = max|W_j| / 448 and s_x[j] = max |input of layer j| / 448
 * (1 when the maximum is 0), as nif_set_fp8_scales would.  scales (host,
 * 2*hidden_layers floats, nullable) receives them.  Needs nif_prepare (any
 * dtype) for the object table; ws: nif_workspace_bytes(ctx, n, 2) bytes.
 * Synchronises `stream`.  n = 0 gives s_x = 1. */
nif_status nif_calibrate_fp8(nif_ctx* ctx, int32_t mlp, const float* rays, const int32_t* object_ids,
                             const float* t_max, int64_t n, float* scales, void* ws, size_t ws_bytes, void* stream);

/* Fill object obj's grid with the initial latents U[-amp, amp) (Sec. 5
 * "Initialization": amp = 1e-4): element i gets the top 24 bits m of word
 * (i mod 4) of Philox4x64-10 (Salmon et al., SC 2011) at counter
 * (i div 4, 0, 0, 0), key (seed, obj), as (m - 2^23) * (amp * 2^-23) in
 * binary32, rounded to nearest-even into grid_dtype. */
nif_status nif_init_grid(nif_ctx* ctx, int32_t obj, uint64_t seed, float amp, void* stream);

/* Upload the object table and pack the weights of every MLP for `dtype`
 * (NIF_F32, NIF_BF16, NIF_F16 or NIF_FP8_E4M3; FP8 needs scales).  Must be
 * called after changing objects, weights or scales and before nif_query with
 * that dtype.  Enqueued on stream. */
nif_status nif_prepare(nif_ctx* ctx, int32_t dtype, void* stream);

/* Options.  NIF_OPT_ORDER: before a query, bucket-sort the queries by
 * (object, Morton code of the AABB entry point) so that a wave's gathers share
 * cache lines and waves use one MLP: 0 never, 1 always, 2 (default) when
 * n >= 65536.  Changes nif_workspace_bytes (the ordering workspace plus the
 * queries as 32-byte records, see nif_order_packed).
 * NIF_OPT_GRID_IMAGE (binary16 grids only): 0 (default) = gather from the
 * grids (and, when ordering, also sort each 4,096-query window by an
 * 8-bit-per-axis Morton key, which pays off only without an image).  1 =
 * queries gather from a query image of each object's grid in which the four
 * latent pairs of a cell face (x..x+1, y..y+1) are one 16-byte span, halving
 * the gathers of a lookup (twice the grid's memory); 2 = a z-y-pair image in
 * which the eight corners of a cell are one 32-byte span (one cache line for
 * most cells; four times the grid's memory).  The image buffers are the
 * caller's: nif_image_bytes gives the size of one object's image for the
 * current mode, nif_set_image registers one per object, and nif_prepare
 * (re)builds them from the grids.  Changing the mode forgets the registered
 * buffers.  NIF_OPT_WINDOW_SORT: whether ordering (nif_query, nif_order,
 * nif_order_packed) also sorts each 4,096-query window by the finer key:
 * 0 never, 1 always, 2 (default) when NIF_OPT_GRID_IMAGE is 0.
 * NIF_OPT_TILE_SHAPE: the fused kernel's tile shape (0 default, 1, 2; see
 * nif_plan_create) for queries outside plans.  NIF_OPT_ORDER_BITS: at most
 * this many Morton bits per axis of the entry point in the ordering's bucket
 * key (-1, the default: as many as 4,096 buckets allow, up to 4); 0 orders
 * by object alone (many objects with many queries each gain little from the
 * finer buckets).  Plans order by their own schedule instead.  Outputs are
 * bit-identical in every mode. */
enum {
    NIF_OPT_ORDER = 1,
    NIF_OPT_GRID_IMAGE = 2,
    NIF_OPT_WINDOW_SORT = 3,
    NIF_OPT_TILE_SHAPE = 4,
    NIF_OPT_ORDER_BITS = 5
};
nif_status nif_set_option(nif_ctx* ctx, int32_t option, int64_t value);

/* Query images (NIF_OPT_GRID_IMAGE 1 or 2): nif_image_bytes is the size in
 * bytes of one object's image for the current mode (0 when the mode is 0).
 * nif_set_image registers object obj's image buffer (dev, caller-owned,
 * 256-byte aligned, at least nif_image_bytes bytes, else NIF_ERR_WORKSPACE;
 * NIF_ERR_STATE when the mode is 0).  nif_prepare fails with NIF_ERR_STATE
 * while an object has no image.  The buffer must stay allocated while the
 * context (or a plan of it) may launch a query. */
size_t nif_image_bytes(const nif_ctx* ctx);
nif_status nif_set_image(nif_ctx* ctx, int32_t obj, void* image, size_t bytes);

/* Build object obj's query image from its grid now, on `stream` (nif_prepare
 * builds every object's; this one alone, so that a grid can be released
 * before the next image is allocated).  NIF_ERR_STATE when the image mode is
 * 0 or the object has no image buffer or no grid. */
nif_status nif_build_image(nif_ctx* ctx, int32_t obj, void* stream);

/* Workspace bytes needed by nif_query (mode 0: with ordering, the ordering
 * workspace, the 32-byte query records and the fused kernel's tile counters;
 * 0 without ordering), nif_train_step (mode 1) or nif_calibrate_fp8 (mode 2)
 * for n queries. */
size_t nif_workspace_bytes(const nif_ctx* ctx, int64_t n, int32_t mode);

/* Visibility of n (ray, object) queries (Sec. 4.1: one query per object AABB
 * the ray meets; Sec. 3 Eq. (1): 1 = visible).
 *   rays (dev, n x 6 floats: ox oy oz dx dy dz; d need not be unit, t is in
 *   units of d), object_ids (dev, n), t_max (dev, n; +inf allowed)
 *   visibility (dev, n): sigmoid(z) in [0,1]; a ray that misses the AABB or
 *   whose segment [max(t_near,0), min(t_far,t_max)] is empty is visible (1).
 *   The paper's decision is occluded iff visibility < 0.5 (Sec. 5).
 *   logits (dev, n, nullable): z, +inf for a miss.
 *   dtype: arithmetic of the MLP (binary32, BF16, FP16 or FP8 E4M3 operands,
 *   binary32 accumulation); clip and grid coordinates are always binary32.
 *   ws: workspace of at least nif_workspace_bytes(ctx, n, 0) bytes (dev). */
nif_status nif_query(nif_ctx* ctx, int32_t dtype, const float* rays, const int32_t* object_ids, const float* t_max,
                     int64_t n, float* visibility, float* logits, void* ws, size_t ws_bytes, void* stream);

/* nif_query for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments and outputs as nif_query, without a workspace: the ordering
 * workspace and the 32-byte query records live in a static device array of
 * NIF_QUERY_NOALLOC_SCRATCH_BYTES bytes inside the library, one per GPU, held
 * from the first call on that GPU until the process ends.  The call allocates
 * nothing (no hipMalloc, no hipFree).  n is limited by that array:
 * nif_workspace_bytes(ctx, n, 0) must not exceed it, else NIF_ERR_UNSUPPORTED
 * before anything is enqueued (64 MiB holds about 1.39 million queries of one
 * object).  Every call on one GPU uses that GPU's array: calls that may
 * overlap in time on one GPU (other streams, other host threads, other
 * contexts) race on it and must be serialised by the caller, for instance by
 * issuing them on one stream. */
#define NIF_QUERY_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
nif_status nif_query_noalloc(nif_ctx* ctx, int32_t dtype, const float* rays, const int32_t* object_ids,
                             const float* t_max, int64_t n, float* visibility, float* logits, void* stream);

/* The ordering step and the query on a given order, as two calls (nif_query
 * runs both when NIF_OPT_ORDER selects ordering).
 * nif_order: perm (dev, n uint32) receives a permutation of [0, n): queries
 *   grouped by object, then by Morton code of their AABB entry point; misses
 *   and invalid queries last.  ws: nif_order_workspace_bytes(ctx, n) bytes.
 *   Needs nif_prepare (any dtype) for the object table.
 * nif_query_ordered: as nif_query, processing query perm[i] in slot i; perm
 *   must be a permutation of [0, n) (any order gives the same outputs).
 * nif_order_packed: as nif_order, and the ordering pass, which reads every
 *   query anyway, also stores query i as one 32-byte record: packed (dev,
 *   n x 8 floats, 16-byte aligned) row i = {ox, oy, oz, dx, dy, dz, t_max,
 *   object id (int32 bit pattern)}.  The query kernel, whose reads through
 *   perm are scattered, then fetches one 32-byte span per query instead of
 *   pieces of three arrays.
 * nif_query_packed: as nif_query_ordered with the queries given as those
 *   records (row perm[i] is computed in slot i, output perm[i]); perm may be
 *   NULL: the records in their own order (already grouped, as
 *   nif_expand_pairs_by_object writes them).  nif_query with ordering does
 *   the same internally.
 * Tiles of the fused kernel: the blocks on each XCD take the tiles of that
 * XCD's contiguous share of the order from a counter, so that the queries in
 * flight on an XCD are neighbours in the order and share its L2.  nif_query
 * and plans keep those counters (4 KiB) in their workspace; nif_query_ordered,
 * nif_query_packed and nif_query without ordering take a block of a ring of
 * 64 such blocks that the context allocates in nif_prepare, the next block
 * per call.  So at most 64 of those calls on one context may be in flight at
 * once (calls on one stream never overlap); more, from several streams or
 * threads, must be serialised by the caller. */
size_t nif_order_workspace_bytes(const nif_ctx* ctx, int64_t n);
nif_status nif_order(nif_ctx* ctx, const float* rays, const int32_t* object_ids, const float* t_max, int64_t n,
                     uint32_t* perm, void* ws, size_t ws_bytes, void* stream);
nif_status nif_query_ordered(nif_ctx* ctx, int32_t dtype, const float* rays, const int32_t* object_ids,
                             const float* t_max, const uint32_t* perm, int64_t n, float* visibility, float* logits,
                             void* stream);
nif_status nif_order_packed(nif_ctx* ctx, const float* rays, const int32_t* object_ids, const float* t_max, int64_t n,
                            uint32_t* perm, float* packed, void* ws, size_t ws_bytes, void* stream);
nif_status nif_query_packed(nif_ctx* ctx, int32_t dtype, const float* packed, const uint32_t* perm, int64_t n,
                            float* visibility, float* logits, void* stream);

/* Query plans for repeated batches on fixed buffers (the batched form: rays
 * of many objects of uneven size in one persistent launch, Sec. 4.1 issues one
 * query per (ray, object) pair).  A plan fixes ctx, dtype, the input, output
 * and workspace pointers and n; their contents may change between launches.
 * nif_plan_create: with tuning == NULL, times every candidate schedule
 *   (ordering off / bucket order / bucket order + window sort / by object
 *   alone (order 3: the bucket key's Morton bits 0, no window sort), times the
 *   persistent grid's blocks per compute unit 4..32, times the fused kernel's
 *   tile shape: shape 0 = 6 image lookups (or all 12 grid lookups) of a lane
 *   half gathered together at 3 waves per SIMD (2 for binary32), shape 1 = 12
 *   (6) at 2 waves per SIMD, shape 2 = 3 at 4 waves per SIMD; shapes 1 and 2
 *   exist for 8-level binary16 grids) on these buffers and keeps the fastest;
 *   otherwise uses the schedule of the JSON string `tuning` (as written by
 *   nif_plan_tuning: keys "order" 0..3, "blocks_per_cu" 1..32 and optionally
 *   "shape" 0..2).  When the environment variable NIF_PLAN_CACHE names a file,
 *   a schedule tuned before for the same device architecture, compute-unit
 *   count, model shape, object and MLP counts, image mode, dtype and n
 *   (rounded up to a power of two) is read from it instead of tuning, and a
 *   newly tuned one is appended to it (one JSON object per line).
 *   Then captures the ordering and query kernels into a HIP graph.  Writes the
 *   outputs while tuning; synchronises `stream`.  ws: at least
 *   nif_plan_workspace_bytes(ctx, n) bytes (dev), kept by the plan.  Needs
 *   nif_prepare(ctx, dtype); later nif_prepare calls (new weights, new latents)
 *   are seen by the plan.
 * nif_plan_launch: replays the graph on `stream` (same outputs as nif_query).
 *   Refused with NIF_ERR_STATE, before anything is enqueued, when the context
 *   changed in a way the captured graph cannot follow (nif_set_object,
 *   nif_set_image or a NIF_OPT_GRID_IMAGE change since the capture: create a
 *   new plan) or is not prepared for the plan's dtype (a training step or
 *   nif_set_mlp since the last nif_prepare: call nif_prepare again).
 * nif_plan_tuning: the chosen schedule as JSON (host buffer buf of buf_bytes):
 *   order, blocks_per_cu, shape and its gather_batch and waves_per_simd,
 *   queries_per_wave (32) and waves_per_block (4), tuned_us (-1 when given or
 *   read from the cache), candidates, from_cache.
 * nif_plan_destroy: frees the plan (not the caller's buffers). */
typedef struct nif_plan nif_plan;
size_t nif_plan_workspace_bytes(const nif_ctx* ctx, int64_t n);
nif_status nif_plan_create(nif_ctx* ctx, int32_t dtype, const float* rays, const int32_t* object_ids,
                           const float* t_max, int64_t n, float* visibility, float* logits, void* ws, size_t ws_bytes,
                           const char* tuning, void* stream, nif_plan** out);
nif_status nif_plan_launch(nif_plan* plan, void* stream);
nif_status nif_plan_tuning(const nif_plan* plan, char* buf, size_t buf_bytes);
void nif_plan_destroy(nif_plan* plan);

/* The two stages of a query as separate launches, as the paper's pipeline runs
 * them (Sec. 4.1: a grid-lookup kernel, then an inference kernel).
 * nif_encode: clip, normalise and interpolate the latents of n queries into
 *   features (dev, n x din floats, din = 3*levels*feats, order encoding-major
 *   (entry, exit, direction), then level, then latent); status (dev, n,
 *   nullable): 1 = the segment meets the AABB, 0 = miss (features 0),
 *   -1 = invalid query.  Needs nif_prepare (any dtype) for the object table.
 * nif_mlp: logits z (dev, n) of MLP `mlp` on given features (dev, n x din),
 *   in `dtype` arithmetic as nif_query.
 * nif_encode16 / nif_mlp16: the same with the features stored as 16-bit
 *   values of format fmt / dtype (NIF_F16 or NIF_BF16, rounded to nearest-
 *   even; dev, 8-byte aligned, n x din values): the MLP rounds its input to
 *   that format anyway, so nif_mlp16 on nif_encode16's features gives the
 *   logits of nif_query with that dtype, reading half the bytes. */
nif_status nif_encode(nif_ctx* ctx, const float* rays, const int32_t* object_ids, const float* t_max, int64_t n,
                      float* features, int32_t* status, void* stream);
nif_status nif_mlp(nif_ctx* ctx, int32_t dtype, int32_t mlp, const float* features, int64_t n, float* logits,
                   void* stream);
nif_status nif_encode16(nif_ctx* ctx, int32_t fmt, const float* rays, const int32_t* object_ids, const float* t_max,
                        int64_t n, void* features, int32_t* status, void* stream);
nif_status nif_mlp16(nif_ctx* ctx, int32_t dtype, int32_t mlp, const void* features, int64_t n, float* logits,
                     void* stream);

/* Adam hyper-parameters (Sec. 5 "Training"). */
typedef struct {
    float lr, beta1, beta2, eps;
} nif_adam;

/* Training buffers.
 * nif_set_object_train: latent gradient, Adam moments m and v (dev,
 *   grid_elems floats each) and the touched-latent flags (dev,
 *   nif_touched_bytes: one byte per 64 latents) of object obj.  grad and
 *   touched must be all zero
 *   before the first step; steps with Adam leave them zero again; m and v
 *   start at zero.
 * nif_set_mlp_train: Adam moments of MLP mlp (dev, mlp_params floats each,
 *   zero at the start). */
nif_status nif_set_object_train(nif_ctx* ctx, int32_t obj, float* grad, float* m, float* v, void* touched);
nif_status nif_set_mlp_train(nif_ctx* ctx, int32_t mlp, float* m, float* v);
size_t nif_touched_bytes(const nif_ctx* ctx);

/* One training step of MLP `mlp` and of the grids of the objects that use it
 * (Sec. 4.2 and Sec. 5 "Training": latents and weights are optimised jointly
 * with Adam by back-propagation through the MLP and the interpolation).
 *   rays, object_ids, t_max as nif_query; labels (dev, n bytes): 1 = visible
 *   (no occluder in the segment), 0 = occluded.  Queries that miss their AABB,
 *   are invalid, or whose object uses another MLP take no part.
 *   Loss: binary cross-entropy on the logit, mean over the B queries that take
 *   part; gradients dL/dz = (sigmoid(z) - label) / B, back-propagated through
 *   the ReLU MLP (binary32 MFMA) and into the grids: every interpolation corner
 *   of every lookup receives corner weight x feature gradient (binary32; the
 *   coarse levels' contributions are summed per block on chip first, so the
 *   order of the additions varies from run to run).
 *   adam != NULL: bias-corrected Adam step number `step` (1-based) on every MLP
 *   weight and on every latent whose gradient is non-zero this step (the others
 *   keep latent and moments); latents are updated in binary32 and rounded to
 *   nearest-even into grid_dtype; the MLP master stays binary32.  Packed query
 *   weights become stale: call nif_prepare before the next nif_query.
 *   adam == NULL: gradients only: mlp_grad receives dL/dW, each object's grid
 *   gradient buffer receives dL/dlatent (the caller zeroes it before the next
 *   step), weights and moments are not touched.
 *   loss (dev, 1 float, nullable): batch loss.  mlp_grad (dev, mlp_params
 *   floats, nullable): batch gradient of the MLP.
 *   ws: nif_workspace_bytes(ctx, n, 1) bytes. */
nif_status nif_train_step(nif_ctx* ctx, int32_t mlp, const float* rays, const int32_t* object_ids, const float* t_max,
                          const uint8_t* labels, int64_t n, int32_t step, const nif_adam* adam, float* loss,
                          float* mlp_grad, void* ws, size_t ws_bytes, void* stream);

/* Depth output for primary rays (Sec. 7: besides visibility, the network can
 * encode other information about the first hit, such as its depth).  A
 * context trained with nif_train_step_depth reads its visibility output y as
 * the normalised position of the closest hit in the query's segment.
 * nif_train_step_depth: as nif_train_step with the closest-hit distance
 *   t_hit (dev, n floats, +inf for no hit, as from nif_bvh_closest) instead of
 *   labels.  A query takes part when it meets its AABB, t_hit is finite and the
 *   segment [t_a, t_b] has t_b > t_a; its target is s = (t_hit - t_a) /
 *   (t_b - t_a) clamped to [0, 1] (binary32), and the loss is the mean of
 *   (y - s)^2 over the B queries that take part (L2, as the paper trains,
 *   Sec. 5 "Training"): dL/dz = 2 (y - s) y (1 - y) / B.  Everything else
 *   (gradients, Adam, buffers, workspace) as nif_train_step.
 * nif_depth_from_visibility: depth (dev, n floats) = t_a + y (t_b - t_a) for
 *   the visibilities y (dev, n) of nif_query on the same queries; +inf for a
 *   query that misses its AABB, NaN for an invalid one.  Needs nif_prepare. */
nif_status nif_train_step_depth(nif_ctx* ctx, int32_t mlp, const float* rays, const int32_t* object_ids,
                                const float* t_max, const float* t_hit, int64_t n, int32_t step, const nif_adam* adam,
                                float* loss, float* mlp_grad, void* ws, size_t ws_bytes, void* stream);
nif_status nif_depth_from_visibility(nif_ctx* ctx, const float* rays, const int32_t* object_ids, const float* t_max,
                                     const float* visibility, int64_t n, float* depth, void* stream);

/* Backward pass of a binary32 query for a given upstream gradient, so that the
 * query can sit inside a larger differentiable program (the gradients the
 * paper's training back-propagates through the MLP and the interpolation,
 * Sec. 4.2, for an arbitrary loss of the visibilities).
 *   grad_visibility (dev, n floats): dL/dy_i of the visibility y_i.
 *   Recomputes the forward pass of the queries whose object uses MLP `mlp` and
 *   whose segment meets the AABB, then dL/dz_i = g_i y_i (1 - y_i) (no 1/B
 *   factor); mlp_grad (dev, mlp_params floats, nullable) receives dL/dW;
 *   each such object's registered grid gradient buffer (nif_set_object_train)
 *   is incremented by dL/dlatent.  Touched bitmaps are left zero; weights,
 *   latents and moments are not touched.  ws: nif_workspace_bytes(ctx, n, 1). */
nif_status nif_backward(nif_ctx* ctx, int32_t mlp, const float* rays, const int32_t* object_ids, const float* t_max,
                        const float* grad_visibility, int64_t n, float* mlp_grad, void* ws, size_t ws_bytes,
                        void* stream);

/* The paper's own networks (Sec. 3.1, Sec. 3.2, Sec. 5 "Architecture",
 * Table 1), forward pass.  A query whose origin lies strictly inside its
 * object's AABB goes to the inner network, any other query that meets the
 * AABB to the outer network; a miss is visible (1, logit +inf) and invalid
 * input gives NaN, as for nif_query.
 *   outer: position = the AABB entry point; q = (p - c) / h (c the box
 *   centre, h its half extents); (u, v) = (theta / pi, (phi + pi) / (2 pi))
 *   of the spherical angles of q and of d; bilinear lookups (vertex-aligned,
 *   s = u (R - 1)) in a 256 x 256 grid of 3 latents for each; MLP 6-64-64-1.
 *   inner: position = the origin; the same maps on 128 x 128 grids of 5
 *   latents, plus r = |q| / sqrt(3) looked up linearly in a 1D grid of 128 x 3
 *   latents; MLP 13-48-48-48-1.
 *   Both MLPs: no biases, leaky ReLU (slope 0.01f) after every hidden layer,
 *   sigmoid output; input order [position, direction(, distance)] latents.
 * nif_paper_mlp_params / nif_paper_grid_elems: weights of network 0 (outer)
 *   or 1 (inner) (4,544 / 5,280), and latents of one object's grid buffer for
 *   that network (position grid, direction grid, distance grid, each row-major
 *   [u][v][latent], back to back); -1 for another network number.
 * nif_paper_create / destroy: a handle for num_objects objects.
 * nif_paper_set_object: box (host, 6 floats lo, hi) and the object's two grid
 *   buffers (dev, binary16, caller-owned).
 * nif_paper_init_grid: fills one grid buffer with U[-amp, amp) latents of the
 *   generator of nif_init_grid, keyed by 2 obj + network.
 * nif_paper_set_mlp: the shared weights of a network (dev, binary32, W1
 *   [width][din], W2..WH [width][width], w_out [width], row-major); copied, so
 *   the buffer may be reused.  Synchronises `stream`.
 * nif_paper_prepare: packs both networks' weights for dtype (NIF_F32,
 *   NIF_F16 or NIF_BF16 operands, binary32 accumulation and output layer).
 * nif_paper_query: visibility (and logits, nullable) of n queries, arrays as
 *   in nif_query; one launch on `stream`, in which every wave runs the MLP of
 *   each network that one of its queries needs. */
typedef struct nif_paper nif_paper;
int64_t nif_paper_mlp_params(int32_t network);
int64_t nif_paper_grid_elems(int32_t network);
nif_status nif_paper_create(int32_t num_objects, nif_paper** out);
void nif_paper_destroy(nif_paper* p);
nif_status nif_paper_set_object(nif_paper* p, int32_t obj, const float* aabb, void* outer_grid, void* inner_grid);
nif_status nif_paper_init_grid(nif_paper* p, int32_t obj, int32_t network, uint64_t seed, float amp, void* stream);
nif_status nif_paper_set_mlp(nif_paper* p, int32_t network, const float* w, void* stream);
nif_status nif_paper_prepare(nif_paper* p, int32_t dtype, void* stream);
nif_status nif_paper_query(nif_paper* p, int32_t dtype, const float* rays, const int32_t* object_ids,
                           const float* t_max, int64_t n, float* visibility, float* logits, void* stream);

/* Training of the paper's networks (Sec. 5 "Training": L2 loss, Adam; the
 * latents are trained with the MLP, Fig. 2), binary32.
 * nif_paper_set_train: the binary32 master weights of `network` (dev, the
 *   layout of nif_paper_set_mlp; updated in place by Adam, and also copied
 *   into the inference weights as nif_paper_set_mlp does) and its Adam
 *   moments m, v (dev, same size, caller-initialised).  Synchronises `stream`.
 * nif_paper_set_object_train: for object obj and `network`, the binary32
 *   latent gradient and Adam moments (dev, nif_paper_grid_elems(network)
 *   floats each).
 * nif_paper_train_step: one step on the n queries (dev arrays as in
 *   nif_query; labels dev, n bytes, 1 = visible) of which those of the
 *   network's class form the batch B: L = (1/B) sum (y - t)^2.  Gradients of
 *   the MLP (mlp_grad, dev, nullable) and of every object's latents (its
 *   grid_grad buffer, zeroed first); with adam != NULL also Adam step `step`
 *   (1-based) on the master (dense) and on the binary16 latents whose
 *   gradient is non-zero (moments kept elsewhere), after which the latent
 *   gradient reads 0 and nif_paper_prepare must run again before a query.
 *   loss (dev, nullable) receives L (0 when B = 0).  ws: at least
 *   nif_paper_train_workspace_bytes(p, network, n) bytes (dev). */
nif_status nif_paper_set_train(nif_paper* p, int32_t network, float* w, float* m, float* v, void* stream);
nif_status nif_paper_set_object_train(nif_paper* p, int32_t obj, int32_t network, float* grid_grad, float* grid_m,
                                      float* grid_v);
size_t nif_paper_train_workspace_bytes(const nif_paper* p, int32_t network, int64_t n);
nif_status nif_paper_train_step(nif_paper* p, int32_t network, const float* rays, const int32_t* object_ids,
                                const float* t_max, const uint8_t* labels, int64_t n, int32_t step,
                                const nif_adam* adam, float* loss, float* mlp_grad, void* ws, size_t ws_bytes,
                                void* stream);
/* nif_paper_backward: as nif_paper_train_step without labels or Adam, for a
 * given dL/dy per query (grad_visibility, dev, n): dL/dz = g y (1 - y) for
 * the network's queries, no 1/B; mlp_grad (dev, nullable) and every object's
 * grid_grad buffer receive dL/dW and dL/dlatents (the torch.autograd bridge
 * PaperVisibility calls it for each network). */
nif_status nif_paper_backward(nif_paper* p, int32_t network, const float* rays, const int32_t* object_ids,
                              const float* t_max, const float* grad_visibility, int64_t n, float* mlp_grad,
                              void* ws, size_t ws_bytes, void* stream);

/* Light importance sampling of training rays (Sec. 5 "Training": directions
 * drawn in proportion to radiant flux from a tabulated CDF searched by
 * bisection; Sec. 6 "Comparison of Sampling Method").
 * nif_light_create: num_tris emitting triangles (host, 9 floats each, non-
 *   degenerate) with radiance (host, >= 0, not all 0); flux pi L A, running
 *   sums in triangle order / total as the binary32 table (last entry 1),
 *   copied to the current device (the handle owns it).
 * nif_light_sample: for n shading points (dev, n x 3) and random numbers u
 *   (dev, n x 3, in [0, 1)): triangle = first table entry > u0; point =
 *   v0 + b1 (v1 - v0) + b2 (v2 - v0), b1 = 1 - sqrt(u1), b2 = u2 sqrt(u1);
 *   rays (dev, n x 6) = the point x and the unit direction to the light
 *   point, t_max (dev, n) = the distance, pdf (dev, n, nullable) = the
 *   solid-angle density P(tri) / area * dist^2 / |n . d|, tri (dev, n,
 *   nullable) = the triangle chosen. */
typedef struct nif_light nif_light;
nif_status nif_light_create(const float* tris, const float* radiance, int64_t num_tris, nif_light** out);
void nif_light_destroy(nif_light* light);
nif_status nif_light_sample(const nif_light* light, const float* points, const float* u, int64_t n, float* rays,
                            float* t_max, float* pdf, int32_t* tri, void* stream);

/* Plain BVH any-hit ray casting: exact shadow-ray labels for training and the
 * baseline the paper compares against (Sec. 6 "Performance Evaluation").
 * nif_bvh_create: builds a binned-SAH BVH on the host from num_tris
 *   triangles (host, num_tris x 9 floats: three vertices) and copies it to the
 *   current device (the handle owns that memory).
 * nif_bvh_anyhit: visible[i] (dev, n bytes) = 1 iff no triangle is hit at a
 *   distance t with 0 < t < t_max[i] along rays[i] (dev, n x 6 floats);
 *   binary32 watertight triangle test (Woop, Benthin, Wald, JCGT 2013),
 *   double-sided.
 * nif_bvh_closest: t_hit[i] (dev, n floats) = the smallest such t (binary32
 *   T / det of the same test), +inf when there is none: the depth of primary
 *   rays, the targets of nif_train_step_depth. */
typedef struct nif_bvh nif_bvh;
nif_status nif_bvh_create(const float* tris, int64_t num_tris, nif_bvh** out);
void nif_bvh_destroy(nif_bvh* bvh);
int64_t nif_bvh_num_nodes(const nif_bvh* bvh);
nif_status nif_bvh_anyhit(const nif_bvh* bvh, const float* rays, const float* t_max, int64_t n, uint8_t* visible,
                          void* stream);
nif_status nif_bvh_closest(const nif_bvh* bvh, const float* rays, const float* t_max, int64_t n, float* t_hit,
                           void* stream);

/* Thread-local text of the last error (empty after success). */
const char* nif_last_error(void);

/* Library version string. */
const char* nif_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NIF_H */
