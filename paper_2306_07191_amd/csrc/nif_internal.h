// Internal definitions shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nif {

constexpr int kMaxLevels = 8;
constexpr int kWidth = 64;      // hidden width covered by the MFMA tiling
constexpr int kFeats = 2;       // latents per grid vertex
constexpr int kMaxHidden = 8;
constexpr int kBlock = 256;     // threads per block: 4 waves
constexpr int kQueriesPerWave = 32;  // two lanes per query
constexpr int kQueriesPerBlock = kBlock / 64 * kQueriesPerWave;

// Per-object device record.  ext = hi - lo evaluated in binary32 once.
struct ObjDev {
    float lo[3];
    float hi[3];
    float ext[3];
    int32_t mlp;
    const void* grid;
    const void* image;  // y-pair query image of a binary16 grid, or null
};

enum Flavor { kF32 = 0, kF16 = 1, kBF16 = 2, kFP8 = 3 };

// Packed weight image of one MLP for one arithmetic flavour.
//
// The MLP runs as 32x32 MFMA tiles with the 32 queries of a wave on the N
// dimension; the two 32-lane halves of the wave split the K dimension.  Half h
// owns "local" input features c = 0..Kh-1 of every layer:
//  - layer 1: global feature h*(din/2) + c (the half encodes those lookups);
//  - layer j > 1: the accumulator rows it holds, f(c) = 32*(c/16) + 8*((c%16)/4)
//    + 4h + (c%4) (output row of accumulator register c%16 of M-tile c/16).
// A K-step consumes the same local positions from both halves, so the packed
// A operand of lane l (row 32*mt + l%32, half l/32) stores W[row][global(half, c)]
// in local order.  Layout: per layer, per M-tile (2), per K-group, 64 lanes x
// 16 bytes; w_out follows in binary32 permuted per half: wout[h][c] = w_out[f_h(c)].
struct PackInfo {
    int32_t din;        // MLP input width (3 * levels * feats)
    int32_t hidden;
    int64_t layer_off[kMaxHidden + 1];  // byte offsets of each layer's A image, [H] = w_out
    int64_t bytes;      // total bytes per MLP
};

struct FwdArgs {
    const float* rays;
    const int32_t* ids;
    const float* tmax;
    int64_t n;
    float* vis;
    float* logit;
    const ObjDev* objs;
    int32_t num_objects;
    int32_t hidden;
    const uint8_t* packed;  // num_mlps x pack.bytes
    PackInfo pack;
    const float* fp8_scales;  // num_mlps x 2H (s_W then s_x) or null
    int64_t toff[3 * kMaxLevels];
    int32_t res[kMaxLevels];
    const uint32_t* perm;    // processing order: query perm[q] is handled in slot q (null = identity)
    float* features;         // grid stage output / inference stage input: n x din, or null
    int32_t feat16;          // features stored as 16-bit values: 0 binary32, kF16 or kBF16
    int32_t* status_out;     // grid stage: 1 query, 0 miss, -1 invalid (nullable)
    int32_t fixed_mlp;       // inference stage: the MLP used by every query
    int32_t tiles_per_block_num;  // tiles are split evenly: block b gets [b*T/G, (b+1)*T/G)
    int32_t num_tiles;
    int32_t xcd_stride;           // logical block = (b % 8) * xcd_stride + b / 8
    int32_t blocks_per_cu;        // persistent grid size per compute unit (0: 16)
    int32_t use_image;            // gather from the objects' images: 0 none, 1 y-pair, 2 z-y-pair
    uint32_t* flags;              // domain-error bits of the launch are OR-ed in here (nullable)
    int64_t ioff[3 * kMaxLevels];  // table offsets inside an image (elements)
    const float4* qrec;           // nullable: query i as a 32-byte record {o, d.x}, {d.y, d.z, t_max, id bits}
    int32_t shape;                // tile shape of the fused query (0 default, 1, 2; see shape_batch)
    uint32_t* tile_ctr;           // fused query: tile counters (kTileCtrBytes); null = static tiles
    int32_t tile_ctr_reset;       // 1: the counters are zero at launch and its last block zeroes them again;
                                  // 0: of unknown content, zeroed by a kernel before the launch
};

// Tile counters of one fused-query launch: per XCD a 32-bit tile counter and
// a count of its finished blocks, each on its own 256-byte line.
constexpr int kTileCtrStride = 64;
constexpr int kTileCtrWords = 16 * kTileCtrStride;
constexpr size_t kTileCtrBytes = kTileCtrWords * sizeof(uint32_t);

// The paper's own networks: per object its box and its grid buffer of each
// network (binary16: position grid, direction grid, and for the inner network
// the distance grid, back to back).
struct PaperObj {
    float lo[3], hi[3];
    float c[3], ih[3];  // box centre and reciprocal half extents
    const void* grid[2];
};

struct PaperArgs {
    const float* rays;
    const int32_t* ids;
    const float* tmax;
    int64_t n;
    float* vis;
    float* logit;
    const PaperObj* objs;
    int32_t num_objects;
    int32_t hidden[2];
    const uint8_t* packed[2];  // each network's MLP image (pack_forward layout, padded to width 64)
    PackInfo pack[2];
    int32_t num_tiles, tiles_per_block_num, xcd_stride;
    uint32_t* flags;
};

// Both networks in one launch: outer and inner queries, misses and invalid input.
hipError_t launch_paper(int flavor, const PaperArgs& a, int num_cus, hipStream_t s);

struct AdamDev {
    float lr, beta1, beta2, eps;
    float bc1, bc2;  // 1 - beta^step
};

// Training of one of the paper's networks (binary32, L2 loss).
struct PaperTrainArgs {
    const float* rays;
    const int32_t* ids;
    const float* tmax;
    const uint8_t* labels;  // 1 = visible
    int64_t n;
    const PaperObj* objs;
    int32_t num_objects;
    float* w;               // binary32 master, unpadded [W1 | W2..WH | w_out], updated by Adam
    float* mlp_m;
    float* mlp_v;
    float* padded;          // the inference master (64-wide), refreshed after the update
    float* ws_h;            // rows h0 [n][din], h1..hH [n][width]
    float* ws_d;            // rows delta_1..delta_H [n][width]
    float* dz;              // [n], dL/dz times the batch size
    float* const* grid_grad;  // per object: gradient of this network's grid buffer (binary32)
    float* const* grid_m;
    float* const* grid_v;
    void* const* grid;        // per object: the binary16 grid buffer
    float* dw;              // [P] sums over the batch
    float* loss_sum;
    uint32_t* count;        // queries of this network's class
    float* grad_out;        // nullable: dL/dW
    float* loss_out;        // nullable
    AdamDev adam;
    int32_t use_adam;
    const float* grad_y;    // nullable: dL/dy per query instead of labels (gradients only, no 1/B)
};
size_t paper_train_workspace_bytes(int network, int64_t n);
hipError_t launch_paper_train(int network, PaperTrainArgs a, void* ws, hipStream_t s);
hipError_t launch_paper_zero(float* p, int64_t n, hipStream_t s);

// Light importance sampling (opaque table on the device).
hipError_t light_create(const float* tris, const float* radiance, int64_t L, void** out, const char** why);
void light_destroy(void* h);
int32_t light_count(const void* h);
hipError_t launch_light_sample(const void* h, const float* points, const float* u, int64_t n, float* rays,
                               float* tmax, float* pdf, int32_t* which, hipStream_t s);

struct OrderArgs {
    const float* rays;
    const int32_t* ids;
    const float* tmax;
    int64_t n;
    const ObjDev* objs;
    int32_t num_objects;
    int32_t bits;          // Morton bits per axis
    uint32_t num_buckets;  // (num_objects << 3 bits) + 1; the last holds misses and invalid queries
    int64_t tile;          // queries per block
    int64_t num_tiles;
    uint32_t* table;       // num_tiles x num_buckets counts, then per-bucket offsets over the tiles
    uint32_t* block_sums;  // per bucket: total, then offset of the bucket
    uint16_t* key;         // bucket of every query
    uint32_t* fine;        // finer key of every query
    uint32_t* coarse;      // bucket order (before the window refinement)
    int32_t fine_bits;
    int32_t no_refine;     // 1: bucket order only (skip the window sort)
    uint32_t* perm;
    float4* qrec;          // nullable: receives query i as a 32-byte record {o, d.x}, {d.y, d.z, t_max, id bits}
    uint32_t* zero_words;  // nullable: kTileCtrWords words the count pass zeroes (the next query's tile counters)
    const uint32_t* key_in;  // nullable: given fine keys (no queries read, no records written)
    int32_t max_bits = -1;   // bucket Morton bits per axis at most this (-1: order_bits alone)
};

int order_bits(int32_t num_objects);
int order_bucket_bits(int32_t num_objects, int32_t max_bits);  // the bits a launch uses
int order_fine_bits(int32_t num_objects);  // Morton bits per axis of the fine key
size_t order_workspace_bytes(int64_t n, int32_t num_objects);
hipError_t launch_order(OrderArgs A, void* ws, hipStream_t s, const uint32_t** perm_out);


struct TrainArgs {
    const float* rays;
    const int32_t* ids;
    const float* tmax;
    const uint8_t* labels;
    const float* grad_y;  // upstream dL/dy per query (backward mode) or null
    const float* t_hit;   // closest-hit distance per query (depth mode: L2 on the normalised depth) or null
    int64_t n;
    const uint32_t* perm;
    const ObjDev* objs;
    int32_t num_objects;
    int32_t mlp;
    int32_t hidden;
    int32_t din;
    int64_t P;
    int64_t toff[3 * kMaxLevels];
    int32_t res[kMaxLevels];
    const float* fwd;  // binary32 forward image of the trained MLP
    PackInfo pack;
    const float* bwd;  // backward (transposed) image
    float* const* grid_grad;
    float* const* grid_m;
    float* const* grid_v;
    uint8_t* const* touched;  // dirty flag per 64 latents
    void* const* grids;
    float* master;
    float* mlp_m;
    float* mlp_v;
    float* act;
    int64_t act_off[kMaxHidden + 1];
    float* delta;
    int64_t delta_off[kMaxHidden];
    float* dz;
    float* dw_part;
    float* dw;
    int64_t dw_chunk;
    int64_t w_off[kMaxHidden + 1];
    unsigned* count;
    float* loss_sum;
    float* loss_out;
    float* grad_out;
    int32_t apply_adam;  // 0: gradients only (scaled by 1/B, left in grid_grad)
    AdamDev adam;
};

size_t train_workspace_bytes(int64_t n, int din, int hidden, int64_t P, int64_t* chunk_out);
size_t calib_workspace_bytes(int64_t n, int din);
hipError_t launch_calibrate(const FwdArgs& enc, int levels, int grid_dtype, int num_cus, int32_t mlp, const float* W,
                            int din, int hidden, void* ws, unsigned* amax_host, hipStream_t s);
hipError_t launch_train(TrainArgs A, void* ws, const int32_t* obj_of_mlp, int32_t num_obj_of_mlp,
                        const int64_t* elems_per_obj, int grid_dtype, int levels, int num_cus, hipStream_t s);

size_t backward_image_bytes(int hidden);
hipError_t launch_pack_forward(const float* W, uint8_t* out, const PackInfo& P, int flav, int din, int width,
                               const float* scales_w, hipStream_t s);
hipError_t launch_pack_backward(const float* W, float* out, int hidden, int din, int width, hipStream_t s);
// Output feature of an MLP layer held in accumulator register (c % 16) of
// M-tile c / 16 by lane half h of a 32x32 MFMA: row 8 (r / 4) + 4 h + r % 4.
__host__ __device__ __forceinline__ int acc_feature(int half, int c) {
    return 32 * (c / 16) + 8 * ((c % 16) / 4) + 4 * half + (c % 4);
}

PackInfo pack_info(int flavor, int din, int hidden);
size_t lds_bytes(const PackInfo& p);

hipError_t launch_forward(int flavor, int levels, int grid_dtype, const FwdArgs& a, int num_cus, hipStream_t s);
hipError_t launch_encode(int levels, int grid_dtype, const FwdArgs& a, int num_cus, hipStream_t s);
hipError_t launch_mlp(int flavor, int levels, const FwdArgs& a, int num_cus, hipStream_t s);
hipError_t launch_mlp16(int flavor, int levels, const FwdArgs& a, int num_cus, hipStream_t s);
// y-pair query image of a binary16 grid: for every table (N cells per axis),
// entry (x, y, z), x, z in [0, N], y in [0, N-1], holds the two latents of
// vertex (x, y, z) then those of (x, y+1, z); entries are x-fastest, so one
// 16-byte load at entry (x, y, z) returns the four corners (x..x+1, y..y+1) of
// a cell face.
// z-y-pair image (kind 2): entry (x, y, z), x in [0, N], y, z in [0, N-1],
// holds the latent pairs of (x, y, z), (x, y+1, z), (x, y, z+1), (x, y+1, z+1);
// the eight corners of a cell are then 32 contiguous bytes.
int64_t image_table_elems(int32_t N, int kind);
hipError_t launch_build_image(const void* grid, void* image, const int64_t* toff, const int64_t* ioff,
                              const int32_t* res, int levels, int kind, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
// Two-level 64-wide box tree of the pair expansion.  With at most 64 objects
// one level: slot j of mbox / mid is object j.  Otherwise C <= 64 clusters of
// up to 64 objects consecutive in the Morton order of their box centres:
// cbox[c] is cluster c's union box, slots c*64 .. c*64+63 of mbox / mid its
// members (empty slots: lo = +inf, hi = -inf, id -1).  root: union of all
// boxes.  Boxes are lo xyz, hi xyz.
struct PairTree {
    const float* cbox;
    const float* mbox;
    const int32_t* mid;
    int32_t C;
    float root[6];
};
size_t pairs_workspace_bytes(int64_t n_rays, int32_t K);
// round: 0 every pair; 1 each ray's first pair; 2 the other pairs of the rays
// with ray_visible != 0 (see nif_pairs.hip).
hipError_t launch_expand_pairs(const float* rays, const float* tmax, int64_t n, const PairTree& T, int32_t K,
                               int num_cus, int32_t round, const uint8_t* ray_visible, int64_t max_pairs,
                               float* pair_rays, float* pair_tmax, int32_t* pair_ids, uint32_t* pair_ray,
                               int64_t* total, void* ws, hipStream_t s, float4* rec = nullptr,
                               uint32_t* keys = nullptr, const ObjDev* objs = nullptr, bool object_keys = false,
                               bool grouped = false, int64_t* obj_off = nullptr);
// t = t_a + y (t_b - t_a) of the query's segment; +inf for a miss, NaN for an
// invalid query.
hipError_t launch_depth_from_visibility(const float* rays, const int32_t* ids, const float* tmax, const float* vis,
                                        int64_t n, const ObjDev* objs, int32_t K, float* depth, int num_cus,
                                        hipStream_t s);
// init: set every ray visible first; else only clear the rays of occluded pairs.
hipError_t launch_combine_pairs(const uint32_t* pair_ray, const float* vis, int64_t n_pairs, int64_t n_rays,
                                uint8_t* ray_visible, bool init, hipStream_t s);
hipError_t launch_init_grid(void* grid, int grid_dtype, int64_t count, uint64_t seed, uint64_t obj, float amp,
                            hipStream_t s);

}  // namespace nif
