// Ordering keys of queries, shared by the ordering passes and by pair
// expansion (which writes each pair's key with the pair).
#pragma once

#include "nif_device.h"

namespace nif {

// Morton spread of the low 10 bits of v to every third bit.
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Ordering key of a query: (object id, Morton code of the binary32 AABB entry
// point with fine_bits per axis), 0xffffffff for an invalid query or a miss.
// The ordering's bucket (bucket_of_fine) is a prefix of it.
__device__ __forceinline__ uint32_t fine_order_key(const float o[3], const float d[3], float tm, int32_t id,
                                                   const ObjDev* __restrict__ objs, int32_t K, int fine_bits) {
    if (!valid_query(o, d, tm, id, K)) return 0xffffffffu;
    float uin[3];
    if (!clip_entry(o, d, tm, objs[id], uin)) return 0xffffffffu;
    const uint32_t cells = 1u << fine_bits;
    uint32_t c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const uint32_t v = (uint32_t)(uin[a] * (float)cells);  // u in [0, 1]
        c[a] = v < cells ? v : cells - 1;
    }
    const uint32_t m = spread3(c[0]) | (spread3(c[1]) << 1) | (spread3(c[2]) << 2);
    return ((uint32_t)id << (3 * fine_bits)) | m;
}

// Bucket of a fine key: the object and the top `bits` Morton bits per axis;
// the last bucket (nb - 1) for a miss or an invalid query.
__device__ __forceinline__ uint32_t bucket_of_fine(uint32_t fine, int fine_bits, int bits, uint32_t nb) {
    if (fine == 0xffffffffu) return nb - 1;
    const uint32_t id = fine >> (3 * fine_bits), m = fine & ((1u << (3 * fine_bits)) - 1u);
    return (id << (3 * bits)) | (m >> (3 * (fine_bits - bits)));
}

}  // namespace nif
