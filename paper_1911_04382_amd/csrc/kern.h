// Launch shapes and device helpers shared by the embedding kernels.
#pragma once
#include "state.h"

namespace grass {

#define KP_DISPATCH(kp, ...)                                                                    \
    switch (kp) {                                                                               \
    case 1: { constexpr int KP = 1; __VA_ARGS__; } break;                                       \
    case 2: { constexpr int KP = 2; __VA_ARGS__; } break;                                       \
    case 4: { constexpr int KP = 4; __VA_ARGS__; } break;                                       \
    case 8: { constexpr int KP = 8; __VA_ARGS__; } break;                                       \
    case 16: { constexpr int KP = 16; __VA_ARGS__; } break;                                     \
    case 32: { constexpr int KP = 32; __VA_ARGS__; } break;                                     \
    case 64: { constexpr int KP = 64; __VA_ARGS__; } break;                                     \
    default: throw Error(GRASS_ERR_INVALID, "k must be in 1..64");                              \
    }

constexpr int kThreads = 256;
constexpr int kRowsPerGroup = 16;  // rows per lane group in the row-block vector kernels
constexpr int kColThreads = 1024;
constexpr int kPersist = 2048;     // largest grid of the Gram kernels (partials in a fixed order)
// blocks of the Gram kernels: full occupancy for k <= 32, fewer partials for wide blocks
inline int gram_blocks(int kp) { return kp <= 32 ? 2048 : 512; }

// 8 XCDs: consecutive workgroup ids land on different XCDs; remap them so that each
// XCD works on one contiguous range of rows (its L2 then holds the neighbourhood).
__device__ __forceinline__ int xcd_block(int bid, int grid) {
    int per = grid >> 3;
    return (bid & 7) * per + (bid >> 3);
}
inline int xcd_grid(int nb) { return (nb + 7) / 8 * 8; }
inline int grid_nk(long long nk) { return (int)std::min<long long>(std::max<long long>(1, (nk + 255) / 256), 8192); }
inline int vec_blocks(const Dims &d) { return div_up(d.n, (kThreads / d.kp) * kRowsPerGroup); }

}  // namespace grass
