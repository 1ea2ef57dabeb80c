// Constants shared by the streaming kernels.
#pragma once

#include <stdint.h>

namespace trk {

constexpr int kNT = 256;            // threads of the streaming kernels
constexpr double kTwoPi = 6.283185307179586;
constexpr uint32_t kDevNonFinite = 0x1u;
constexpr uint32_t kDevZeroDist = 0x2u;
constexpr uint32_t kDevBadIndex = 0x4u;  // a sparse row index outside the mode

template <typename T>
struct RowsPerChunk {
  static constexpr int value = sizeof(T) == 4 ? 32 : 16;  // 128 B per fiber chunk
};

}  // namespace trk
