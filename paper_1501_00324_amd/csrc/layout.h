// The device data layout of a matrix handle, shared by the host builder and
// the kernels.
//
// One row group is processed by one 64-lane wavefront.  A group holds
// 64 / T consecutive layout rows, T lanes per row (T a power of two); entry
// e of a row (columns ascending) goes to lane (row_in_group * T + e % T),
// slot e / T of that lane.  Slots are interleaved so that one wave-wide
// load of V consecutive slots per lane (V = 1 or 2, per matrix) is one
// contiguous 64*V element block:
//     element index = base + (s / V) * 64 * V + lane * V + s % V.
#pragma once

#include <cstdint>

namespace fs {

constexpr int kWave = 64;
constexpr int kBlock = 256;        // threads per workgroup (4 waves)

struct Group {                     // 16 bytes, read once per wave
    int32_t base64;                // first element index / 64
    int32_t row0;                  // first layout row
    int32_t nrows;                 // rows in the group (1..64/T)
    int32_t width_lt;              // slots per lane | log2(T) << 24
};

}  // namespace fs
