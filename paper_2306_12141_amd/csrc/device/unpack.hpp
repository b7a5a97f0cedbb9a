// Device-side unpacking of the split-point metadata (Sec. 4.3) into the per-unit
// and per-lane records the decode kernels read (decode.hpp).
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

#include "decode.hpp"

namespace recoil {

// The packed metadata section of a stream with M units (M - 1 split points),
// MSB first: a signed word-offset series and a signed group series (each a 5-bit
// width-1 field, then per split point a sign bit and `width` magnitude bits),
// then per split point a block of W 16-bit states, a 4-bit width-1 field and W
// unsigned group differences of that width. Split point k (0-based, k < M - 1)
// has word offset o_k = next_k - (k+1) ceil(B/M) and group value
// x_k = anchor_k + 1 - (k+1) ceil(G/M).
//
// Output unit u (0-based, u < units) starts at split point k = (u+1) step - 1
// (every step-th split point, Sec. 3.3: step = 1 keeps all), the last unit at
// the final states; its records equal those the host planner builds for the
// stream combined to `units` units.
struct UnpackParams {
    const uint8_t *bits;          // packed metadata section, readable 8 bytes past its end
    const uint32_t *block_bit;    // M - 1: bit offset of split point k's block
    const uint32_t *final_states; // W
    UnitMeta *meta;               // units records (written)
    uint32_t *lanes;              // units x W (written)
    uint64_t words;               // B
    uint64_t groups;              // G
    uint64_t eb, eg;              // ceil(B/M), ceil(G/M)
    uint32_t splits;              // M of the packed stream
    uint32_t step;
    uint32_t units;               // records written: (M - 1) / step + 1
    uint32_t lanes_per_unit;      // W: 32 or 64
};

// One 64-lane wave per output unit. Returns hipSuccess or the launch error.
hipError_t launch_unpack(const UnpackParams &p, hipStream_t stream);

}  // namespace recoil
