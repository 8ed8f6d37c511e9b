// Layout of the population buffers in device memory: alignment of every
// region and the stride between consecutive q-blocks of a box. The step
// kernels' HBM traffic depends on these (and on the kernel sources), not on
// the rest of the host code.
#pragma once

#include <cstdint>

namespace lbm {

constexpr uint64_t ALIGN = 256;  // bytes; every region and q-block starts on this

inline uint64_t align_up(uint64_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// Elements from one q-block of a box to the next: the block rounded up to
// 256 bytes, plus 1 MiB + 256 bytes for 16-bit storage when the block is a
// multiple of 1 MiB. Without it the 41 streams of a step sit at the same
// address modulo a large power of two (a 512^3 FP16 q-block is 2^29 bytes);
// measured on MI355X at 512^3: FP16-shifted+SR 9.25 -> 8.69 ms per step,
// BF16-shifted+SR 9.65 -> 9.09 ms, while FP32 and FP64 gained nothing (FP64
// lost 2%), so they keep the plain stride.
constexpr uint64_t QPAD_16 = (1u << 20) + 256;
inline uint32_t qstride(uint64_t nodes, int eb)
{
    const uint64_t bytes = align_up(nodes * uint64_t(eb));
    const uint64_t pad = (eb == 2 && bytes % (1u << 20) == 0) ? QPAD_16 : 0;
    return uint32_t((bytes + pad) / uint64_t(eb));
}

}  // namespace lbm
