// smap_copy.hpp -- copy of the simplex cells of a uint8 box: the ceiling
// that the (n+1)^m bounding-box layout puts on any one-pass kernel over
// Delta_n^m (m = 2, 3).
//
// A kernel that reads every simplex cell once and writes it once moves the
// automata's algorithmic bytes (Section 5.1's CA test: one read and one
// write per cell) and nothing else.  The cells of one row (x_2..x_m fixed)
// are contiguous, n + 1 - (x_2 + ... + x_m) bytes long, and the rows lie
// n + 1 bytes apart at arbitrary byte offsets, so the copy works row by row,
// with no tiles and no halo.
//
// Work split.  A workgroup of 256 threads (4 waves) takes 16 consecutive
// rows of one slab (x_3 fixed for m = 3); wave w takes rows 4w .. 4w+3 of
// them, one 1 KiB piece of each row per pass (lane l: bytes 16 l .. 16 l + 15
// of the piece, as one unaligned 16-byte access, like the automata's
// lanes), the four loads of a pass issued before its stores.  A lane whose
// 16 bytes all belong to the row copies them with one 16-byte load and
// store; the lane that the row's end cuts loads 16 bytes (within the
// buffer for n >= 15: the last row starts at least 16 bytes before the end
// of the box) and stores whole dwords, then single bytes; lanes past the
// end do nothing.  Boxes with n < 15 copy byte by byte.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smap {

constexpr int kCopyRowsPerWg = 16;   // rows per workgroup (4 per wave)

// Grid: (ceil((n+1) / 16), n+1 for m = 3 or 1 for m = 2); x = block of 16
// rows y, y = the slab z.
template <int M>
__global__ __launch_bounds__(256) void k_simplex_copy(int32_t n, int64_t pitch, const uint8_t *__restrict__ in,
                                                      uint8_t *__restrict__ out)
{
    const int32_t z = (M == 3) ? (int32_t)blockIdx.y : 0;
    const int32_t yw = (int32_t)blockIdx.x * kCopyRowsPerWg + 4 * (int32_t)(threadIdx.x >> 6);
    const int32_t len0 = n + 1 - yw - z;                  // the wave's longest row (uniform)
    if (len0 <= 0) return;
    const int lane = threadIdx.x & 63;
    const int64_t slab = (int64_t)z * pitch * pitch;

    if (n < 15) {                                         // tiny boxes: byte by byte
        for (int r = 0; r < 4; ++r) {
            const int64_t base = slab + (int64_t)(yw + r) * pitch;
            for (int32_t x = lane; x < len0 - r; x += 64) out[base + x] = in[base + x];
        }
        return;
    }
    for (int32_t p = 0; 1024 * p < len0; ++p) {           // 1 KiB pieces of the rows
        uint4 v[4];
        int32_t left[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            left[r] = len0 - r - (1024 * p + 16 * lane);  // row bytes from this lane's first on
            if (left[r] > 0)
                v[r] = *reinterpret_cast<const uint4 *>(in + slab + (int64_t)(yw + r) * pitch + 1024 * p + 16 * lane);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (left[r] <= 0) continue;
            uint8_t *d = out + slab + (int64_t)(yw + r) * pitch + 1024 * p + 16 * lane;
            if (left[r] >= 16) {
                *reinterpret_cast<uint4 *>(d) = v[r];
            } else {
                const uint32_t w[4] = {v[r].x, v[r].y, v[r].z, v[r].w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int32_t k = left[r] - 4 * i;    // bytes of dword i in the row
                    if (k >= 4) {
                        *reinterpret_cast<uint32_t *>(d + 4 * i) = w[i];
                    } else if (k > 0) {
#pragma unroll
                        for (int b = 0; b < 3; ++b)
                            if (b < k) d[4 * i + b] = (uint8_t)(w[i] >> (8 * b));
                    }
                }
            }
        }
    }
}

}  // namespace smap
