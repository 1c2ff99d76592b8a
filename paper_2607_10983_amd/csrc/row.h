// Helpers shared by the row-wave kernels (one wavefront per full x-row of a
// periodic level, lane l holding VEC = n/64 contiguous elements): vector row
// accesses, the rotating cross-lane move that supplies x-neighbours, the
// wave index as a scalar, XCD-aware block renumbering and row addressing.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace mg {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));

// Row segment of VEC contiguous elements through 16-byte (or 8/4-byte) vector
// accesses.  Plain cached accesses: measured faster than non-temporal ones
// here, since streaming hints keep the fields out of the Infinity Cache.
template <typename T, int VEC>
__device__ __forceinline__ void ldrow(T (&v)[VEC], const T* p) {
    constexpr int B = VEC * (int)sizeof(T);
    if constexpr (B >= 16) {
#pragma unroll
        for (int k = 0; k < B / 16; ++k) {
            const v4i t = *(reinterpret_cast<const v4i*>(p) + k);
            __builtin_memcpy(&v[k * 16 / (int)sizeof(T)], &t, 16);
        }
    } else if constexpr (B == 8) {
        const v2i t = *reinterpret_cast<const v2i*>(p);
        __builtin_memcpy(&v[0], &t, 8);
    } else {
        v[0] = p[0];
    }
}

template <typename T, int VEC>
__device__ __forceinline__ void strow(T* p, const T (&v)[VEC]) {
    constexpr int B = VEC * (int)sizeof(T);
    if constexpr (B >= 16) {
#pragma unroll
        for (int k = 0; k < B / 16; ++k) {
            v4i t;
            __builtin_memcpy(&t, &v[k * 16 / (int)sizeof(T)], 16);
            *(reinterpret_cast<v4i*>(p) + k) = t;
        }
    } else if constexpr (B == 8) {
        v2i t;
        __builtin_memcpy(&t, &v[0], 8);
        *reinterpret_cast<v2i*>(p) = t;
    } else {
        p[0] = v[0];
    }
}

// Rotating cross-lane move: value of lane (lane + delta) mod 64, delta = +1
// or -1.  A DPP move across the whole wave (wave_rol:1 brings lane + 1,
// wave_ror:1 lane - 1): plain VALU, no trip through the LDS crossbar.
__device__ __forceinline__ int lane_rot32(int v, int delta) {
    return delta > 0 ? __builtin_amdgcn_update_dpp(0, v, 0x134, 0xF, 0xF, false)
                     : __builtin_amdgcn_update_dpp(0, v, 0x13C, 0xF, 0xF, false);
}
template <typename T>
__device__ __forceinline__ T lane_rot(T v, int delta) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, lane_rot32(__builtin_bit_cast(int, v), delta));
    } else {
        v2i h = __builtin_bit_cast(v2i, v);
        h.x = lane_rot32(h.x, delta);
        h.y = lane_rot32(h.y, delta);
        return __builtin_bit_cast(T, h);
    }
}

// Block id renumbering so that each XCD (blocks are dealt round-robin to the
// eight XCDs) receives a contiguous range of logical blocks.
__device__ __forceinline__ int xcd_logical(int bid, int nb) {
    if (nb & 7) return bid;
    return (bid & 7) * (nb >> 3) + (bid >> 3);
}

// Index of the calling wave in its block, as a wave-uniform (scalar) value:
// row and plane offsets derived from it are then formed by the scalar unit.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// A row's copy in LDS.  Rows of at most 16 bytes per lane keep the global
// layout (lane l at element l * VEC).  Longer rows are stored in 16-byte
// pieces with piece j of every lane together (lane l's piece j at element
// (j * 64 + l) * P), so that every 16-byte LDS access of a wave covers
// consecutive addresses instead of a lane stride of VEC elements, which
// conflicts on the LDS banks.
template <typename T, int VEC>
__device__ __forceinline__ void lds_strow(T* row, int lane, const T (&v)[VEC]) {
    constexpr int B = VEC * (int)sizeof(T);
    if constexpr (B <= 16) {
        strow<T, VEC>(row + (size_t)lane * VEC, v);
    } else {
        constexpr int P = 16 / (int)sizeof(T);
#pragma unroll
        for (int j = 0; j < VEC / P; ++j) {
            v4i t;
            __builtin_memcpy(&t, &v[j * P], 16);
            *reinterpret_cast<v4i*>(row + (size_t)(j * 64 + lane) * P) = t;
        }
    }
}
template <typename T, int VEC>
__device__ __forceinline__ void lds_ldrow(T (&v)[VEC], const T* row, int lane) {
    constexpr int B = VEC * (int)sizeof(T);
    if constexpr (B <= 16) {
        ldrow<T, VEC>(v, row + (size_t)lane * VEC);
    } else {
        constexpr int P = 16 / (int)sizeof(T);
#pragma unroll
        for (int j = 0; j < VEC / P; ++j) {
            const v4i t = *reinterpret_cast<const v4i*>(row + (size_t)(j * 64 + lane) * P);
            __builtin_memcpy(&v[j * P], &t, 16);
        }
    }
}

// Row addressing of a periodic n^3 level.  Every row kernel is instantiated
// for n = 64 * VEC (a lane holds VEC points of a row), so the kernels build
// it from VEC and its sizes are compile-time constants.
struct RowGrid {
    int n, mask;
    __device__ __forceinline__ size_t row(int y, int z) const {
        return ((size_t)(z & mask) * (size_t)n + (size_t)(y & mask)) * (size_t)n;
    }
};

}  // namespace mg
