// panel.h -- the row-panel storage of the data matrix shared by the
// single-pass kernels (fused.hip, pass.hip): panel b holds rows
// [b*PR, b*PR + PR) of ldp >= N columns, the PR values of each column
// contiguous in 16 bytes (PR = 2, 4, 8, 16 for FP64, FP32, BF16, FP8 codes),
// so a wave reading 64 consecutive columns of a panel reads 1 KiB of
// contiguous memory.  Element codecs and the wave reductions of the pass.
#pragma once

#include <float.h>
#include <hip/hip_bf16.h>
#include <math.h>

#include <type_traits>

#include "internal.h"

namespace gspca {

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// Element codecs of a 16-byte panel segment (PR rows of one column).
struct CodecF64 {
    using acc = double;
    using raw = f64x2_t;
    static constexpr int PR = 2;
    static constexpr bool scaled = false;
    __device__ static inline void decode(const raw &v, acc (&o)[PR]) { o[0] = v[0]; o[1] = v[1]; }
};
struct CodecF32 {
    using acc = float;
    using raw = f32x4_t;
    static constexpr int PR = 4;
    static constexpr bool scaled = false;
    __device__ static inline void decode(const raw &v, acc (&o)[PR])
    {
        o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
    }
};
// bfloat16: the upper half of a binary32, so decoding is a shift.
struct CodecBF16 {
    using acc = float;
    using raw = u32x4_t;
    static constexpr int PR = 8;
    static constexpr bool scaled = true;
    __device__ static inline void decode(const raw &v, acc (&o)[PR])
    {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            o[2 * i] = __uint_as_float(v[i] << 16);
            o[2 * i + 1] = __uint_as_float(v[i] & 0xFFFF0000u);
        }
    }
    __device__ static inline float decode_one(const unsigned char *seg, int r)
    {
        const unsigned short h = reinterpret_cast<const unsigned short *>(seg)[r];
        return __uint_as_float((unsigned int)h << 16);
    }
};
// OCP E4M3 (gfx950 converts it in hardware, two codes per instruction).
struct CodecFP8 {
    using acc = float;
    using raw = u32x4_t;
    static constexpr int PR = 16;
    static constexpr bool scaled = true;
    __device__ static inline void decode(const raw &v, acc (&o)[PR])
    {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const f32x2_t lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)v[i], false);
            const f32x2_t hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)v[i], true);
            o[4 * i] = lo[0];
            o[4 * i + 1] = lo[1];
            o[4 * i + 2] = hi[0];
            o[4 * i + 3] = hi[1];
        }
    }
    __device__ static inline float decode_one(const unsigned char *seg, int r)
    {
        const unsigned int word = reinterpret_cast<const unsigned int *>(seg)[r >> 2];
        const f32x2_t pr = ((r >> 1) & 1) ? __builtin_amdgcn_cvt_pk_f32_fp8((int)word, true)
                                          : __builtin_amdgcn_cvt_pk_f32_fp8((int)word, false);
        return (r & 1) ? pr[1] : pr[0];
    }
};

template <typename T>
__device__ inline T fwave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}


// Sums of the PR values v[r] over the 64 lanes of a wave, scattered over the
// lanes: the first log2(PR) exchange steps (lane offsets 32, 16, ...) each
// keep half of the rows -- the lower half where the offset bit of the lane is
// clear -- and add the partner's copy of that half; the remaining offsets
// complete the one row left.  Lane l ends with the total of row `row` (read
// from the offset bits of l); 6 + PR - 2 shuffles instead of 6 PR.
template <typename T, int PR>
__device__ inline T wave_scatter_sum(const T (&v)[PR], int lane, int &row)
{
    T cur[PR];
#pragma unroll
    for (int r = 0; r < PR; ++r)
        cur[r] = v[r];
    int r0 = 0;
    int o = 32;
#pragma unroll
    for (int h = PR / 2; h >= 1; h >>= 1, o >>= 1) {
        const bool up = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < h; ++i) {
            const T keep = up ? cur[i + h] : cur[i];
            const T send = up ? cur[i] : cur[i + h];
            cur[i] = keep + __shfl_xor(send, o, 64);
        }
        r0 += up ? h : 0;
    }
    T x = cur[0];
#pragma unroll
    for (int oo = 64 / PR / 2; oo > 0; oo >>= 1)
        x += __shfl_xor(x, oo, 64);
    row = r0;
    return x;
}

// Panels of at least this many rows (FP8) reduce t with wave_scatter_sum:
// at 65536 x 8192 the FP8 pass went from 140 to 128 us; for BF16 the extra
// registers cost more than the shuffles saved (191 -> 196 us).
constexpr int kScatterMinRows = 16;

// Element (m, j) of the panel matrix in the arithmetic type (scaled for codes).
template <class C>
__device__ inline typename C::acc panel_elem(const unsigned char *A, int64_t ldp, int64_t m,
                                             int64_t j, const float *scale)
{
    const unsigned char *seg = A + ((m / C::PR) * ldp + j) * 16;
    const int r = (int)(m % C::PR);
    if constexpr (C::scaled)
        return C::decode_one(seg, r) * scale[j];
    else
        return reinterpret_cast<const typename C::acc *>(seg)[r];
}

static inline unsigned fcdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

template <int F> struct CodecOf;
template <> struct CodecOf<kFmtF64> { using type = CodecF64; };
template <> struct CodecOf<kFmtF32> { using type = CodecF32; };
template <> struct CodecOf<kFmtBF16> { using type = CodecBF16; };
template <> struct CodecOf<kFmtFP8> { using type = CodecFP8; };

}  // namespace gspca
