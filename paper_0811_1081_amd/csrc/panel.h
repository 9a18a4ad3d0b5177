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

// ---- Cross-lane sums without the LDS crossbar.  Every exchange pairs lane l
// with lane l ^ O, the pairs __shfl_xor(x, O) would form, so the sums (and
// their rounding) are the same: distances 32 and 16 swap register halves
// between lanes (v_permlane32_swap, v_permlane16_swap), 8 and 4 move values
// between the lower and upper half of each group of 2 O lanes with
// bank-masked DPP row shifts (a bank is 4 lanes of a 16-lane row), 2 and 1
// use DPP quad permutes.  64-bit values move as two 32-bit words.

template <typename T> struct LaneWords { static constexpr int n = sizeof(T) / 4; };

template <typename T>
__device__ inline void to_words(T v, unsigned (&w)[LaneWords<T>::n])
{
    __builtin_memcpy(w, &v, sizeof(T));
}

template <typename T>
__device__ inline T from_words(const unsigned (&w)[LaneWords<T>::n])
{
    T v;
    __builtin_memcpy(&v, w, sizeof(T));
    return v;
}

// For the pair (a, b): lanes whose index has bit O clear return
// a + (the partner's a), lanes with the bit set (the partner's b) + b.
template <int O, typename T>
__device__ inline T pair_sum(T a, T b, int lane)
{
    constexpr int W = LaneWords<T>::n;
    unsigned wa[W], wb[W];
    to_words(a, wa);
    to_words(b, wb);
    if constexpr (O == 32 || O == 16) {
        // lanes of the upper half of a's register trade places with lanes of
        // the lower half of b's
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const auto r = O == 32 ? __builtin_amdgcn_permlane32_swap(wa[i], wb[i], false, false)
                                   : __builtin_amdgcn_permlane16_swap(wa[i], wb[i], false, false);
            wa[i] = r[0];
            wb[i] = r[1];
        }
        return from_words<T>(wa) + from_words<T>(wb);
    } else if constexpr (O == 8 || O == 4) {
        // row_shl:O (lane i reads lane i + O) into the lower-half banks,
        // row_shr:O (lane i reads lane i - O) into the upper-half banks
        constexpr int lo = O == 8 ? 0x3 : 0x5, hi = O == 8 ? 0xC : 0xA;
        unsigned na[W], nb[W];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            nb[i] = (unsigned)__builtin_amdgcn_update_dpp((int)wb[i], (int)wa[i], 0x100 + O, 0xF,
                                                          lo, false);
            na[i] = (unsigned)__builtin_amdgcn_update_dpp((int)wa[i], (int)wb[i], 0x110 + O, 0xF,
                                                          hi, false);
        }
        return from_words<T>(na) + from_words<T>(nb);
    } else {
        static_assert(O == 2 || O == 1, "lane distance");
        const bool up = (lane & O) != 0;
        const T keep = up ? b : a, send = up ? a : b;
        unsigned ws[W];
        to_words(send, ws);
#pragma unroll
        for (int i = 0; i < W; ++i) // quad_perm [2,3,0,1] / [1,0,3,2]
            ws[i] = (unsigned)__builtin_amdgcn_mov_dpp((int)ws[i], O == 2 ? 0x4E : 0xB1, 0xF, 0xF,
                                                       false);
        return keep + from_words<T>(ws);
    }
}

// x + (lane l ^ O's x) in every lane l.
template <int O, typename T>
__device__ inline T xor_add(T x)
{
    if constexpr (O >= 4) {
        return pair_sum<O>(x, x, 0);
    } else {
        constexpr int W = LaneWords<T>::n;
        unsigned ws[W];
        to_words(x, ws);
#pragma unroll
        for (int i = 0; i < W; ++i)
            ws[i] = (unsigned)__builtin_amdgcn_mov_dpp((int)ws[i], O == 2 ? 0x4E : 0xB1, 0xF, 0xF,
                                                       false);
        return x + from_words<T>(ws);
    }
}

template <int O, typename T>
__device__ inline T fold_from(T x)
{
    if constexpr (O >= 1)
        return fold_from<O / 2>(xor_add<O>(x));
    else
        return x;
}

// Sum over the 64 lanes of a wave, in every lane (lane distances 32, 16, ..., 1).
template <typename T>
__device__ inline T fwave_sum(T v)
{
    return fold_from<32>(v);
}

template <int H, int O, typename T, int PR>
__device__ inline void scatter_halve(T (&cur)[PR], int lane, int &r0)
{
    if constexpr (H >= 1) {
#pragma unroll
        for (int i = 0; i < H; ++i)
            cur[i] = pair_sum<O>(cur[i], cur[i + H], lane);
        r0 += (lane & O) ? H : 0;
        scatter_halve<H / 2, O / 2>(cur, lane, r0);
    }
}

// Sums of the PR values v[r] over the 64 lanes of a wave, scattered over the
// lanes: the first log2(PR) exchange steps (lane distances 32, 16, ...) each
// keep half of the rows -- the lower half where the distance bit of the lane
// is clear -- and add the partner's copy of that half; the remaining
// distances complete the one row left.  Lane l ends with the total of row
// `row` (read from the distance bits of l); PR - 1 + 6 - log2(PR) exchanges
// instead of 6 PR.
template <typename T, int PR>
__device__ inline T wave_scatter_sum(const T (&v)[PR], int lane, int &row)
{
    T cur[PR];
#pragma unroll
    for (int r = 0; r < PR; ++r)
        cur[r] = v[r];
    int r0 = 0;
    scatter_halve<PR / 2, 32>(cur, lane, r0);
    row = r0;
    return fold_from<64 / PR / 2>(cur[0]);
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
