// Device-side building blocks of the gfx950 preconditioned-DCA library.
//
// The hot path is one kernel per sweep.  It forms Z = What V for the normalized
// weights What = D^{-1/2} W D^{-1/2} (so L_s V = V - Z, Section 2.2), and fuses in
// the same pass the right-hand side b = c u - (u^3 - u)/eps + eta Lambda y (Prop. 1),
// the residual r = b - T v with T = eps L_s + eta Lambda + c I (Section 3), the
// diagonal update v + r/g (Section 3.1) and the block partial sums of |r|^2 and of
// the energy terms (Section 2.1).
//
// The row kernels of each operator layout (direct CSR, tile, grid, window) are
// in their own headers; this one holds the storage types, row loads and stores
// and the fixed-order wavefront and block reductions they share.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gl {

// ----------------------------------------------------------------------------
// storage types
// ----------------------------------------------------------------------------
struct bf16 {
    uint16_t bits;
};
typedef _Float16 f16;

template <typename T> struct acc_of { typedef float type; };
template <> struct acc_of<double> { typedef double type; };

template <typename A> __device__ __forceinline__ A cvt(double x) { return (A)x; }
template <typename A> __device__ __forceinline__ A cvt(float x) { return (A)x; }
template <typename A> __device__ __forceinline__ A cvt(f16 x) { return (A)(float)x; }
template <typename A> __device__ __forceinline__ A cvt(bf16 x) {
    return (A)__uint_as_float((uint32_t)x.bits << 16);
}

// The value of a 16-bit load, opaque to the optimizer from here on, so that
// its conversion to the accumulator type stays where the value is used:
// moved up next to the load, the conversion would bring the wait for that load
// ahead of later requests.  Wider types need no conversion.
__device__ __forceinline__ float late(float x) { return x; }
__device__ __forceinline__ double late(double x) { return x; }
__device__ __forceinline__ f16 late(f16 x) {
    uint32_t b = __builtin_bit_cast(uint16_t, x);
    asm volatile("" : "+v"(b));
    return __builtin_bit_cast(f16, (uint16_t)b);
}
__device__ __forceinline__ bf16 late(bf16 x) {
    uint32_t b = x.bits;
    asm volatile("" : "+v"(b));
    return bf16{(uint16_t)b};
}

template <typename T> struct store_as;
template <> struct store_as<double> {
    static __device__ __forceinline__ double from(double x) { return x; }
    static __device__ __forceinline__ double from(float x) { return (double)x; }
};
template <> struct store_as<float> {
    static __device__ __forceinline__ float from(float x) { return x; }
    static __device__ __forceinline__ float from(double x) { return (float)x; }
};
// Single rounding (to nearest even) from double.  Normal results: round the
// double's significand to the target width on the bit pattern; the rounded
// value is then exact in float and in the target.  Subnormal results: round to
// the fixed quantum with rint (round-half-even in the default mode).
__device__ __forceinline__ float round_double_to_width(double x, int drop_bits, double min_normal,
                                                       double quantum_inv, double quantum) {
    const double ax = fabs(x);
    if (!(ax >= min_normal)) {
        if (x != x) return __builtin_nanf("");
        return (float)(rint(x * quantum_inv) * quantum);
    }
    uint64_t d = (uint64_t)__double_as_longlong(x);
    const uint64_t half = (1ull << (drop_bits - 1)) - 1ull;
    d += half + ((d >> drop_bits) & 1ull);
    d &= ~((1ull << drop_bits) - 1ull);
    return (float)__longlong_as_double((long long)d);
}

template <> struct store_as<f16> {
    // round to nearest even (the default rounding of the conversion)
    static __device__ __forceinline__ f16 from(float x) { return (f16)x; }
    static __device__ __forceinline__ f16 from(double x) {
        if (fabs(x) > 65504.0) return (f16)(float)x;
        // 10 stored significand bits: drop 42 of the double's 52
        return (f16)round_double_to_width(x, 42, 6.103515625e-05, 16777216.0, 5.9604644775390625e-08);
    }
};
template <> struct store_as<bf16> {
    // round to nearest even on the bit pattern; NaN stays NaN
    static __device__ __forceinline__ bf16 from(float x) {
        uint32_t u = __float_as_uint(x);
        if ((u & 0x7fffffffu) > 0x7f800000u) return bf16{(uint16_t)((u >> 16) | 0x40u)};
        u += 0x7fffu + ((u >> 16) & 1u);
        return bf16{(uint16_t)(u >> 16)};
    }
    static __device__ __forceinline__ bf16 from(double x) {
        if (fabs(x) > 3.0e38) return from((float)x);
        // 7 stored significand bits: drop 45 of the double's 52; quantum 2^-133 below 2^-126
        const float f = round_double_to_width(x, 45, 1.1754943508222875e-38,
                                              1.0889035741470030e+40, 9.1835496157991212e-41);
        return bf16{(uint16_t)(__float_as_uint(f) >> 16)};
    }
};

// ----------------------------------------------------------------------------
// vector gather of one K-wide row of V
// ----------------------------------------------------------------------------
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <int B> struct chunk_t;
template <> struct chunk_t<16> { typedef u32x4 type; };
template <> struct chunk_t<8> { typedef u32x2 type; };
template <> struct chunk_t<4> { typedef uint32_t type; };
template <> struct chunk_t<2> { typedef uint16_t type; };

template <int K, typename T, typename A>
__device__ __forceinline__ void load_row(const T* __restrict__ p, A (&out)[K]) {
    constexpr int RB = K * (int)sizeof(T);
    constexpr int CB = (RB % 16 == 0) ? 16 : (RB % 8 == 0) ? 8 : (RB % 4 == 0) ? 4 : 2;
    typedef typename chunk_t<CB>::type C;
    C buf[RB / CB];
    const C* src = reinterpret_cast<const C*>(p);
#pragma unroll
    for (int c = 0; c < RB / CB; ++c) buf[c] = src[c];
    T vals[K];
    __builtin_memcpy(vals, buf, RB);
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = cvt<A>(vals[k]);
}

// K values of one row as stored, without conversion.
template <int K, typename T>
__device__ __forceinline__ void load_raw(const T* __restrict__ p, T (&out)[K]) {
    constexpr int RB = K * (int)sizeof(T);
    constexpr int CB = (RB % 16 == 0) ? 16 : (RB % 8 == 0) ? 8 : (RB % 4 == 0) ? 4 : 2;
    typedef typename chunk_t<CB>::type C;
    C buf[RB / CB];
    const C* src = reinterpret_cast<const C*>(p);
#pragma unroll
    for (int c = 0; c < RB / CB; ++c) buf[c] = src[c];
    __builtin_memcpy(out, buf, RB);
}

// K values of one row, stored as they are in as few vector stores as the row's
// size allows.
template <int K, typename T>
__device__ __forceinline__ void store_raw(T* __restrict__ p, const T (&in)[K]) {
    constexpr int RB = K * (int)sizeof(T);
    constexpr int CB = (RB % 16 == 0) ? 16 : (RB % 8 == 0) ? 8 : (RB % 4 == 0) ? 4 : 2;
    typedef typename chunk_t<CB>::type C;
    C buf[RB / CB];
    __builtin_memcpy(buf, in, RB);
    C* dst = reinterpret_cast<C*>(p);
#pragma unroll
    for (int c = 0; c < RB / CB; ++c) dst[c] = buf[c];
}

// Fused multiply-add with one rounding, written out where the result must not
// depend on how the compiler contracts an expression in a given kernel.
__device__ __forceinline__ float fma_acc(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_acc(double a, double b, double c) { return __builtin_fma(a, b, c); }

// runtime-index read of a register array without spilling it to scratch
template <int K, typename A>
__device__ __forceinline__ A pick(const A (&z)[K], int k) {
    A r = z[0];
#pragma unroll
    for (int i = 1; i < K; ++i) r = (k == i) ? z[i] : r;
    return r;
}

// The same pointer, known to address global memory: a pointer read from memory
// (rather than passed as a kernel argument) is otherwise accessed with flat
// instructions, and every wait for a flat load waits for all outstanding
// loads and LDS operations alike.  The round trip through the global address
// space lets the compiler's address-space inference use global loads.
template <typename T> __device__ __forceinline__ T* as_global(T* p) {
    typedef __attribute__((address_space(1))) T* G;
    return (T*)(G)(uintptr_t)p;
}

// Hardware dispatch hands consecutive workgroup ids round-robin to the 8 XCDs.
// Give every XCD a contiguous range of logical blocks so that the rows it works
// on at any moment, and the V rows they gather, stay in that XCD's own L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
    const int64_t q = nb >> 3, r = nb & 7;
    const int64_t x = b & 7, i = b >> 3;
    return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Sum over the 64 lanes of a wavefront in a fixed order, with DPP lane moves
// (no LDS traffic); the total is valid in lane 63.  Steps: lane ^ 1, lane ^ 2,
// mirror within 8 lanes, mirror within 16 lanes (every lane then holds its
// row's sum), rows 1 and 3 add the last lane of rows 0 and 2, rows 2 and 3
// add lane 31.
template <int CTRL, int ROWS> __device__ __forceinline__ int dpp_mov(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, false);  // 0 in rows outside ROWS
}

template <int CTRL, int ROWS, typename A> __device__ __forceinline__ A dpp_add(A x) {
    if constexpr (sizeof(A) == 4) {
        return x + __builtin_bit_cast(A, dpp_mov<CTRL, ROWS>(__builtin_bit_cast(int, x)));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, x);
        const uint32_t lo = (uint32_t)dpp_mov<CTRL, ROWS>((int)(uint32_t)u);
        const uint32_t hi = (uint32_t)dpp_mov<CTRL, ROWS>((int)(uint32_t)(u >> 32));
        return x + __builtin_bit_cast(A, ((uint64_t)hi << 32) | lo);
    }
}

template <typename A> __device__ __forceinline__ A wave_sum63(A x) {
    x = dpp_add<0xb1, 0xf>(x);   // quad_perm [1, 0, 3, 2]
    x = dpp_add<0x4e, 0xf>(x);   // quad_perm [2, 3, 0, 1]
    x = dpp_add<0x141, 0xf>(x);  // row_half_mirror
    x = dpp_add<0x140, 0xf>(x);  // row_mirror
    x = dpp_add<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
    return dpp_add<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
}

// Largest value of a non-negative int over the wavefront (same steps), as a
// wave-uniform value.
__device__ __forceinline__ int wave_max_nonneg(int x) {
    x = max(x, dpp_mov<0xb1, 0xf>(x));
    x = max(x, dpp_mov<0x4e, 0xf>(x));
    x = max(x, dpp_mov<0x141, 0xf>(x));
    x = max(x, dpp_mov<0x140, 0xf>(x));
    x = max(x, dpp_mov<0x142, 0xa>(x));
    x = max(x, dpp_mov<0x143, 0xc>(x));
    return __builtin_amdgcn_readlane(x, 63);
}

// x + x of lane (lane ^ off), the partner's value added to this lane's: a DPP
// quad permute for off = 1 and 2 (the same lane pairs as the shuffle, without
// an LDS permute; every lane of the wavefront must be active), the shuffle
// otherwise.  For compile-time offsets only: with a run-time offset the tests
// cost more than the permutes save.
template <typename A> __device__ __forceinline__ A xor_add(A x, int off) {
    if (off == 1) return dpp_add<0xb1, 0xf>(x);
    if (off == 2) return dpp_add<0x4e, 0xf>(x);
    return x + __shfl_xor(x, off, 64);
}

// The value of lane (lane ^ OFF) within aligned groups of 2 OFF lanes, by DPP
// moves where the pattern allows (every lane of the wavefront must be active):
// OFF = 1, 2 quad permutes; 4 = mirror within 8 lanes, then reverse within 4
// (i ^ 7 ^ 3); 8 = mirror within 16, then within 8 (i ^ 15 ^ 7); larger
// offsets cross DPP rows and use the LDS permute.
template <int OFF> __device__ __forceinline__ int xor_partner32(int v) {
    if constexpr (OFF == 1) return dpp_mov<0xb1, 0xf>(v);
    else if constexpr (OFF == 2) return dpp_mov<0x4e, 0xf>(v);
    else if constexpr (OFF == 4) return dpp_mov<0x1b, 0xf>(dpp_mov<0x141, 0xf>(v));
    else if constexpr (OFF == 8) return dpp_mov<0x141, 0xf>(dpp_mov<0x140, 0xf>(v));
    else return __shfl_xor(v, OFF, 64);
}

template <int OFF, typename A> __device__ __forceinline__ A xor_partner(A x) {
    if constexpr (sizeof(A) == 4) {
        return __builtin_bit_cast(A, xor_partner32<OFF>(__builtin_bit_cast(int, x)));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, x);
        const uint32_t lo = (uint32_t)xor_partner32<OFF>((int)(uint32_t)u);
        const uint32_t hi = (uint32_t)xor_partner32<OFF>((int)(uint32_t)(u >> 32));
        return __builtin_bit_cast(A, ((uint64_t)hi << 32) | lo);
    }
}

// Butterfly over aligned groups of G = 2^log2G lanes (4 <= G <= 64): every
// lane of a group ends with the group's sum of z[k], added in the same order
// as the shuffle form z[k] += shfl_xor(z[k], off) for off = G/2, ..., 1.
template <int L2, int K, typename A> __device__ __forceinline__ void butterfly_fixed(A (&z)[K]) {
    if constexpr (L2 > 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) z[k] += xor_partner<(1 << (L2 - 1))>(z[k]);
        butterfly_fixed<L2 - 1, K>(z);
    }
}

template <int K, typename A> __device__ __forceinline__ void group_butterfly(A (&z)[K], int log2G) {
    switch (log2G) {
        case 2: butterfly_fixed<2, K>(z); break;
        case 3: butterfly_fixed<3, K>(z); break;
        case 4: butterfly_fixed<4, K>(z); break;
        case 5: butterfly_fixed<5, K>(z); break;
        default: butterfly_fixed<6, K>(z); break;
    }
}

// Sum the per-lane column partials of a 256-thread block.  Lane q of every group
// holds columns q, q+G, ...; after the cross-group swaps lanes 0..G-1 of each
// wavefront hold the wavefront's sums, which four LDS slots combine in wavefront
// order.  Thread s < 2K writes statistic s (energies then residuals) of this block.
template <int K, int CPL, typename A>
__device__ __forceinline__ void block_stats(A (&e)[CPL], A (&r)[CPL], int G, A* __restrict__ partials,
                                            int64_t nb, int64_t b) {
    __shared__ A sh[4][2][K];
    for (int off = G; off < 64; off <<= 1) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            e[c] += __shfl_xor(e[c], off, 64);
            r[c] += __shfl_xor(r[c], off, 64);
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < G) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int k = lane + c * G;
            if (k < K) {
                sh[wave][0][k] = e[c];
                sh[wave][1][k] = r[c];
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * K) {
        const int kind = threadIdx.x / K, k = threadIdx.x - kind * K;
        const A s = ((sh[0][kind][k] + sh[1][kind][k]) + sh[2][kind][k]) + sh[3][kind][k];
        partials[(int64_t)threadIdx.x * nb + b] = s;
    }
}

}  // namespace gl
