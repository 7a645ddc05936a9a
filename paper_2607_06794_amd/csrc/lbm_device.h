// Device-side lattice constants and population storage codecs for gfx950.
//
// D3Q19 velocity set (the discrete velocities c_i of the lattice Boltzmann
// equation, Eq. 1) with weights w_i of the second-order equilibrium (Eq. 2),
// c_s^2 = 1/3.  Direction order: rest; +x,-x,+y,-y,+z,-z; then the twelve
// (+-1,+-1,0)-type permutations with each direction followed by its opposite.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 19;

// Components of c_i, two bits per direction (value + 1) in one constant, so
// that a run-time index costs a shift and a mask instead of a table in
// private memory.
__host__ __device__ constexpr int cx(int i) { return int((0x1548889549ull >> (2 * i)) & 3ull) - 1; }
__host__ __device__ constexpr int cy(int i) { return int((0x895609495ull >> (2 * i)) & 3ull) - 1; }
__host__ __device__ constexpr int cz(int i) { return int((0x20A0954955ull >> (2 * i)) & 3ull) - 1; }
// opposite direction: pairs (1,2), (3,4), ... are adjacent
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// compile-time check of the encoded velocity set: c_0 = 0, opposite pairs,
// six axis and twelve edge directions
constexpr bool d3q19_ok() {
    int axis = 0, edge = 0;
    for (int i = 1; i < Q; ++i) {
        if (cx(opp(i)) != -cx(i) || cy(opp(i)) != -cy(i) || cz(opp(i)) != -cz(i)) return false;
        const int n2 = cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i);
        axis += n2 == 1;
        edge += n2 == 2;
    }
    return cx(0) == 0 && cy(0) == 0 && cz(0) == 0 && axis == 6 && edge == 12;
}
static_assert(d3q19_ok(), "D3Q19 velocity set");

template <class C>
__host__ __device__ constexpr C wgt(int i) {
    return i == 0 ? C(1) / C(3) : (i <= 6 ? C(1) / C(18) : C(1) / C(36));
}

// material byte: low nibble = material id, bit 7 = fluid node next to a static wall
constexpr uint8_t MAT_FLUID = 0, MAT_GHOST = 1, MAT_ROD = 8;
constexpr uint8_t MAT_ID_MASK = 0x0F, MAT_NEAR_WALL = 0x80;
__host__ __device__ inline bool is_static_wall(uint8_t id) { return id >= 2 && id <= 7; }

// status bits
constexpr unsigned ST_NAN = 1u, ST_RHO = 2u, ST_SPEED = 4u, ST_ROD = 8u, ST_ROD_WALL = 16u, ST_ROD_LIST = 32u;
// notice, not a fault: an uncovered node had no fluid neighbour and took its
// densities from a farther ring (a pocket enclosed by touching capsules)
constexpr unsigned ST_REFILL_FAR = 64u;
constexpr unsigned ST_NOTICES = ST_REFILL_FAR;

// ---------------------------------------------------------------------------
// storage codecs: S = element type in HBM, C = compute type in registers.
// The kernels store and compute the deviation d_i = f_i - w_i*rho_ref[k]
// (rho_ref = 0 stores f_i itself); the codecs only convert d_i between the
// storage and the compute type.
// ---------------------------------------------------------------------------
struct bf16_t {
    uint16_t bits;
};

template <class S>
struct Codec;

template <>
struct Codec<double> {
    using C = double;
    __device__ static inline double dec(double s) { return s; }
    __device__ static inline double enc(double v) { return v; }
};

template <>
struct Codec<float> {
    using C = float;
    __device__ static inline float dec(float s) { return s; }
    __device__ static inline float enc(float v) { return v; }
};

// IEEE half, round to nearest even (hardware conversion)
template <>
struct Codec<_Float16> {
    using C = float;
    __device__ static inline float dec(_Float16 s) { return static_cast<float>(s); }
    __device__ static inline _Float16 enc(float v) { return static_cast<_Float16>(v); }
};

// bfloat16, round to nearest even on the float bit pattern
template <>
struct Codec<bf16_t> {
    using C = float;
    __device__ static inline float dec(bf16_t s) { return __uint_as_float(static_cast<uint32_t>(s.bits) << 16); }
    __device__ static inline bf16_t enc(float d) {
        uint32_t u = __float_as_uint(d);
        bf16_t r;
        if ((u & 0x7f800000u) == 0x7f800000u) {  // inf or nan: keep, quiet the nan
            r.bits = static_cast<uint16_t>((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
        } else {
            u += 0x7fffu + ((u >> 16) & 1u);
            r.bits = static_cast<uint16_t>(u >> 16);
        }
        return r;
    }
};

// ---------------------------------------------------------------------------
// stochastic rounding of the 16-bit storage forms: a value between two
// neighbouring representable numbers goes to the upper one with probability
// equal to its distance from the lower one in units of their spacing, so the
// stored errors have zero mean (round to nearest biases the mass of a state
// whose values cluster).  The random bits come from a counter-based hash of
// (node, population array, step); the same key always gives the same result.
// ---------------------------------------------------------------------------
__device__ inline uint32_t hash32(uint32_t x) {
    // xorshift-multiply finaliser (two 32-bit multiplies, three shifts)
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
__device__ inline uint32_t sr_bits(uint32_t step_key, int64_t node, int array) {
    return hash32(uint32_t(node) * 38u + uint32_t(array) + hash32(step_key ^ uint32_t(node >> 32)));
}

template <class S>
struct Stochastic {
    // wider storage rounds exactly as the plain codec
    __device__ static inline S enc(typename Codec<S>::C v, uint32_t) { return Codec<S>::enc(v); }
};

// IEEE half: round to nearest of v + (r - 1/2) ulp(v), r uniform on 13 bits,
// is the upper neighbour with probability (v - lower) / ulp; the shift is
// exact in FP32 (ulp of half = 2^13 ulp of float in the same binade, and a
// fixed 2^-24 below the normal range)
template <>
struct Stochastic<_Float16> {
    __device__ static inline _Float16 enc(float v, uint32_t r) {
        const uint32_t u = __float_as_uint(v);
        const int e = int((u >> 23) & 0xFFu) - 127;  // binade of |v|
        const int ue = e - 10 < -24 ? -24 : e - 10;  // exponent of the half spacing
        if (e > 15) return static_cast<_Float16>(v);  // beyond the half range: plain conversion
        const float ulp = __uint_as_float(uint32_t(ue + 127) << 23);
        const float dither = (float(int(r >> 19)) * (1.0f / 8192.0f) - 0.5f) * ulp;
        return static_cast<_Float16>(v + dither);
    }
};

// bfloat16: add 16 random bits below the kept ones and truncate
template <>
struct Stochastic<bf16_t> {
    __device__ static inline bf16_t enc(float d, uint32_t r) {
        uint32_t u = __float_as_uint(d);
        bf16_t o;
        if ((u & 0x7f800000u) == 0x7f800000u) {
            o.bits = static_cast<uint16_t>((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
        } else {
            u += r & 0xffffu;
            o.bits = static_cast<uint16_t>(u >> 16);
        }
        return o;
    }
};

}  // namespace lbm
