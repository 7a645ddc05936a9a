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

// A pointer into device memory seen in the global address space.  Pointers
// read from an argument record are generic (flat) to the compiler, and a flat
// load also counts as an LDS/scalar access: any later wait for a scalar load
// then waits for it too, which serialises loads that could overlap.  Loads and
// stores through this view are global accesses, tracked on their own.
template <class T>
__device__ inline __attribute__((address_space(1))) T *gptr(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}
// one element read through that view (class types, such as bf16_t, as their bits)
template <class T>
__device__ inline T gload(const T *p) {
    if constexpr (__is_class(T)) {
        static_assert(sizeof(T) == 2, "2-byte storage types only");
        return __builtin_bit_cast(T, *gptr(reinterpret_cast<const uint16_t *>(p)));
    } else {
        return *gptr(p);
    }
}

// status bits
constexpr unsigned ST_NAN = 1u, ST_RHO = 2u, ST_SPEED = 4u, ST_ROD = 8u, ST_ROD_WALL = 16u, ST_ROD_LIST = 32u;
// notice, not a fault: an uncovered node had no fluid neighbour and took its
// densities from a farther ring (a pocket enclosed by touching capsules)
constexpr unsigned ST_REFILL_FAR = 64u;
constexpr unsigned ST_NOTICES = ST_REFILL_FAR;

// Adds per-node status bits to a lattice's status word.  `known` is the word
// as the kernel found it at its start: bits already set are not sent again,
// and the rest go out in one atomic per wavefront (the bits ORed over the
// active lanes by ballots), so a lattice that has gone bad everywhere costs
// no atomics at all after its first bad step (one per node and step to a
// single word made such a lattice several times slower than a healthy one).
// Every active lane of the wavefront calls it with its own bits.
__device__ inline void post_status(unsigned *status, unsigned known, unsigned st) {
    const unsigned fresh = st & ~known;
    if (__ballot(fresh != 0) == 0) return;
    unsigned w = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b)
        if (__ballot((fresh >> b) & 1u)) w |= 1u << b;
    const unsigned long long act = __ballot(1);
    if (__lane_id() == __ffsll(static_cast<long long>(act)) - 1) atomicOr(status, w);
}

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
// whose values cluster).  Random bits: a xorshift32 stream per node and step,
// seeded by a hash of (node, step key); each 32-bit draw serves two
// population arrays (16 bits each) in array order, so the bits of an element
// depend on (node, array, step) only.
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
// nonzero seed of a node's stream in the step keyed by step_key
__device__ inline uint32_t sr_seed(uint32_t step_key, int64_t node) {
    return hash32(uint32_t(node) ^ hash32(step_key ^ uint32_t(node >> 32))) | 1u;
}
// Marsaglia's xorshift32 (shifts 13, 17, 5): full period on nonzero states
__device__ inline uint32_t xorshift32(uint32_t x) {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}
// 16 random bits for population array arr (0, 1, 2, ... in order): even
// arrays advance the stream and take its low half, odd ones its high half
struct SrStream {
    uint32_t state, word;
    __device__ inline uint32_t bits(int arr) {
        if ((arr & 1) == 0) {
            state = xorshift32(state);
            word = state;
            return word & 0xffffu;
        }
        return word >> 16;
    }
};

template <class S>
struct Stochastic {
    // wider storage rounds exactly as the plain codec
    __device__ static inline S enc(typename Codec<S>::C v, uint32_t) { return Codec<S>::enc(v); }
};

// IEEE half from float, r: 16 random bits.  From 2^-14 up the float keeps
// 13 more fraction bits than the half: adding 13 random bits to the
// magnitude's bit pattern and clearing them rounds up with probability
// (v - lower) / spacing, and the conversion of the result is exact (a carry
// moves on into the exponent, the next representable number; beyond the
// half's range the conversion overflows as a plain one would).  Below 2^-14
// the half's spacing is the fixed 2^-24: there round to nearest of
// v + (r - 1/2) 2^-24, exact in float (a rarely taken branch).
template <>
struct Stochastic<_Float16> {
    __device__ static inline _Float16 enc(float v, uint32_t r) {
        const uint32_t u = __float_as_uint(v);
        if (__builtin_expect(((u >> 23) & 0xFFu) < 113u, 0)) {
            const float dither = (float(int(r & 0x1FFFu)) * (1.0f / 8192.0f) - 0.5f) * 5.9604644775390625e-08f;
            return static_cast<_Float16>(v + dither);
        }
        return static_cast<_Float16>(__uint_as_float((u + (r & 0x1FFFu)) & ~0x1FFFu));
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
