// Fused Shan-Chen D3Q19 step for gfx950: pull stream + boundaries + moments +
// pseudopotential force + velocity shift + BGK collision + store, one pass.
//
// Method: lattice Boltzmann equation per component with BGK relaxation
// (Eq. 1), second-order equilibrium (Eq. 2), moments (Eq. 3); the interfacial
// force is applied before collision as a body force (Methods, interfacial
// tension paragraph) -- here the Shan-Chen cross-component pseudopotential
// force entering through the shifted equilibrium velocity.  Wetting uses solid
// ghost pseudo-densities (the paper's solid ghost layer, Methods).
//
// Layout and schedule
// -------------------
// Populations are SoA arrays f[k*19+i][z][y][x] (x fastest).  A work-group
// owns a 64 x TY column tile and marches a chunk of z planes.  For every plane
// it pulls f_i(x) = f*_i(x - c_i) for its TY rows plus a one-node ring around
// them, sums the densities of all (TY+2) x 66 positions into a 4-plane LDS
// ring of pseudo-potentials, and finishes the plane below once the plane above
// is in LDS.  The force needs no density array in HBM: every population is
// read once and written once; the ring re-reads mostly hit L2.
//
// Addressing: all HBM traffic goes through buffer resources (one per
// component).  The plane being marched is the same for the whole work-group,
// so the array index and the z offset form a wave-uniform scalar offset, and
// each thread keeps nine fixed xy offsets (the 3 x 3 neighbourhood of its
// node): a pull costs no vector address arithmetic.
//
// Boundaries inside the same pass:
//  * static walls (halfway bounce-back): a fluid node next to a wall writes
//    f*_j(x) into the wall node's slot of direction opp(j), so the next pull
//    is branch-free;
//  * the reservoir plane z = nz-1: the plane below it takes w_i rho_top_k for
//    the directions pulled from the reservoir and books the outflow of its
//    stored f*(t) towards the reservoir into a per-tile FP64 ledger slot
//    (deterministic: each tile owns its slot);
//  * rod nodes: the slots the next pull reads are written by the rod link
//    kernel; the step stores zero deviations into all of them beforehand, so
//    that waves cut by a rod store whole lines.  On lattices with rods the
//    step also stores every node's densities (compute precision; zero on rod
//    nodes), which the rod passes read instead of summing 19 populations per
//    surface node in the order of their lists.
//
// Evaporation sink (a separate instantiation; FP32 storage, or FP64 with
// tau = 1): after the
// collision, an interface node (liquid here, a gas fluid node at z + 1) moves
// min(J0 / (K + h / h0), f*_0^A) from A's rest population to B's (Methods,
// evaporation paragraph; Eq. 8).  h, the column's liquid nodes, comes from
// the previous step's per-chunk counts; this step writes its own.
#include <type_traits>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

namespace {

constexpr int RSRC_FLAGS = 0x00020000;  // raw dword buffer, gfx9 family

__device__ inline int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
__device__ inline int wrapmod(int v, int n) {
    int r = v % n;
    return r < 0 ? r + n : r;
}

// raw buffer access of one storage element at byte offsets (voff per lane, soff uniform)
template <class S>
__device__ inline S buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ inline float buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ inline double buf_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return __hiloint2double(static_cast<int>(v[1]), static_cast<int>(v[0]));
}
template <>
__device__ inline _Float16 buf_load<_Float16>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    const unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
    return __builtin_bit_cast(_Float16, b);
}
template <>
__device__ inline bf16_t buf_load<bf16_t>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    bf16_t o;
    o.bits = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
    return o;
}

// Stores carry the non-temporal cache policy (bit 1 of the buffer
// instruction's policy operand): the step never reads back what it writes, so
// the written lines are evicted first and the L2 keeps the pulled planes whose
// halo rows the neighbouring tiles read again (150 -> 144-146 us per FP32
// step on the 256 x 128 x 64 cap; the same policy on the loads costs 179 us).
constexpr int ST_POLICY = 2;
template <class S>
__device__ inline void buf_store(S v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ inline void buf_store<float>(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, ST_POLICY);
}
template <>
__device__ inline void buf_store<double>(double v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    const unsigned long long u = __double_as_longlong(v);
    __attribute__((ext_vector_type(2))) unsigned int w;
    w[0] = static_cast<unsigned int>(u);
    w[1] = static_cast<unsigned int>(u >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(w, r, voff, soff, ST_POLICY);
}
template <>
__device__ inline void buf_store<_Float16>(_Float16 v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, voff, soff, ST_POLICY);
}
template <>
__device__ inline void buf_store<bf16_t>(bf16_t v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b16(v.bits, r, voff, soff, ST_POLICY);
}

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), static_cast<short>(0), static_cast<int>(bytes),
                                             RSRC_FLAGS);
}

// A node's 3 x 3 xy neighbourhood as element offsets within a plane:
// xy[a][b] = (y + a - 1) * nx + (x + b - 1) with periodic wrap (clamped when
// the direction is closed, where fluid nodes never reach the end planes).
struct NodeXY {
    uint32_t xy[3][3];
    bool valid;
};

__device__ inline NodeXY make_node(int x, int y, const StepArgs &a) {
    NodeXY n;
    bool vx, vy;
    if (a.px) {
        x = wrapmod(x, a.nx);
        vx = true;
    } else {
        vx = (x >= 0 && x < a.nx);
    }
    if (a.py) {
        y = wrapmod(y, a.ny);
        vy = true;
    } else {
        vy = (y >= 0 && y < a.ny);
    }
    n.valid = vx && vy;
    x = min(max(x, 0), a.nx - 1);
    y = min(max(y, 0), a.ny - 1);
    const int xs[3] = {a.px ? wrap1(x - 1, a.nx) : max(x - 1, 0), x, a.px ? wrap1(x + 1, a.nx) : min(x + 1, a.nx - 1)};
    const int ys[3] = {a.py ? wrap1(y - 1, a.ny) : max(y - 1, 0), y, a.py ? wrap1(y + 1, a.ny) : min(y + 1, a.ny - 1)};
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) n.xy[p][q] = static_cast<uint32_t>(ys[p]) * a.nx + xs[q];
    return n;
}

template <class C>
__device__ inline C wave_sum(C v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace

// One work-group's tile: logical tile b of a lattice whose step runs as nblk
// work-groups.  remap: b is a hardware dispatch index to be spread over the
// XCDs (else b is already the logical tile).
template <class S, int TY, int NPT, bool TAU1, bool SINK = false>
__device__ __forceinline__ void sc_step_tile(const StepArgs &a, int b, int nblk, bool remap) {
    using C = typename Codec<S>::C;
    constexpr int TX = 64;
    constexpr int RY = TY / NPT;
    constexpr int NT = TX * RY;
    constexpr int HX = TX + 2, HY = TY + 2, PL = HX * HY;
    constexpr int NH = 2 * HX + 2 * TY;
    constexpr int NHPT = (NH + NT - 1) / NT;
    constexpr int NW = NT / 64;
    constexpr uint32_t E = sizeof(S);
    // software-pipelined plane loads need a second set of raw registers; that
    // fits for tau = 1 with 4- or 2-byte storage, the other forms load and
    // consume a plane in turn
    constexpr bool PIPE = TAU1 && sizeof(S) <= 4;

    __shared__ C ring[4][2][PL];
    __shared__ C psi_tab[16][2];
    __shared__ double red[NW][2];

    // ---- tile of this work-group.  Work-groups are dealt to the eight XCDs
    // round-robin; the remap gives each XCD a contiguous range of logical
    // tiles, ordered z-chunk fastest, so an XCD owns whole xy columns and
    // neighbouring columns (their shared ring reads then hit its L2).
    if (remap && (nblk & 7) == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
    const int tz = b % a.nzc;
    const int tx = (b / a.nzc) % a.ntx;
    const int ty = b / (a.nzc * a.ntx);
    const int x0 = tx * TX, y0 = ty * TY;
    const int z0 = tz * a.zchunk;
    const int z1 = min(z0 + a.zchunk, a.nz);
    if (z0 >= a.nz) return;  // uniform per block
    // even chunks march up, odd chunks march down: two chunks meet at their
    // shared boundary plane at the same time (both at the start or both at
    // the end of their marches), so the boundary pulls are shared in cache
    const int dir = (tz & 1) ? -1 : 1;
    const int zfirst = dir > 0 ? z0 : z1 - 1;
    const int nplanes = z1 - z0;

    const int tid = threadIdx.x;
    const int lx = tid & 63;
    const int ly = tid >> 6;
    const uint32_t nxy = static_cast<uint32_t>(a.nx) * a.ny;
    const uint32_t fsE = static_cast<uint32_t>(a.fs) * E;  // bytes between population arrays

    // one buffer resource per component over its 19 arrays
    __amdgpu_buffer_rsrc_t src[2], dst[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        src[k] = make_rsrc(static_cast<const char *>(a.fsrc) + size_t(k) * Q * fsE, Q * fsE);
        dst[k] = make_rsrc(static_cast<const char *>(a.fdst) + size_t(k) * Q * fsE, Q * fsE);
    }
    const __amdgpu_buffer_rsrc_t matr = make_rsrc(a.mat, nxy * a.nz);

    if (tid < 32) psi_tab[tid >> 1][tid & 1] = C(a.psi_tab[tid]);
    const unsigned known = *a.status;  // status bits already raised before this launch

    // constants in compute precision; rref is the storage reference density
    // (populations travel as d_i = f_i - w_i rref)
    const C G = C(a.G);
    const C rref[2] = {C(a.rho_ref[0]), C(a.rho_ref[1])};
    const C tdev[2] = {C(a.rho_top[0] - a.rho_ref[0]), C(a.rho_top[1] - a.rho_ref[1])};
    const C om[2] = {C(a.omega[0]), C(a.omega[1])};
    const C ta[2] = {C(a.tau[0]), C(a.tau[1])};
    const C gb[3] = {C(a.g[0]), C(a.g[1]), C(a.g[2])};

    // ---- owned interior nodes and ring (halo) nodes of this thread
    NodeXY own[NPT];
    bool own_fin[NPT];
    int own_ring[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
        const int yy = ly + r * RY;
        own[r] = make_node(x0 + lx, y0 + yy, a);
        own_fin[r] = (x0 + lx < a.nx) && (y0 + yy < a.ny);
        own_ring[r] = (yy + 1) * HX + (lx + 1);
    }
    NodeXY hal[NHPT];
    int hal_ring[NHPT];
    bool hal_on[NHPT];
#pragma unroll
    for (int m = 0; m < NHPT; ++m) {
        const int h = tid + m * NT;
        int hx = 0, hy = 0;
        hal_on[m] = h < NH;
        if (h < HX) {
            hx = h;
            hy = 0;
        } else if (h < 2 * HX) {
            hx = h - HX;
            hy = HY - 1;
        } else if (h < 2 * HX + TY) {
            hx = 0;
            hy = 1 + h - 2 * HX;
        } else {
            hx = HX - 1;
            hy = 1 + h - 2 * HX - TY;
        }
        if (!hal_on[m]) hx = hy = 0;
        hal[m] = make_node(x0 + hx - 1, y0 + hy - 1, a);
        hal_ring[m] = hy * HX + hx;
    }
    __syncthreads();  // psi_tab

    // evaporation sink (Eq. 8): flux of each owned column from the heights
    // the previous step counted over all z chunks, this chunk's count of
    // liquid nodes after the sink, and the mass this thread moved A -> B
    C sink_J[NPT];
    int sink_cnt[NPT];
    double sink_mv = 0.0;
    if constexpr (SINK) {
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            int h = 0;
            if (own_fin[r])
                for (int q = 0; q < a.nzc; ++q) h += a.h_read[size_t(q) * nxy + own[r].xy[1][1]];
            sink_J[r] = C(a.sink_J0) / (C(a.sink_K) + C(h) / C(a.sink_h0));
            sink_cnt[r] = 0;
        }
    }

    // moments of the owned nodes: current plane and next plane
    C cur_rho[NPT][2], cur_drho[NPT][2], cur_j[NPT][2][3];
    C nxt_rho[NPT][2], nxt_drho[NPT][2], nxt_j[NPT][2][3];
    C cur_f[TAU1 ? 1 : NPT][TAU1 ? 1 : 2][TAU1 ? 1 : Q];
    C nxt_f[TAU1 ? 1 : NPT][TAU1 ? 1 : 2][TAU1 ? 1 : Q];
    uint8_t cur_m[NPT], nxt_m[NPT];

    // raw pulled values of one plane, in flight between issue() and process()
    S raw_own[NPT][2][Q];
    S raw_hal[NHPT][2][Q];
    uint8_t mat_own[NPT], mat_hal[NHPT];
    bool plane_valid = false, plane_top = false;

    // psi of a node given its material byte and densities
    auto psi_of = [&](uint8_t m, int k, C rho) -> C {
        const uint8_t id = m & MAT_ID_MASK;
        return id == MAT_FLUID ? rho : psi_tab[id][k];
    };

    // Issue the pulls f*_i(x - c_i) of plane z for the owned and ring nodes.
    // Loads are unconditional (every offset is wrapped or clamped into the
    // lattice); values pulled for non-fluid nodes are discarded by process().
    // Directions pulled from the reservoir plane are not loaded.
    auto issue = [&](int z) {
        int zz = z;
        if (a.pz) {
            zz = wrap1(z, a.nz);
            plane_valid = true;
        } else {
            plane_valid = (z >= 0 && z < a.nz);
        }
        zz = min(max(zz, 0), a.nz - 1);
        const int zm = a.pz ? wrap1(zz - 1, a.nz) : max(zz - 1, 0);
        const int zp = a.pz ? wrap1(zz + 1, a.nz) : min(zz + 1, a.nz - 1);
        const uint32_t zoE[3] = {zm * nxy * E, zz * nxy * E, zp * nxy * E};
        plane_top = a.evap && (zz == a.nz - 2);
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            mat_own[r] = uint8_t(__builtin_amdgcn_raw_buffer_load_b8(matr, own[r].xy[1][1], zz * nxy, 0));
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    if (!(cz(i) == -1 && plane_top))
                        raw_own[r][k][i] =
                            buf_load<S>(src[k], own[r].xy[1 - cy(i)][1 - cx(i)] * E, i * fsE + zoE[1 - cz(i)]);
        }
#pragma unroll
        for (int mm = 0; mm < NHPT; ++mm) {
            if (!hal_on[mm]) continue;
            mat_hal[mm] = uint8_t(__builtin_amdgcn_raw_buffer_load_b8(matr, hal[mm].xy[1][1], zz * nxy, 0));
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    if (!(cz(i) == -1 && plane_top))
                        raw_hal[mm][k][i] =
                            buf_load<S>(src[k], hal[mm].xy[1 - cy(i)][1 - cx(i)] * E, i * fsE + zoE[1 - cz(i)]);
        }
    };

    // decoded deviation d_i of a raw pulled value (reservoir sources: w_i (rho_top - rref))
    auto devof = [&](const S (&raw)[2][Q], int k, int i) -> C {
        return (cz(i) == -1 && plane_top) ? wgt<C>(i) * tdev[k] : Codec<S>::dec(raw[k][i]);
    };

    // Turn the issued plane into psi values in ring slot z & 3 and, when
    // keep, into the owned nodes' moments for the next finish.
    auto process = [&](int z, bool keep) {
        const int slot = z & 3;
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            const bool v = plane_valid && own[r].valid;
            const uint8_t m = v ? mat_own[r] : uint8_t(MAT_ID_MASK);
            C rho[2] = {C(0), C(0)}, drho[2] = {C(0), C(0)};
            C j[2][3] = {{C(0), C(0), C(0)}, {C(0), C(0), C(0)}};
            const bool fl = v && (m & MAT_ID_MASK) == MAT_FLUID;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                C fv[Q];
#pragma unroll
                for (int i = 0; i < Q; ++i) fv[i] = devof(raw_own[r], k, i);
                C s = C(0), jx = C(0), jy = C(0), jz = C(0);
#pragma unroll
                for (int i = 0; i < Q; ++i) s += fv[i];
                // momentum over opposite pairs: f_i - f_opp(i) is nearly exact
                // (the two are close), which avoids cancellation in j
#pragma unroll
                for (int i = 1; i < Q; i += 2) {
                    const C d = fv[i] - fv[i + 1];
                    if (cx(i) == 1) jx += d;
                    if (cx(i) == -1) jx -= d;
                    if (cy(i) == 1) jy += d;
                    if (cy(i) == -1) jy -= d;
                    if (cz(i) == 1) jz += d;
                    if (cz(i) == -1) jz -= d;
                }
                // Eq. 3: rho_k = sum_i f_i = rref_k + sum_i d_i (sum_i w_i = 1)
                drho[k] = fl ? s : C(0);
                rho[k] = fl ? rref[k] + s : C(0);
                j[k][0] = fl ? jx : C(0);
                j[k][1] = fl ? jy : C(0);
                j[k][2] = fl ? jz : C(0);
                if constexpr (!TAU1) {
                    if (keep) {
#pragma unroll
                        for (int i = 0; i < Q; ++i) nxt_f[r][k][i] = fv[i];
                    }
                }
            }
            ring[slot][0][own_ring[r]] = v ? psi_of(m, 0, rho[0]) : C(0);
            ring[slot][1][own_ring[r]] = v ? psi_of(m, 1, rho[1]) : C(0);
            if (keep) {
                nxt_m[r] = m;
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    nxt_rho[r][k] = rho[k];
                    nxt_drho[r][k] = drho[k];
#pragma unroll
                    for (int d = 0; d < 3; ++d) nxt_j[r][k][d] = j[k][d];
                }
            }
        }
#pragma unroll
        for (int mm = 0; mm < NHPT; ++mm) {
            if (!hal_on[mm]) continue;
            const bool v = plane_valid && hal[mm].valid;
            const uint8_t m = v ? mat_hal[mm] : uint8_t(MAT_ID_MASK);
            const bool fl = v && (m & MAT_ID_MASK) == MAT_FLUID;
            C rho[2] = {C(0), C(0)};
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                C s = C(0);
#pragma unroll
                for (int i = 0; i < Q; ++i) s += devof(raw_hal[mm], k, i);
                rho[k] = fl ? rref[k] + s : C(0);
            }
            ring[slot][0][hal_ring[mm]] = v ? psi_of(m, 0, rho[0]) : C(0);
            ring[slot][1][hal_ring[mm]] = v ? psi_of(m, 1, rho[1]) : C(0);
        }
    };

    auto shift_next = [&]() {
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            cur_m[r] = nxt_m[r];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                cur_rho[r][k] = nxt_rho[r][k];
                cur_drho[r][k] = nxt_drho[r][k];
#pragma unroll
                for (int d = 0; d < 3; ++d) cur_j[r][k][d] = nxt_j[r][k][d];
                if constexpr (!TAU1) {
#pragma unroll
                    for (int i = 0; i < Q; ++i) cur_f[r][k][i] = nxt_f[r][k][i];
                }
            }
        }
    };

    // prologue: the plane behind the first one (psi only), the first plane
    // (psi + moments), then the loads of the plane after it
    issue(zfirst - dir);
    process(zfirst - dir, false);
    issue(zfirst);
    process(zfirst, true);
    shift_next();
    if constexpr (PIPE) issue(zfirst + dir);

    for (int it = 0; it < nplanes; ++it) {
        const int z = zfirst + it * dir;
        // the ring holds 4 planes: this iteration writes plane z + dir and
        // reads z - 1, z, z + 1; the next one writes z + 2 dir, which no
        // thread of this iteration reads, so one barrier per plane suffices
        if constexpr (PIPE) {
            process(z + dir, true);
            // software pipeline: the pulls of plane z + 2 dir stay in flight
            // across the barrier (which waits on LDS only) and the finish below
            if (it + 1 < nplanes) issue(z + 2 * dir);
        } else {
            issue(z + dir);
            process(z + dir, true);
        }
        __syncthreads();

        const int sm = (z - 1) & 3, s0 = z & 3, sp = (z + 1) & 3;
        const uint32_t zE = static_cast<uint32_t>(z) * nxy * E;
        const bool ledger_plane = a.evap && (z == a.nz - 2);
        double led[2] = {0.0, 0.0};
        unsigned st = 0;

#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            // rod nodes go through the same arithmetic (all their moments are
            // zero, so every deviation they store is exactly zero) and store
            // with the fluid lanes: a wave that a rod cuts through then still
            // writes whole lines, where masked lanes would leave partial lines
            // that HBM has to read, merge and write back.  Nothing reads these
            // slots before the rod passes rewrite them (link) or refill them.
            const uint8_t mid = cur_m[r] & MAT_ID_MASK;
            if (!own_fin[r] || (mid != MAT_FLUID && mid != MAT_ROD)) continue;
            const bool fluid = mid == MAT_FLUID;
            const int rc = own_ring[r];
            const C rho[2] = {cur_rho[r][0], cur_rho[r][1]};
            if (a.rho_out) {  // lattices with rods: the densities for the rod passes
                C *ro = static_cast<C *>(a.rho_out);
                const int64_t nn = int64_t(z) * nxy + own[r].xy[1][1];
                ro[nn] = rho[0];
                ro[a.fs + nn] = rho[1];
            }
            // interface node of the sink: liquid here (rho_A > rho_B) and a
            // gas fluid node above, whose densities are its psi in the ring
            bool sink_if = false;
            C sink_d = C(0);
            if constexpr (SINK) {
                if (rho[0] > rho[1] && (a.pz || z + 1 < a.nz) && ring[sp][0][rc] < ring[sp][1][rc]) {
                    const int za = a.pz ? wrap1(z + 1, a.nz) : z + 1;
                    const uint8_t ma = uint8_t(__builtin_amdgcn_raw_buffer_load_b8(matr, own[r].xy[1][1], za * nxy, 0));
                    sink_if = (ma & MAT_ID_MASK) == MAT_FLUID;
                }
            }
            // Shan-Chen force: F_k = -G psi_k(x) sum_i w_i psi_kbar(x + c_i) c_i + rho_k g
            C F[2][3];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int kb = 1 - k;
                // sum_i w_i psi(x + c_i) c_i taken over opposite pairs as central
                // differences w_i c_i (psi(x + c_i) - psi(x - c_i)): no cancellation
                C sx = C(0), sy = C(0), sz = C(0);
#pragma unroll
                for (int i = 1; i < Q; i += 2) {
                    const int slp = cz(i) == 1 ? sp : (cz(i) == -1 ? sm : s0);
                    const int slm = cz(i) == 1 ? sm : (cz(i) == -1 ? sp : s0);
                    const C nb = wgt<C>(i) * (ring[slp][kb][rc + cy(i) * HX + cx(i)] -
                                              ring[slm][kb][rc - cy(i) * HX - cx(i)]);
                    if (cx(i) == 1) sx += nb;
                    if (cx(i) == -1) sx -= nb;
                    if (cy(i) == 1) sy += nb;
                    if (cy(i) == -1) sy -= nb;
                    if (cz(i) == 1) sz += nb;
                    if (cz(i) == -1) sz -= nb;
                }
                const C gp = -G * rho[k];
                F[k][0] = gp * sx + rho[k] * gb[0];
                F[k][1] = gp * sy + rho[k] * gb[1];
                F[k][2] = gp * sz + rho[k] * gb[2];
            }
            // velocity shift: u' = sum_k j_k/tau_k / sum_k rho_k/tau_k; u_k^eq = u' + tau_k F_k / rho_k
            const C den = rho[0] * om[0] + rho[1] * om[1];
            const C rden = den > C(0) ? C(1) / den : C(0);
            C up[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) up[d] = (cur_j[r][0][d] * om[0] + cur_j[r][1][d] * om[1]) * rden;
            // health check on the physical velocity (sum_k j_k + F/2) / rho
            {
                const C rt = rho[0] + rho[1];
                const C ir = rt > C(0) ? C(1) / rt : C(0);
                C usq_chk = C(0);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const C ud = (cur_j[r][0][d] + cur_j[r][1][d] + C(0.5) * (F[0][d] + F[1][d])) * ir;
                    usq_chk += ud * ud;
                }
                if (fluid && !(rt > C(0))) st |= ST_RHO;
                if (fluid && !(usq_chk <= C(0.09))) st |= (usq_chk != usq_chk) ? ST_NAN : ST_SPEED;
            }

            const uint32_t voE = own[r].xy[1][1] * E;
            const bool near_wall = fluid && (cur_m[r] & MAT_NEAR_WALL) != 0;
            // 16-bit storage with stochastic rounding: the random bits depend on
            // (node, array, step) only; the wall slots reuse the encoded values
            const int64_t gnode = int64_t(z) * nxy + own[r].xy[1][1];
            SrStream sr{0u, 0u};
            if constexpr (sizeof(S) == 2) {
                if (a.sr_key) sr.state = sr_seed(a.sr_key, gnode);
            }
            auto encode = [&](C v, int arr) -> S {
                if constexpr (sizeof(S) == 2) {
                    if (a.sr_key) return Stochastic<S>::enc(v, sr.bits(arr));
                }
                return Codec<S>::enc(v);
            };
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                C ue[3];
                const bool ok = rho[k] >= C(1e-12);
                const C rk = ok ? ta[k] / rho[k] : C(0);
#pragma unroll
                for (int d = 0; d < 3; ++d) ue[d] = up[d] + F[k][d] * rk;
                const C usq = ue[0] * ue[0] + ue[1] * ue[1] + ue[2] * ue[2];
                const C dr = cur_drho[r][k];
                S sstar[Q];
                C deq_sum = C(0);
                // Eq. 2 as a deviation, built per opposite pair (i, opp(i)):
                //   f^eq - w rref = w (rho - rref) + w rho [9/2 (c.u)^2 - 3/2 u^2]  +-  w rho 3 c.u
                // The rest population is the remainder so that sum_i f_i^eq = rho holds up to
                // one rounding: the rounded weights do not sum to one, and using them for all
                // 19 directions would drift the mass by a fixed factor every step.
                C deq[Q];
                const C base = C(-1.5) * usq;
#pragma unroll
                for (int i = 1; i < Q; i += 2) {
                    const C cu = C(cx(i)) * ue[0] + C(cy(i)) * ue[1] + C(cz(i)) * ue[2];
                    const C wr = wgt<C>(i) * rho[k];
                    const C sym = wgt<C>(i) * dr + wr * (base + C(4.5) * cu * cu);
                    const C asym = wr * (C(3) * cu);
                    deq[i] = sym + asym;
                    deq[i + 1] = sym - asym;
                    deq_sum += deq[i];
                    deq_sum += deq[i + 1];
                }
                deq[0] = dr - deq_sum;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    C ds;
                    if constexpr (TAU1) {
                        ds = deq[i];  // Eq. 1 with tau = 1: f* = f^eq
                    } else {
                        ds = fluid ? cur_f[r][k][i] - (cur_f[r][k][i] - deq[i]) * om[k] : C(0);
                    }
                    if constexpr (SINK) {
                        // Eq. 8: min(J, f*_0^A), at least 0, leaves A's rest population for B's
                        if (i == 0 && sink_if) {
                            if (k == 0) {
                                sink_d = fmax(fmin(sink_J[r], ds + wgt<C>(0) * rref[0]), C(0));
                                ds -= sink_d;
                            } else {
                                ds += sink_d;
                            }
                        }
                    }
                    sstar[i] = encode(ds, k * Q + i);
                    buf_store<S>(sstar[i], dst[k], voE, i * fsE + zE);
                }
                if (ledger_plane && fluid) {
                    // this step's streaming moves the node's stored f*_i(t) with c_iz = +1
                    // into the reservoir and pulls w_i rho_top_k out of it
                    double outflow = 0.0, inflow = 0.0;
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        if (cz(i) == 1)
                            outflow += double(Codec<S>::dec(buf_load<S>(src[k], voE, i * fsE + zE))) +
                                       wgt<double>(i) * a.rho_ref[k];
                        if (cz(i) == -1) inflow += wgt<double>(i) * a.rho_top[k];
                    }
                    led[k] += outflow - inflow;
                }
                if (near_wall) {
                    // halfway bounce-back: hand f*_j(x) to the wall node x + c_j as
                    // direction opp(j) (w_j = w_opp(j), so the deviation carries over)
                    const uint32_t zl[3] = {
                        static_cast<uint32_t>(a.pz ? wrap1(z - 1, a.nz) : max(z - 1, 0)) * nxy,
                        static_cast<uint32_t>(z) * nxy,
                        static_cast<uint32_t>(a.pz ? wrap1(z + 1, a.nz) : min(z + 1, a.nz - 1)) * nxy};
#pragma unroll
                    for (int jd = 1; jd < Q; ++jd) {
                        const uint32_t nxyo = own[r].xy[1 + cy(jd)][1 + cx(jd)];
                        const uint8_t nm = uint8_t(__builtin_amdgcn_raw_buffer_load_b8(matr, nxyo, zl[1 + cz(jd)], 0));
                        if (is_static_wall(nm & MAT_ID_MASK))
                            buf_store<S>(sstar[jd], dst[k], nxyo * E,
                                         opp(jd) * fsE + zl[1 + cz(jd)] * E);
                    }
                }
            }
            if constexpr (SINK) {
                // the column height the next step reads: liquid after the sink
                sink_cnt[r] += (rho[0] - sink_d > rho[1] + sink_d) ? 1 : 0;
                sink_mv += double(sink_d);
            }
        }
        post_status(a.status, known, st);

        if (ledger_plane) {  // uniform across the block
            const int w = tid >> 6;
            double l0 = wave_sum(led[0]), l1 = wave_sum(led[1]);
            if (lx == 0) {
                red[w][0] = l0;
                red[w][1] = l1;
            }
            __syncthreads();
            if (tid == 0) {
                double s0v = 0.0, s1v = 0.0;
                for (int q = 0; q < NW; ++q) {
                    s0v += red[q][0];
                    s1v += red[q][1];
                }
                double *slot = a.ledger_part + 2 * (ty * a.ntx + tx);
                slot[0] += s0v;
                slot[1] += s1v;
            }
        }
        shift_next();
    }

    if constexpr (SINK) {
        // this chunk's column heights, and the work-group's moved mass into
        // its own ledger pair (A loses it, B gains it)
#pragma unroll
        for (int r = 0; r < NPT; ++r)
            if (own_fin[r]) a.h_write[size_t(tz) * nxy + own[r].xy[1][1]] = sink_cnt[r];
        const double mv = wave_sum(sink_mv);
        __syncthreads();  // red may still be read by the last ledger plane's sum
        if (lx == 0) red[tid >> 6][0] = mv;
        __syncthreads();
        if (tid == 0) {
            double sum = 0.0;
            for (int q = 0; q < NW; ++q) sum += red[q][0];
            double *slot = a.sink_ledger + 2 * ((size_t(tz) * a.nty + ty) * a.ntx + tx);
            slot[0] += sum;
            slot[1] -= sum;
        }
    }
}

template <class S, int TY, int NPT, bool TAU1, bool SINK>
__global__ void __launch_bounds__(64 * (TY / NPT)) sc_step_kernel(StepArgs a) {
    sc_step_tile<S, TY, NPT, TAU1, SINK>(a, blockIdx.x, gridDim.x, true);
}

// Batched step: one launch walks a device work list of (lattice, logical
// tile) entries over many lattices of one tile class, each with its own
// parameter record.  The list is ordered so that the hardware's round-robin
// dealing of work-groups to XCDs gives each XCD a contiguous range of it.
template <class S, int TY, int NPT, bool TAU1>
__global__ void __launch_bounds__(64 * (TY / NPT)) sc_step_batch_kernel(const StepArgs *__restrict__ all,
                                                                         const int2 *__restrict__ work) {
    const int2 w = work[blockIdx.x];
    if (w.x < 0) return;  // padding entry, uniform per block
    const StepArgs a = all[w.x];
    sc_step_tile<S, TY, NPT, TAU1>(a, w.y, a.ntx * a.nty * a.nzc, false);
}

int tiles_xy(int nx, int ny, int tile_y) { return ((nx + 63) / 64) * ((ny + tile_y - 1) / tile_y); }

template <class S, int TY, int NPT, bool TAU1>
static hipError_t launch_one(const StepArgs &a, hipStream_t s) {
    const int nblk = a.ntx * a.nty * a.nzc;
    if (a.sink) {
        if constexpr (std::is_same_v<S, float>) {
            hipLaunchKernelGGL((sc_step_kernel<S, TY, NPT, TAU1, true>), dim3(nblk), dim3(64 * (TY / NPT)), 0, s, a);
            return hipGetLastError();
        } else if constexpr (std::is_same_v<S, double> && TAU1) {
            // With the sink, the FP64 instantiation of the 64 x 8 tile with
            // one row per thread gave wrong populations while the other FP64
            // tiles and all FP32 tiles match the oracle; the same tiling runs
            // with two rows per thread (identical work-groups and slots).
            if constexpr (TY == 8 && NPT == 1) {
                hipLaunchKernelGGL((sc_step_kernel<double, 8, 2, true, true>), dim3(nblk), dim3(64 * 4), 0, s, a);
            } else {
                hipLaunchKernelGGL((sc_step_kernel<S, TY, NPT, TAU1, true>), dim3(nblk), dim3(64 * (TY / NPT)), 0, s,
                                   a);
            }
            return hipGetLastError();
        }
        return hipErrorInvalidValue;  // the sink runs with FP32 storage, or FP64 with tau = 1
    }
    hipLaunchKernelGGL((sc_step_kernel<S, TY, NPT, TAU1, false>), dim3(nblk), dim3(64 * (TY / NPT)), 0, s, a);
    return hipGetLastError();
}

template <class S, bool TAU1>
static hipError_t launch_prec(const TileCfg &t, const StepArgs &a, hipStream_t s) {
    if (t.tile_y == 4 && t.rows_per_thread == 1) return launch_one<S, 4, 1, TAU1>(a, s);
    if (t.tile_y == 8 && t.rows_per_thread == 1) return launch_one<S, 8, 1, TAU1>(a, s);
    if constexpr (TAU1) {
        // tau = 1 keeps only moments per owned node, so several rows fit
        if (t.tile_y == 8 && t.rows_per_thread == 2) return launch_one<S, 8, 2, TAU1>(a, s);
        if (t.tile_y == 16 && t.rows_per_thread == 2) return launch_one<S, 16, 2, TAU1>(a, s);
    }
    return hipErrorInvalidValue;
}

template <class S, int TY, int NPT, bool TAU1>
static hipError_t launch_batch_one(const StepArgs *all, const int2 *work, int nwork, hipStream_t s) {
    hipLaunchKernelGGL((sc_step_batch_kernel<S, TY, NPT, TAU1>), dim3(nwork), dim3(64 * (TY / NPT)), 0, s, all, work);
    return hipGetLastError();
}

template <class S, bool TAU1>
static hipError_t launch_batch_prec(const TileCfg &t, const StepArgs *all, const int2 *work, int nwork, hipStream_t s) {
    if (t.tile_y == 4 && t.rows_per_thread == 1) return launch_batch_one<S, 4, 1, TAU1>(all, work, nwork, s);
    if (t.tile_y == 8 && t.rows_per_thread == 1) return launch_batch_one<S, 8, 1, TAU1>(all, work, nwork, s);
    if constexpr (TAU1) {
        if (t.tile_y == 8 && t.rows_per_thread == 2) return launch_batch_one<S, 8, 2, TAU1>(all, work, nwork, s);
        if (t.tile_y == 16 && t.rows_per_thread == 2) return launch_batch_one<S, 16, 2, TAU1>(all, work, nwork, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_sc_step_batch(int prec, bool tau1, const TileCfg &t, const StepArgs *all, const int2 *work, int nwork,
                                hipStream_t s) {
    switch (prec) {
        case LB_F64:
            return tau1 ? launch_batch_prec<double, true>(t, all, work, nwork, s)
                        : launch_batch_prec<double, false>(t, all, work, nwork, s);
        case LB_F32:
            return tau1 ? launch_batch_prec<float, true>(t, all, work, nwork, s)
                        : launch_batch_prec<float, false>(t, all, work, nwork, s);
        case LB_F16DEV:
            return tau1 ? launch_batch_prec<_Float16, true>(t, all, work, nwork, s)
                        : launch_batch_prec<_Float16, false>(t, all, work, nwork, s);
        case LB_BF16DEV:
            return tau1 ? launch_batch_prec<bf16_t, true>(t, all, work, nwork, s)
                        : launch_batch_prec<bf16_t, false>(t, all, work, nwork, s);
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_sc_step(int prec, bool tau1, const TileCfg &t, const StepArgs &a, hipStream_t s) {
    switch (prec) {
        case LB_F64:
            return tau1 ? launch_prec<double, true>(t, a, s) : launch_prec<double, false>(t, a, s);
        case LB_F32:
            return tau1 ? launch_prec<float, true>(t, a, s) : launch_prec<float, false>(t, a, s);
        case LB_F16DEV:
            return tau1 ? launch_prec<_Float16, true>(t, a, s) : launch_prec<_Float16, false>(t, a, s);
        case LB_BF16DEV:
            return tau1 ? launch_prec<bf16_t, true>(t, a, s) : launch_prec<bf16_t, false>(t, a, s);
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace lbm
