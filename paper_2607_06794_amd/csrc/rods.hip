// Rigid capsule rods coupled to the Shan-Chen fluid (gfx950).
//
// The paper's nanowires are bead-spring filaments moved with five particle
// substeps per lattice Boltzmann step (Methods, filament paragraph; Eqs. 9-12).
// Here they are rigid capsules (the stiff limit) coupled by moving
// bounce-back on every boundary link:
//   f_i(x, t+1) = f*_opp(i)(x, t) + 2 w_i rho_k(x) (c_i . u_b) / c_s^2,
//   u_b = V + Omega x (x_b - X) at the link midpoint x_b = x - c_i / 2,
// the rod receiving dP = -c_i (f*_opp(i)(x) + f_i(x, t+1)) per link, plus the
// reaction to the adhesion force of its ghost pseudo-densities.  Rod-rod
// excluded volume (Eq. 10) and shifted cohesion (Eq. 12) act between the
// closest points of the axis segments; a WCA wall keeps rods off the
// substrate.  All rod arithmetic is FP64.
//
// Work decomposition: the re-mask builds, per rod, the list of lattice nodes
// near its surface; every per-node pass runs one thread per listed node, and
// every sum is a fixed-order block or wavefront reduction, so results do not
// depend on scheduling.  Pair forces use a per-step neighbour list; the
// integrator is one work-group with one thread per rod.
#include <type_traits>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

namespace {

struct d3 {
    double x, y, z;
};
__device__ inline d3 mk(double x, double y, double z) { return {x, y, z}; }
__device__ inline d3 operator+(d3 a, d3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline d3 operator-(d3 a, d3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline d3 operator*(double s, d3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline d3 cross(d3 a, d3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

__device__ inline d3 ld3(const double *p) { return {p[0], p[1], p[2]}; }
// the same from device memory (rod records), as global loads
__device__ inline d3 gld3(const double *p) {
    const auto *g = gptr(p);
    return {g[0], g[1], g[2]};
}
__device__ inline void st3(double *p, d3 v) {
    p[0] = v.x;
    p[1] = v.y;
    p[2] = v.z;
}

// e = R(q) e_z for q = (w, x, y, z)
__device__ inline d3 quat_axis(const double *q) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    return {2.0 * (x * z + w * y), 2.0 * (y * z - w * x), 1.0 - 2.0 * (x * x + y * y)};
}

__device__ inline double min_img(double d, double box, int per) { return per ? d - box * rint(d / box) : d; }
__device__ inline d3 min_image(d3 d, const RodArgs &a) {
    return {min_img(d.x, a.nx, a.px), min_img(d.y, a.ny, a.py), min_img(d.z, a.nz, a.pz)};
}

__device__ inline d3 omega_of(const double *rod, const RodArgs &a) {
    const d3 L = ld3(rod + ROD_L);
    const d3 e = quat_axis(rod + ROD_Q);
    return (1.0 / a.Iperp) * L + ((1.0 / a.Ipar - 1.0 / a.Iperp) * dot(L, e)) * e;
}

__device__ inline d3 velocity_at(const double *rod, d3 x, const RodArgs &a) {
    const d3 d = min_image(x - ld3(rod + ROD_X), a);
    return ld3(rod + ROD_V) + cross(omega_of(rod, a), d);
}

// phi(d) = (d0/d)^12 - 2 (d0/d)^6 and its derivative
__device__ inline double ljf(double d, double d0) {
    const double x = d0 / d, x6 = x * x * x * x * x * x;
    return x6 * x6 - 2.0 * x6;
}
__device__ inline double ljf_d(double d, double d0) {
    const double x = d0 / d, x6 = x * x * x * x * x * x;
    return (-12.0 * x6 * x6 + 12.0 * x6) / d;
}

// -dU/dd of the rod-rod potential (excluded volume + shifted cohesion)
// divided by d, for d > 0; one potential shape, its strength chosen by the
// range d falls in, one reciprocal of d
__device__ inline double pair_force_over_d(double d, const RodArgs &a) {
    const double eps = d <= a.d0 ? a.eps_rep : ((a.eps_att > 0.0 && d < a.r_cut) ? a.eps_att : 0.0);
    const double id = 1.0 / d, x = a.d0 * id, x6 = x * x * x * x * x * x;
    return eps != 0.0 ? -(eps * ((-12.0 * x6 * x6 + 12.0 * x6) * id)) * id : 0.0;
}

// closest points of segments [p1, q1], [p2, q2]: stationary point of the
// squared distance if interior, else the best of the four clamped edges
__device__ inline double seg_seg(d3 p1, d3 q1, d3 p2, d3 q2, d3 &c1, d3 &c2) {
    const d3 d1 = q1 - p1, d2 = q2 - p2, r = p1 - p2;
    const double aa = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r), c = dot(d1, r), b = dot(d1, d2);
    double best = 1e300;  // squared distance of the best candidate so far
    auto tryst = [&](double s, double t) {
        const d3 x1 = p1 + s * d1, x2 = p2 + t * d2;
        const d3 dd = x1 - x2;
        const double v = dot(dd, dd);
        if (v < best) {
            best = v;
            c1 = x1;
            c2 = x2;
        }
    };
    // one reciprocal per denominator (FP64 division is a long sequence)
    const double den = aa * e - b * b;
    if (den > 1e-14 * fmax(aa * e, 1e-300)) {
        const double iden = 1.0 / den;
        const double s = (b * f - c * e) * iden, t = (aa * f - b * c) * iden;
        if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0) tryst(s, t);
    }
    const double ie = e == 0.0 ? 0.0 : 1.0 / e, ia = aa == 0.0 ? 0.0 : 1.0 / aa;
    for (int k = 0; k < 2; ++k) {
        const double s = k;
        const double t = e == 0.0 ? 0.0 : fmin(fmax((b * s + f) * ie, 0.0), 1.0);
        tryst(s, t);
    }
    for (int k = 0; k < 2; ++k) {
        const double t = k;
        const double s = aa == 0.0 ? 0.0 : fmin(fmax((b * t - c) * ia, 0.0), 1.0);
        tryst(s, t);
    }
    return sqrt(best);
}

template <class S>
__device__ inline double decf(const S *f, int64_t idx) {
    return static_cast<double>(Codec<S>::dec(gload(f + idx)));
}

// integer bounding box of the capsule (plus margin) in lattice coordinates
struct Box {
    int lo[3], hi[3];
};
__device__ inline Box rod_box(const double *rod, const RodArgs &a, int margin) {
    const d3 X = ld3(rod + ROD_X);
    const d3 e = quat_axis(rod + ROD_Q);
    const double ext[3] = {a.half * fabs(e.x) + a.radius, a.half * fabs(e.y) + a.radius, a.half * fabs(e.z) + a.radius};
    const double c[3] = {X.x, X.y, X.z};
    const int n[3] = {a.nx, a.ny, a.nz}, per[3] = {a.px, a.py, a.pz};
    Box b;
    for (int d = 0; d < 3; ++d) {
        // clamp in floating point first: a rod state gone bad (huge or NaN
        // coordinates) must still give a small, bounded box
        const double lo = fmin(fmax(floor(c[d] - ext[d]), -4.0 * n[d]), 4.0 * n[d]);
        const double hi = fmin(fmax(ceil(c[d] + ext[d]), -4.0 * n[d]), 4.0 * n[d]);
        b.lo[d] = static_cast<int>(lo) - margin;
        b.hi[d] = static_cast<int>(hi) + margin;
        if (per[d]) {
            // never visit a node twice through the periodic wrap
            if (b.hi[d] - b.lo[d] + 1 > n[d]) b.hi[d] = b.lo[d] + n[d] - 1;
        } else {
            b.lo[d] = max(b.lo[d], -margin);
            b.hi[d] = min(b.hi[d], n[d] - 1 + margin);
        }
    }
    return b;
}

// wrap a box coordinate into the lattice; false if outside a closed direction
__device__ inline bool wrap_coord(int &v, int n, int per) {
    if (per) {
        v %= n;
        if (v < 0) v += n;
        return true;
    }
    return v >= 0 && v < n;
}

// squared distance from lattice point p (unwrapped, near the rod) to the axis segment
__device__ inline double axis_dist2(const double *rod, d3 p, const RodArgs &a) {
    const d3 d = min_image(p - ld3(rod + ROD_X), a);
    const d3 e = quat_axis(rod + ROD_Q);
    const double t = fmin(fmax(dot(d, e), -a.half), a.half);
    const d3 c = d - t * e;
    return dot(c, c);
}

// out[q] = work-group sum of v[q], q < N: a fixed xor butterfly per wavefront,
// then the wavefront sums in order (sh: N x wavefronts doubles; out written by
// threads 0 .. N-1, zeros instead when `zero`)
template <int N>
__device__ inline void block_sums(double (&v)[N], double *sh, double *out, bool zero = false) {
#pragma unroll
    for (int q = 0; q < N; ++q)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0)
#pragma unroll
        for (int q = 0; q < N; ++q) sh[w * N + q] = v[q];
    __syncthreads();
    if (int(threadIdx.x) < N) {
        double s = 0.0;
        for (int k = 0; k < int(blockDim.x >> 6); ++k) s += sh[k * N + threadIdx.x];
        out[threadIdx.x] = zero ? 0.0 : s;
    }
}

constexpr int RB = 256;  // threads per per-rod work-group

}  // namespace

// ---------------------------------------------------------------------------
// Per-rod surface lists.  The re-mask (one work-group per rod) scans the
// rod's bounding box once and writes, in box order, every lattice node within
// R + 3/2 of the axis: all of the rod's nodes before and after a move of less
// than one node, and every fluid node that shares a link with them.  The
// passes that follow run one thread per listed node, work-group (b, r) on
// entries [b RB, (b + 1) RB) of rod r's list, and write their partial sums to
// slot [r][b]; consumers add the slots with a fixed wavefront butterfly.
// ---------------------------------------------------------------------------
constexpr int MB = 1024;  // threads of the re-mask work-group

__device__ inline double wave_sum_d(double v) {
    // xor butterfly: every lane ends with the same, order-fixed sum
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline double *part_slot(double *base, const RodArgs &a, int r, int b) {
    return base + (size_t(r) * a.nblk + b) * ROD_PART;
}

// The sum over rod r's nblk work-groups of their partial-sum slots of `part`
// (N values each), in work-group order, eight slots' loads in flight at a
// time (a slot past the end reads the last one again and adds zero; a select,
// not a branch, so that no load is deferred past it)
template <int N>
__device__ inline void slot_sums(const RodArgs &a, double *part, int r, double (&out)[N]) {
#pragma unroll
    for (int q = 0; q < N; ++q) out[q] = 0.0;
    for (int b0 = 0; b0 < a.nblk; b0 += 8) {
        double v[8][N];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double *ps = part_slot(part, a, r, min(b0 + u, a.nblk - 1));
#pragma unroll
            for (int q = 0; q < N; ++q) v[u][q] = gptr(ps)[q];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int q = 0; q < N; ++q) out[q] += b0 + u < a.nblk ? v[u][q] : 0.0;
    }
}

// record and local index of global rod g (one lattice when bt.map is null)
__device__ inline RodArgs rod_of(const RodBatch &bt, int g, int &r) {
    int lat = 0;
    r = g;
    if (bt.map) {
        const int2 m = bt.map[g];
        lat = m.x;
        r = m.y;
    }
    return bt.all[lat];
}

__device__ inline double shell_r2(const RodArgs &a) { return (a.radius + 1.5) * (a.radius + 1.5); }

// A work-group wholly past the end of rod r's surface list (the list holds
// far fewer nodes than its capacity) does no work: it writes the n zeros its
// block sums would have produced into its partial-sum slot (if any) and ends.
__device__ inline bool idle_block(const RodArgs &a, int r, double *slot, int n) {
    if (int(blockIdx.x) * RB < gptr(a.shell_cnt)[r]) return false;
    if (slot && int(threadIdx.x) < n) slot[threadIdx.x] = 0.0;
    return true;
}

// densities rho_k of fluid node n: from the density array while it holds the
// current state, else the FP64 sum of the node's populations
template <class S>
__device__ inline void node_densities(const RodArgs &a, int fresh, const S *f, int64_t n, double rho[2]) {
    if (fresh) {
        const typename Codec<S>::C *ro = static_cast<const typename Codec<S>::C *>(a.rho);
        rho[0] = double(ro[n]);
        rho[1] = double(ro[a.fs + n]);
        return;
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < Q; ++j) s += decf(f, (k * Q + j) * a.fs + n) + wgt<double>(j) * a.rho_ref[k];
        rho[k] = s;
    }
}

// densities rho_k of fluid node n as stored in the density array (which
// exists on every lattice with rods): loaded ahead of the neighbour ids and
// used only while the array holds the current state
template <class S>
__device__ inline void stored_densities(const RodArgs &a, int64_t n, double rho[2]) {
    const auto *ro = gptr(static_cast<const typename Codec<S>::C *>(a.rho));
    rho[0] = double(ro[n]);
    rho[1] = double(ro[a.fs + n]);
}

// listed node of this thread: false if the entry is past the end of the list
__device__ inline bool shell_node(const RodArgs &a, int r, int64_t &n, int &x, int &y, int &z) {
    const int idx = blockIdx.x * RB + threadIdx.x;
    if (idx >= gptr(a.shell_cnt)[r]) return false;
    // list entries are 32-bit node indices: 32-bit division
    const uint32_t u = static_cast<uint32_t>(gptr(a.shell)[size_t(r) * a.shell_cap + idx]);
    const uint32_t nx = a.nx, ny = a.ny, row = u / nx;
    n = u;
    x = int(u - row * nx);
    y = int(row % ny);
    z = int(row / ny);
    return true;
}

// Directions i (bit i) in which the node (x, y, z) + sgn c_i (sgn = +1 or -1,
// the node inside the lattice) belongs to rod r by the id array ids.  The neighbour across a
// closed boundary is read at its wrapped index and ignored, so that all 18
// loads are issued together instead of one after another behind the bounds
// tests.
template <class T>
__device__ inline unsigned rod_neighbours(const T *ids, const RodArgs &a, int x, int y, int z, int sgn, int r) {
    int id[Q];
    unsigned in = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        int xx = x + sgn * cx(i), yy = y + sgn * cy(i), zz = z + sgn * cz(i);
        const bool out = ((xx < 0 || xx >= a.nx) && !a.px) || ((yy < 0 || yy >= a.ny) && !a.py) ||
                         ((zz < 0 || zz >= a.nz) && !a.pz);
        xx = xx < 0 ? xx + a.nx : (xx >= a.nx ? xx - a.nx : xx);
        yy = yy < 0 ? yy + a.ny : (yy >= a.ny ? yy - a.ny : yy);
        zz = zz < 0 ? zz + a.nz : (zz >= a.nz ? zz - a.nz : zz);
        in |= out ? 0u : 1u << i;
        id[i] = gptr(ids)[(int64_t(zz) * a.ny + yy) * a.nx + xx];
    }
    unsigned m = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) m |= ((in >> i) & 1u) && id[i] == r ? 1u << i : 0u;
    return m;
}

// index of the node (x, y, z) + sgn c_i, for a direction rod_neighbours
// reported (so inside the lattice after one wrap)
__device__ inline int64_t step_node(const RodArgs &a, int x, int y, int z, int sgn, int i) {
    int xx = x + sgn * cx(i), yy = y + sgn * cy(i), zz = z + sgn * cz(i);
    xx = xx < 0 ? xx + a.nx : (xx >= a.nx ? xx - a.nx : xx);
    yy = yy < 0 ? yy + a.ny : (yy >= a.ny ? yy - a.ny : yy);
    zz = zz < 0 ? zz + a.nz : (zz >= a.nz ? zz - a.nz : zz);
    return (int64_t(zz) * a.ny + yy) * a.nx + xx;
}

// ---------------------------------------------------------------------------
// 1. reaction to the adhesion force: for fluid x next to rod node y = x + c_i,
//    F_rod += G psi_k(x) w_i psi^s_kbar c_i (psi_k(x) = rho_k(x), the collision
//    invariant of the current post-collision state), torque about X at y
// ---------------------------------------------------------------------------
// The pass also returns rod r's entries of newid to -1 for the next re-mask
// (the previous step's commit left them equal to the occupancy).
template <class S>
__global__ void __launch_bounds__(RB) rod_adhesion_kernel(RodBatch bt) {
    __shared__ double sh[RB / 64 * 8];
    int r;
    const RodArgs a = rod_of(bt, blockIdx.y, r);
    if (int(blockIdx.x) >= a.nblk) return;  // uniform per block
    double *rod = a.rods + r * ROD_STRIDE;
    if (idle_block(a, r, part_slot(a.part_adh, a, r, blockIdx.x), 6)) return;
    const S *f = static_cast<const S *>(a.f);
    const d3 X = ld3(rod + ROD_X);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    int64_t n;
    int x, y, z;
    if (shell_node(a, r, n, x, y, z)) {
        // material, densities and the 18 neighbour ids are loaded together
        const uint8_t mt = gptr(a.mat)[n];
        const int nid = gptr(a.newid)[n];
        double rho[2];
        stored_densities<S>(a, n, rho);
        unsigned links = rod_neighbours(a.rodid, a, x, y, z, 1, r);
        if ((mt & MAT_ID_MASK) != MAT_FLUID) links = 0;
        if (nid == r) a.newid[n] = -1;
        if (links) {
            if (!bt.rho_fresh) node_densities<S>(a, 0, f, n, rho);
            // every link's force is G (rho_A psi_B + rho_B psi_A) w_i c_i, and
            // its torque about X at the rod node x + c_i equals that of the
            // same force at x (c_i x c_i = 0): the node adds sum_i w_i c_i once
            double wx = 0.0, wy = 0.0, wz = 0.0;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const double w = (links >> i) & 1u ? wgt<double>(i) : 0.0;
                if (cx(i)) wx += cx(i) * w;
                if (cy(i)) wy += cy(i) * w;
                if (cz(i)) wz += cz(i) * w;
            }
            const double g = a.G * (rho[0] * a.psi_rod[1] + rho[1] * a.psi_rod[0]);
            const d3 fr = mk(g * wx, g * wy, g * wz);
            const d3 tq = cross(min_image(mk(x, y, z) - X, a), fr);
            acc[0] = fr.x;
            acc[1] = fr.y;
            acc[2] = fr.z;
            acc[3] = tq.x;
            acc[4] = tq.y;
            acc[5] = tq.z;
        }
    }
    block_sums(acc, sh, part_slot(a.part_adh, a, r, blockIdx.x));
}

// ---------------------------------------------------------------------------
// 2a. per rod (one wavefront, run as an extra work-group of the re-mask
//     launch, after the rods have moved): the list of rods that can come
//     within interaction range during the next step (each point of a rod
//     moves less than 0.9 per step, so a pair farther apart than r_int + 2 at
//     the start stays out of range)
// ---------------------------------------------------------------------------
__device__ void rod_list(const RodBatch &bt, int g) {
    int r;
    const RodArgs a = rod_of(bt, g, r);
    const int lane = threadIdx.x;
    const double *rod = a.rods + r * ROD_STRIDE;
    const double r_int = fmax(a.d0, a.eps_att > 0.0 ? a.r_cut : a.d0);
    const double keep = r_int + 2.0, reach = 2.0 * a.half + keep;
    const d3 Xa = ld3(rod + ROD_X), ea = quat_axis(rod + ROD_Q);
    const d3 pa = Xa - a.half * ea, qa = Xa + a.half * ea;
    int base = 0;
    for (int s0 = 0; s0 < a.n_rods; s0 += 64) {
        const int s = s0 + lane;
        bool near = false;
        if (s < a.n_rods && s != r) {
            const double *rb = a.rods + s * ROD_STRIDE;
            const d3 Xb = ld3(rb + ROD_X);
            const d3 dx = min_image(Xb - Xa, a);
            if (dot(dx, dx) < reach * reach) {
                const d3 shift = dx - (Xb - Xa);
                const d3 eb = quat_axis(rb + ROD_Q);
                d3 ca, cb;
                near = seg_seg(pa, qa, Xb - a.half * eb + shift, Xb + a.half * eb + shift, ca, cb) < keep;
            }
        }
        const uint64_t bal = __ballot(near);
        const int slot = base + __popcll(bal & ((uint64_t(1) << lane) - 1));
        if (near) {
            if (slot < ROD_NBR) a.nbr[r * ROD_NBR + slot] = static_cast<int16_t>(s);
            else atomicOr(a.status, ST_ROD_LIST);  // more neighbours than the list holds
        }
        base += __popcll(bal);
    }
    if (lane == 0) a.nbr_cnt[r] = min(base, ROD_NBR);
}

// ---------------------------------------------------------------------------
// 2b. rigid-body substeps: one work-group of LB_MAX_RODS threads.  Centres
//     and axes of all rods live in shared memory for the whole step.  Pair
//     forces: the neighbour lists are laid end to end into one list of
//     (rod, neighbour) terms, dealt to all threads of the work-group (one
//     term per thread while there are fewer terms than threads), so that the
//     FP64 work spreads over every wavefront instead of following the longest
//     list; each term's force and torque go to shared memory, and thread r
//     adds rod r's terms in list order.  Rod update: thread r keeps rod r's
//     velocity, angular momentum and fluid load in registers and advances it.
// ---------------------------------------------------------------------------
constexpr int RS_X = 0, RS_Q = 3, RS_N = 7;  // shared-memory record per rod: X, q
constexpr int TCAP = 1024;  // pair terms whose results shared memory holds at a time
constexpr int TPK = 4096;   // pair terms whose (rod, neighbour) is kept for the step

__global__ void __launch_bounds__(LB_MAX_RODS) rod_integrate_kernel(RodBatch bt) {
    extern __shared__ double rs[];  // [n_rods][RS_N]
    __shared__ int toff[LB_MAX_RODS + 1];  // rod r's terms: [toff[r], toff[r + 1])
    __shared__ int tpair[TPK];             // term g < TPK: rod | neighbour << 16
    __shared__ double tres[TCAP][6];       // force, torque of the terms of one chunk
    __shared__ int wsum[LB_MAX_RODS / 64];
    __shared__ double lsum[LB_MAX_RODS / 2][8];
    const RodArgs a = bt.all[blockIdx.x];  // one work-group per lattice
    const int nr = a.n_rods;
    if (nr == 0) return;  // uniform per work-group
    const int me = threadIdx.x, lane = me & 63, wv = me >> 6;
    const bool mine = me < nr;
    const double dt = 1.0 / a.n_sub;
    d3 V = mk(0, 0, 0), Lm = mk(0, 0, 0), Fx = mk(0, 0, 0), Tx = mk(0, 0, 0), F = mk(0, 0, 0), T = mk(0, 0, 0);
    double *rm = rs + (mine ? me : 0) * RS_N;
    const double *rod = a.rods + (mine ? me : 0) * ROD_STRIDE;
    d3 X0 = mk(0, 0, 0), e0 = mk(0, 0, 1);
    const int nn = mine ? gptr(a.nbr_cnt)[me] : 0;
    const bool split = nr <= LB_MAX_RODS / 2;
    double ad[6], ls[8];
    if (mine) {
        // every load of the prologue is issued before the first store to
        // shared memory (which the compiler must assume may alias them)
        double xq[7];
#pragma unroll
        for (int q = 0; q < 7; ++q) xq[q] = gptr(rod)[ROD_X + q];  // X then q
        V = gld3(rod + ROD_V);
        Lm = gld3(rod + ROD_L);
        // the adhesion reaction of the step that just ran
        slot_sums(a, a.part_adh, me, ad);
        if (!split) slot_sums(a, a.part_link, me, ls);
#pragma unroll
        for (int q = 0; q < 7; ++q) rm[RS_X + q] = xq[q];
        X0 = mk(xq[0], xq[1], xq[2]);
        e0 = quat_axis(xq + 3);
    }
    // the momentum of the links the fluid step just streamed (their mass is
    // booked now): summed by the upper half of the work-group when the rods
    // fit in the lower half
    if (split && me >= LB_MAX_RODS / 2 && me - LB_MAX_RODS / 2 < nr) {
        double t[8];
        slot_sums(a, a.part_link, me - LB_MAX_RODS / 2, t);
#pragma unroll
        for (int q = 0; q < 8; ++q) lsum[me - LB_MAX_RODS / 2][q] = t[q];
    }
    // term offsets: exclusive scan of the list lengths over the work-group
    int v = nn;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) wsum[wv] = v;
    __syncthreads();
    int base = 0, total = 0;
    for (int w = 0; w < LB_MAX_RODS / 64; ++w) {
        base += w < wv ? wsum[w] : 0;
        total += wsum[w];
    }
    const int my_off = base + v - nn;
    if (mine) {
        if (split)
#pragma unroll
            for (int q = 0; q < 8; ++q) ls[q] = lsum[me][q];
        double *rw = a.rods + me * ROD_STRIDE;
#pragma unroll
        for (int q = 0; q < 6; ++q) rw[ROD_FS + q] = ls[q];
#pragma unroll
        for (int q = 0; q < 6; ++q) rw[ROD_FA + q] = ad[q];
        rw[ROD_SOLID] += ls[6];
        rw[ROD_SOLID + 1] += ls[7];
        Fx = mk(ls[0], ls[1], ls[2]) + mk(ad[0], ad[1], ad[2]);
        Tx = mk(ls[3], ls[4], ls[5]) + mk(ad[3], ad[4], ad[5]);
        toff[me] = my_off;
    }
    if (me == 0) toff[nr] = total;
    const int nterm = total;
    // rod me's list into the kept term table (entries in list order)
    if (mine) {
        for (int l0 = 0; l0 < nn; l0 += 8) {
            int16_t sb[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) sb[u] = gptr(a.nbr)[me * ROD_NBR + min(l0 + u, nn - 1)];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (l0 + u < nn && my_off + l0 + u < TPK) tpair[my_off + l0 + u] = me | (int(sb[u]) << 16);
        }
    }
    const double dt_m = dt / a.mass, iIperp = 1.0 / a.Iperp, dI = 1.0 / a.Ipar - 1.0 / a.Iperp;
    const double reach = a.half + a.radius;
    bool moved_far = false;
    // distance check of the previous substep's pose, made while the next
    // substep's pair forces are computed (off the update's critical path)
    d3 Xc = X0, ec = e0;
    __syncthreads();

    // force and torque on rod ra from rod rb at this substep's poses; exactly
    // zero for touching axes (d = 0) and beyond the potential's range
    auto term = [&](int g, double (&out)[6]) {
        int ra, rb;
        if (g < TPK) {
            const int pq = tpair[g];
            ra = pq & 0xffff;
            rb = pq >> 16;
        } else {  // past the kept table: the owning rod by bisection of the offsets
            int lo = 0, hi = nr - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (toff[mid] <= g) lo = mid;
                else hi = mid - 1;
            }
            ra = lo;
            rb = gptr(a.nbr)[ra * ROD_NBR + (g - toff[ra])];
        }
        const double *pa_ = rs + ra * RS_N, *pb_ = rs + rb * RS_N;
        const d3 Xa = ld3(pa_ + RS_X), ea = quat_axis(pa_ + RS_Q);
        const d3 Xb = ld3(pb_ + RS_X), eb = quat_axis(pb_ + RS_Q);
        const d3 pa = Xa - a.half * ea, qa = Xa + a.half * ea;
        const d3 dx = min_image(Xb - Xa, a);
        const d3 shift = dx - (Xb - Xa);
        const d3 pb = Xb - a.half * eb + shift, qb = Xb + a.half * eb + shift;
        d3 ca, cb;
        const double d = seg_seg(pa, qa, pb, qb, ca, cb);
        const double fmd = d > 0.0 ? pair_force_over_d(d, a) : 0.0;
        const d3 fv = fmd * (ca - cb);
        const d3 tv = cross(ca - Xa, fv);
        out[0] = fv.x;
        out[1] = fv.y;
        out[2] = fv.z;
        out[3] = tv.x;
        out[4] = tv.y;
        out[5] = tv.z;
    };

    for (int sub = 0; sub < a.n_sub; ++sub) {
        // contact forces between rods at the positions of this substep, in
        // chunks of TCAP terms (a single chunk unless the lists are long)
        d3 Fp = mk(0, 0, 0), Tp = mk(0, 0, 0);
        for (int c0 = 0; c0 < nterm; c0 += TCAP) {
            const int c1 = min(nterm, c0 + TCAP);
            // two terms per thread and iteration, so that their dependent
            // FP64 chains interleave
            for (int g = c0 + me; g < c1; g += 2 * LB_MAX_RODS) {
                double o0[6], o1[6];
                const int g1 = g + LB_MAX_RODS;
                term(g, o0);
                if (g1 < c1) term(g1, o1);
#pragma unroll
                for (int q = 0; q < 6; ++q) tres[g - c0][q] = o0[q];
                if (g1 < c1)
#pragma unroll
                    for (int q = 0; q < 6; ++q) tres[g1 - c0][q] = o1[q];
            }
            __syncthreads();
            if (mine) {  // rod me's terms of this chunk, in list order
                const int l0 = max(my_off, c0), l1 = min(my_off + nn, c1);
                for (int l = l0; l < l1; ++l) {
                    Fp = Fp + mk(tres[l - c0][0], tres[l - c0][1], tres[l - c0][2]);
                    Tp = Tp + mk(tres[l - c0][3], tres[l - c0][4], tres[l - c0][5]);
                }
            }
            if (c1 < nterm) __syncthreads();  // the next chunk overwrites the results
        }
        if (mine) {
            {
                const d3 dX = min_image(Xc - X0, a);
                const d3 de = ec - e0;
                moved_far |= !(sqrt(dot(dX, dX)) + reach * sqrt(dot(de, de)) < 0.9);
            }
            F = Fp;
            T = Tp;
            if (a.wall_on) {
                const d3 Xa = ld3(rm + RS_X), ea = quat_axis(rm + RS_Q);
                const d3 pa = Xa - a.half * ea, qa = Xa + a.half * ea;
                const d3 low = pa.z <= qa.z ? pa : qa;
                const double h = low.z - a.wall_z;
                if (h > 0.0 && h <= a.d0_wall) {
                    const d3 fw = mk(0, 0, -a.eps_wall * ljf_d(h, a.d0_wall));
                    F = F + fw;
                    T = T + cross(low - Xa, fw);
                }
            }
            V = V + dt_m * (Fx + F);
            d3 X = ld3(rm + RS_X) + dt * V;
            Lm = Lm + dt * (Tx + T);
            // omega = I^-1 L with the current axis, then q <- exp(omega dt / 2) q
            const d3 e = quat_axis(rm + RS_Q);
            const d3 w = iIperp * Lm + (dI * dot(Lm, e)) * e;
            const double wn = sqrt(dot(w, w));
            if (wn > 0.0) {
                const double h = 0.5 * wn * dt;
                double sn, cs;
                sincos(h, &sn, &cs);
                const double sh = sn / wn;
                const double dq[4] = {cs, sh * w.x, sh * w.y, sh * w.z};
                const double q[4] = {rm[RS_Q], rm[RS_Q + 1], rm[RS_Q + 2], rm[RS_Q + 3]};
                double qn[4] = {dq[0] * q[0] - dq[1] * q[1] - dq[2] * q[2] - dq[3] * q[3],
                                dq[0] * q[1] + dq[1] * q[0] + dq[2] * q[3] - dq[3] * q[2],
                                dq[0] * q[2] - dq[1] * q[3] + dq[2] * q[0] + dq[3] * q[1],
                                dq[0] * q[3] + dq[1] * q[2] - dq[2] * q[1] + dq[3] * q[0]};
                const double nq = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
#pragma unroll
                for (int c = 0; c < 4; ++c) rm[RS_Q + c] = qn[c] / nq;
            }
            if (a.px) X.x = X.x - a.nx * floor(X.x / a.nx);
            if (a.py) X.y = X.y - a.ny * floor(X.y / a.ny);
            if (a.pz) X.z = X.z - a.nz * floor(X.z / a.nz);
            st3(rm + RS_X, X);
            // every point of the rod stays within 0.9 of where it started the
            // step (the re-mask and the neighbour list rely on it): checked at
            // the start of the next substep and after the last
            Xc = X;
            ec = quat_axis(rm + RS_Q);
        }
        __syncthreads();
    }
    if (mine) {
        const d3 dX = min_image(Xc - X0, a);
        const d3 de = ec - e0;
        moved_far |= !(sqrt(dot(dX, dX)) + reach * sqrt(dot(de, de)) < 0.9);
        double *rw = a.rods + me * ROD_STRIDE;
#pragma unroll
        for (int q = 0; q < 7; ++q) rw[ROD_X + q] = rm[RS_X + q];
        st3(rw + ROD_V, V);
        st3(rw + ROD_L, Lm);
        st3(rw + ROD_VPRE, V);
        st3(rw + ROD_LPRE, Lm);
        st3(rw + ROD_FC, F);
        st3(rw + ROD_TC, T);
        if (moved_far) atomicOr(a.status, ST_ROD);
    }
}

// ---------------------------------------------------------------------------
// 3. re-mask: new occupancy of every rod (newid is -1 everywhere on entry) and
//    the rod's surface list; one work-group per rod
//
// A rod's axis-aligned box is mostly empty for an oblique rod (a 24-node rod
// on a diagonal fills a few percent of it), so the nodes visited are the
// box's x-rows cut down to the x-interval within the shell radius of the
// infinite axis line (a quadratic in x per row; the capsule's shell lies
// inside that cylinder), widened by a node on each side.  Rows keep the box
// order (z, then y, then x ascending), so the list is the one a walk over
// the whole box gives.  Where the box wraps round a periodic x (lattices
// about as small as the rod) or has more rows than the row table holds, the
// walk covers whole rows.
// ---------------------------------------------------------------------------
constexpr int MASK_ROWS = 4096;  // row table of the re-mask work-group
static_assert(MASK_ROWS % MB == 0, "rows are scanned MB at a time");

__global__ void __launch_bounds__(MB) rod_mask_kernel(RodBatch bt) {
    __shared__ int wcount[MB / 64];
    __shared__ int row_start[MASK_ROWS + 1];
    __shared__ int row_x0[MASK_ROWS];
    // the launch has twice as many work-groups as rods: the second half
    // builds the neighbour lists for the next step
    const int nrod = gridDim.x / 2;
    if (int(blockIdx.x) >= nrod) {
        if (threadIdx.x < 64) rod_list(bt, blockIdx.x - nrod);
        return;
    }
    int r;
    const RodArgs a = rod_of(bt, blockIdx.x, r);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double *rod = a.rods + r * ROD_STRIDE;
    const Box b = rod_box(rod, a, 2);
    const int ex = b.hi[0] - b.lo[0] + 1, ey = b.hi[1] - b.lo[1] + 1, ez = b.hi[2] - b.lo[2] + 1;
    // a box is a few thousand nodes: 32-bit index arithmetic; a box beyond
    // 2^30 nodes can only come from a rod state gone bad, which is flagged
    const int64_t nbox64 = (ex > 0 && ey > 0 && ez > 0) ? int64_t(ex) * ey * ez : 0;
    if (nbox64 > (int64_t(1) << 30) && threadIdx.x == 0) atomicOr(a.status, ST_ROD_WALL);
    const int nbox = nbox64 > (int64_t(1) << 30) ? 0 : int(nbox64);
    const int nrows = nbox ? ey * ez : 0;
    const double r2in = a.radius * a.radius, r2sh = shell_r2(a);
    const d3 X = ld3(rod + ROD_X), e = quat_axis(rod + ROD_Q);

    // rows: candidate x-interval and its length, then starts by a block scan
    const bool rows_fit = nrows <= MASK_ROWS;
    int total = nbox;
    if (rows_fit) {
        const bool cull = !a.px || (X.x - b.lo[0] < 0.5 * a.nx - 1.0 && b.hi[0] - X.x < 0.5 * a.nx - 1.0);
        // r2c: the shell radius with a margin far above the rounding of the
        // discriminant; rods within ~2 degrees of x (A < 1e-3) walk whole rows
        const double A = 1.0 - e.x * e.x, r2c = r2sh + 1e-6;
        int carry = 0;
        for (int q0 = 0; q0 < MASK_ROWS && q0 < nrows; q0 += MB) {
            const int q = q0 + int(threadIdx.x);
            int x0 = b.lo[0], cnt = 0;
            if (q < nrows) {
                int x1 = b.hi[0];
                if (cull && A > 1e-3) {
                    const int mz = q / ey, my = q - mz * ey;
                    const double dy = min_img(double(b.lo[1] + my) - X.y, a.ny, a.py);
                    const double dz = min_img(double(b.lo[2] + mz) - X.z, a.nz, a.pz);
                    // |d|^2 - (d.e)^2 <= r^2 with d = (x - X.x, dy, dz)
                    const double sp = dy * e.y + dz * e.z;
                    const double B = -2.0 * e.x * sp, C = dy * dy + dz * dz - sp * sp - r2c;
                    const double disc = B * B - 4.0 * A * C;
                    if (disc < 0.0) {
                        x1 = x0 - 1;
                    } else {
                        const double sq = sqrt(disc), i2a = 0.5 / A;
                        const double lo = fmin(fmax(X.x + (-B - sq) * i2a, b.lo[0] - 2.0), b.hi[0] + 2.0);
                        const double hi = fmin(fmax(X.x + (-B + sq) * i2a, b.lo[0] - 2.0), b.hi[0] + 2.0);
                        x0 = max(x0, int(floor(lo)) - 1);
                        x1 = min(x1, int(ceil(hi)) + 1);
                    }
                }
                cnt = max(x1 - x0 + 1, 0);
            }
            // exclusive scan of cnt over the work-group
            int v = cnt;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int u = __shfl_up(v, off, 64);
                if (lane >= off) v += u;
            }
            if (lane == 63) wcount[wv] = v;
            __syncthreads();
            int wbase = 0, tot = 0;
            for (int w = 0; w < MB / 64; ++w) {
                wbase += w < wv ? wcount[w] : 0;
                tot += wcount[w];
            }
            if (q < nrows) {
                row_start[q] = carry + wbase + v - cnt;
                row_x0[q] = x0;
            }
            carry += tot;
            __syncthreads();
        }
        if (threadIdx.x == 0) row_start[nrows] = carry;
        __syncthreads();
        total = carry;
    }

    int base = 0;  // same in every thread
    for (int m0 = 0; m0 < total; m0 += MB) {
        const int m = m0 + int(threadIdx.x);
        bool listed = false;
        int64_t n = 0;
        if (m < total) {
            int x, y, z;
            if (rows_fit) {
                // the row holding candidate m: the last start <= m
                int lo = 0, hi = nrows - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (row_start[mid] <= m) lo = mid;
                    else hi = mid - 1;
                }
                const int mz = lo / ey, my = lo - mz * ey;
                x = row_x0[lo] + (m - row_start[lo]);
                y = b.lo[1] + my;
                z = b.lo[2] + mz;
            } else {
                const int exy = ex * ey;
                const int mz = m / exy, rem = m - mz * exy, my = rem / ex;
                x = b.lo[0] + (rem - my * ex);
                y = b.lo[1] + my;
                z = b.lo[2] + mz;
            }
            const double d2 = axis_dist2(rod, mk(x, y, z), a);
            const bool in_box = wrap_coord(x, a.nx, a.px) && wrap_coord(y, a.ny, a.py) && wrap_coord(z, a.nz, a.pz);
            if (d2 <= r2in && !in_box) atomicOr(a.status, ST_ROD_WALL);  // a rod left the lattice
            if (d2 <= r2sh && in_box) {
                n = (int64_t(z) * a.ny + y) * a.nx + x;
                listed = true;
                if (d2 <= r2in) {
                    const uint8_t mt = a.mat[n] & MAT_ID_MASK;
                    // overlapping rods: the highest index keeps the node
                    if (mt == MAT_FLUID || mt == MAT_ROD) atomicMax(&a.newid[n], r);
                    else atomicOr(a.status, ST_ROD_WALL);  // a rod ran into a wall or the reservoir
                }
            }
        }
        // append the listed nodes in box order
        const uint64_t bal = __ballot(listed);
        if (lane == 0) wcount[wv] = __popcll(bal);
        __syncthreads();
        int off = 0, tot = 0;
        for (int q = 0; q < MB / 64; ++q) {
            off += q < wv ? wcount[q] : 0;
            tot += wcount[q];
        }
        if (listed) {
            const int idx = base + off + __popcll(bal & ((uint64_t(1) << lane) - 1));
            if (idx < a.shell_cap) a.shell[size_t(r) * a.shell_cap + idx] = static_cast<int>(n);
            else atomicOr(a.status, ST_ROD_LIST);  // cannot happen for a capsule of the stated size
        }
        base += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) a.shell_cnt[r] = min(base, a.shell_cap);
}

__global__ void fill_i32_kernel(int *p, int64_t n, int v) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------
// 4. cover / uncover (init = 1: place the rods without bookkeeping)
//    A covered node is handled by the thread that finds it.  Uncovered nodes
//    are compacted in thread order into shared memory and refilled by a whole
//    wavefront each (two lanes per neighbour gather the neighbour densities);
//    the finding thread then adds the transfer to its own sums.
// ---------------------------------------------------------------------------
template <class S>
__global__ void __launch_bounds__(RB) rod_update_kernel(RodBatch bt, int init) {
    __shared__ double sh[RB / 64 * 8];
    __shared__ int wcount[RB / 64];
    __shared__ int64_t un_node[RB];
    __shared__ double un_out[RB][8];
    int r;
    const RodArgs a = rod_of(bt, blockIdx.y, r);
    if (int(blockIdx.x) >= a.nblk) return;  // uniform per block
    if (idle_block(a, r, part_slot(a.part_upd, a, r, blockIdx.x), 8)) return;
    S *f = static_cast<S *>(a.f);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double *rod = a.rods + r * ROD_STRIDE;
    const d3 X = ld3(rod + ROD_X);
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // momentum[3], torque[3], mass[2]
    int64_t n = 0;
    int x = 0, y = 0, z = 0;
    bool unc = false;
    if (shell_node(a, r, n, x, y, z)) {
        // a node passing from one rod to another stays solid and is neither
        const int oldid = gptr(a.rodid)[n], newid = gptr(a.newid)[n];
        unc = oldid == r && newid < 0;
        if (newid == r && oldid < 0) {  // covered
            if (!init) {
                const d3 arm = min_image(mk(x, y, z) - X, a);
                d3 mom = mk(0, 0, 0);
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    double s = 0.0;
                    d3 jk = mk(0, 0, 0);
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        const double v = decf(f, (k * Q + i) * a.fs + n) + wgt<double>(i) * a.rho_ref[k];
                        s += v;
                        jk = jk + v * mk(cx(i), cy(i), cz(i));
                    }
                    acc[6 + k] += s;
                    mom = mom + jk;
                }
                const d3 tq = cross(arm, mom);
                acc[0] += mom.x;
                acc[1] += mom.y;
                acc[2] += mom.z;
                acc[3] += tq.x;
                acc[4] += tq.y;
                acc[5] += tq.z;
            }
            a.mat[n] = MAT_ROD;
        }
    }
    // compact the uncovered nodes in thread order
    const uint64_t bal = __ballot(unc);
    if (lane == 0) wcount[wv] = __popcll(bal);
    __syncthreads();
    int off = 0, tot = 0;
    for (int q = 0; q < RB / 64; ++q) {
        off += q < wv ? wcount[q] : 0;
        tot += wcount[q];
    }
    const int slot = off + __popcll(bal & ((uint64_t(1) << lane) - 1));
    if (unc) un_node[slot] = n;
    __syncthreads();
    // refill: f = f^eq(rho_bar, u_b), rho_bar = mean over the neighbours that
    // are fluid before and after the move.  A node with none of them (a
    // pocket enclosed by touching capsules) takes the mean over the first
    // ring x + s c_i, s = 2 .. reach, that holds any, and raises the notice
    // bit ST_REFILL_FAR.
    const int reach = int(ceil(2.0 * a.radius)) + 2;
    for (int e = wv; e < tot; e += RB / 64) {
        const int64_t un = un_node[e];
        const uint32_t uu = static_cast<uint32_t>(un), urow = uu / uint32_t(a.nx);
        const int ux = int(uu - urow * uint32_t(a.nx)), uy = int(urow % uint32_t(a.ny)), uz = int(urow / uint32_t(a.ny));
        const int i = 1 + (lane >> 1), k = lane & 1;
        // select, not index: a run-time index into the argument record would
        // put the whole record in private memory
        const double rref_k = k ? a.rho_ref[1] : a.rho_ref[0];
        double val = 0.0;
        bool ok = false, wall = false;
        int cnt = 0;
        for (int sr = 1; sr <= reach; ++sr) {  // wave-uniform: ends at the first ring with fluid
            val = 0.0;
            ok = false;
            if (lane < 2 * (Q - 1)) {
                int xx = ux + sr * cx(i), yy = uy + sr * cy(i), zz = uz + sr * cz(i);
                const bool okx = wrap_coord(xx, a.nx, a.px), oky = wrap_coord(yy, a.ny, a.py);
                const bool inb = okx && oky && wrap_coord(zz, a.nz, a.pz);
                // material, ids and stored density of the neighbour loaded
                // together (a neighbour outside the lattice reads the node itself)
                const int64_t q = inb ? (int64_t(zz) * a.ny + yy) * a.nx + xx : un;
                const uint8_t mq = gptr(a.mat)[q] & MAT_ID_MASK;
                const int rq = gptr(a.rodid)[q], nq = gptr(a.newid)[q];
                const double dq = double(gptr(static_cast<const typename Codec<S>::C *>(a.rho))[k * a.fs + q]);
                if (sr == 1) wall = inb && is_static_wall(mq);
                ok = inb && mq == MAT_FLUID && rq < 0 && nq < 0;
                double v = dq;  // used on every path, so its load is not deferred into a branch
                if (ok && !bt.rho_fresh) {
                    double s = 0.0;
#pragma unroll
                    for (int j = 0; j < Q; ++j) s += decf(f, (k * Q + j) * a.fs + q) + wgt<double>(j) * rref_k;
                    v = s;
                }
                val = ok ? v : 0.0;
            }
            cnt = __popcll(__ballot(ok && k == 0));
            if (cnt) {
                if (sr > 1 && lane == 0) atomicOr(a.status, ST_REFILL_FAR);
                break;
            }
        }
        const bool near_wall = __ballot(wall) != 0;
        double rb[2] = {wave_sum_d(k == 0 ? val : 0.0), wave_sum_d(k == 1 ? val : 0.0)};
        if (cnt) {
            rb[0] /= cnt;
            rb[1] /= cnt;
        }
        const d3 pu = mk(ux, uy, uz);
        const d3 ub = velocity_at(rod, pu, a);
        const double usq = dot(ub, ub);
        if (lane < 2 * Q) {
            const int kk = lane / Q, ii = lane % Q;
            const double cu = cx(ii) * ub.x + cy(ii) * ub.y + cz(ii) * ub.z;
            const double feq = wgt<double>(ii) * (kk ? rb[1] : rb[0]) * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
            f[(kk * Q + ii) * a.fs + un] =
                Codec<S>::enc(typename Codec<S>::C(feq - wgt<double>(ii) * (kk ? a.rho_ref[1] : a.rho_ref[0])));
        }
        // the refilled node's densities (those of f^eq) keep the density
        // array valid for the passes after this one
        if (bt.rho_fresh && lane < 2)
            static_cast<typename Codec<S>::C *>(a.rho)[lane * a.fs + un] = typename Codec<S>::C(rb[lane]);
        if (lane == 0) {
            const d3 mom = (rb[0] + rb[1]) * ub;
            const d3 tq = cross(min_image(pu - X, a), mom);
            un_out[e][0] = -mom.x;
            un_out[e][1] = -mom.y;
            un_out[e][2] = -mom.z;
            un_out[e][3] = -tq.x;
            un_out[e][4] = -tq.y;
            un_out[e][5] = -tq.z;
            un_out[e][6] = -rb[0];
            un_out[e][7] = -rb[1];
            a.mat[un] = MAT_FLUID | (near_wall ? MAT_NEAR_WALL : 0);
        }
    }
    __syncthreads();
    if (unc) {
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] += un_out[slot][q];
    }
    block_sums(acc, sh, part_slot(a.part_upd, a, r, blockIdx.x), init != 0);
}

// totals over rods in a fixed order: solid ledger [2], rod momentum M V [3]
__global__ void rod_sums_kernel(RodArgs a, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s[5] = {0, 0, 0, 0, 0};
    for (int r = 0; r < a.n_rods; ++r) {
        const double *rod = a.rods + r * ROD_STRIDE;
        s[0] += rod[ROD_SOLID];
        s[1] += rod[ROD_SOLID + 1];
        for (int q = 0; q < 3; ++q) s[2 + q] += a.mass * rod[ROD_V + q];
    }
    for (int q = 0; q < 5; ++q) out[q] = s[q];
}

// ---------------------------------------------------------------------------
// 5. commit and moving bounce-back slots.  COMMIT (after a re-mask): commit
//    the new occupancy of rod r -- every work-group of the update pass has
//    read the old one -- and apply the rod's cover/uncover transfers; then,
//    with the new occupancy (newid, equal to what the commit writes) and the
//    momenta after the transfers, write the slots the next pull reads and the
//    momentum they carry.  Without COMMIT (the occupancy is current, as after
//    a lift): the slots only.
// ---------------------------------------------------------------------------
template <class S, bool COMMIT>
__global__ void __launch_bounds__(RB) rod_link_kernel(RodBatch bt, int init) {
    using C = typename Codec<S>::C;
    __shared__ double sh[RB / 64 * 8];
    __shared__ double tr[8];
    int r;
    const RodArgs a = rod_of(bt, blockIdx.y, r);
    if (int(blockIdx.x) >= a.nblk) return;  // uniform per block
    double *rod = a.rods + r * ROD_STRIDE;
    // work-group 0 books the transfers even when the list is empty
    if (!(COMMIT && blockIdx.x == 0) && idle_block(a, r, part_slot(a.part_link, a, r, blockIdx.x), 8)) return;
    S *f = static_cast<S *>(a.f);
    const d3 X = ld3(rod + ROD_X);
    d3 Vr = ld3(rod + ROD_V), Lr = ld3(rod + ROD_L);
    if (COMMIT && !init) {
        // every work-group sums the update pass's transfers in the same order
        // and adds them to the momenta the integrator left, so that none reads
        // the record work-group 0 rewrites
        if (threadIdx.x < 64) {
            double t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int b = threadIdx.x; b < a.nblk; b += 64) {
                const double *p = part_slot(a.part_upd, a, r, b);
#pragma unroll
                for (int q = 0; q < 8; ++q) t[q] += gptr(p)[q];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) t[q] = wave_sum_d(t[q]);
            if (threadIdx.x == 0)
#pragma unroll
                for (int q = 0; q < 8; ++q) tr[q] = t[q];
        }
        __syncthreads();
        const d3 V0 = ld3(rod + ROD_VPRE), L0 = ld3(rod + ROD_LPRE);
        Vr = mk(V0.x + tr[0] / a.mass, V0.y + tr[1] / a.mass, V0.z + tr[2] / a.mass);
        Lr = mk(L0.x + tr[3], L0.y + tr[4], L0.z + tr[5]);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st3(rod + ROD_V, Vr);
            st3(rod + ROD_L, Lr);
            rod[ROD_SOLID] += tr[6];
            rod[ROD_SOLID + 1] += tr[7];
        }
    }
    // the rod's angular velocity I^-1 L, once per work-group
    const d3 e = quat_axis(rod + ROD_Q);
    const d3 Om = (1.0 / a.Iperp) * Lr + ((1.0 / a.Ipar - 1.0 / a.Iperp) * dot(Lr, e)) * e;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // dP[3], dT[3], mass[2]
    int64_t n;
    int x, y, z;
    if (shell_node(a, r, n, x, y, z)) {
        // material, densities and the 18 neighbour ids are loaded together
        const uint8_t mt = gptr(a.mat)[n];
        const int oid = gptr(a.rodid)[n], nid = gptr(a.newid)[n];
        double rho[2];
        stored_densities<S>(a, n, rho);
        unsigned links = COMMIT ? rod_neighbours(a.newid, a, x, y, z, -1, r) : rod_neighbours(a.rodid, a, x, y, z, -1, r);
        if ((mt & MAT_ID_MASK) != MAT_FLUID) links = 0;
        if (COMMIT && (oid == r || nid == r)) a.rodid[n] = int16_t(nid);
        if (links) {
            if (!bt.rho_fresh) node_densities<S>(a, 0, f, n, rho);
            // f*_opp(i)(x) of every linked direction, all loads in flight
            // together: a lane without the link reads its node's rest
            // population instead (a line the wave reads anyway), so that no
            // load sits behind a branch that would wait for it
            S fo[Q][2];
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const bool l = (links >> i) & 1u;
#pragma unroll
                for (int k = 0; k < 2; ++k) fo[i][k] = gload(f + (l ? (k * Q + opp(i)) * a.fs : 0) + n);
            }
            const d3 dx0 = min_image(mk(x, y, z) - X, a);
            // wall velocity at the link midpoint x - c_i / 2: V + Omega x (dx0 -
            // c_i / 2), whose component along c_i is that of u0 = V + Omega x dx0
            // (Omega x c_i is normal to c_i)
            const d3 u0 = Vr + cross(Om, dx0);
            d3 P = mk(0, 0, 0);
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                if (!((links >> i) & 1u)) continue;
                const int64_t s = step_node(a, x, y, z, -1, i);
                const double cu = cx(i) * u0.x + cy(i) * u0.y + cz(i) * u0.z;
                double q = 0.0;
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const double f_o = double(Codec<S>::dec(fo[i][k])) + wgt<double>(opp(i)) * a.rho_ref[k];
                    const double add = 2.0 * wgt<double>(i) * rho[k] * cu * 3.0;
                    const double fin = f_o + add;
                    f[(k * Q + i) * a.fs + s] = Codec<S>::enc(C(fin - wgt<double>(i) * a.rho_ref[k]));
                    q += f_o + fin;
                    acc[6 + k] -= add;
                }
                // the link's momentum -(f_o + fin) c_i; its torque about X at the
                // midpoint equals that at x (c_i x c_i = 0)
                P = P - q * mk(cx(i), cy(i), cz(i));
            }
            const d3 tq = cross(dx0, P);
            acc[0] = P.x;
            acc[1] = P.y;
            acc[2] = P.z;
            acc[3] = tq.x;
            acc[4] = tq.y;
            acc[5] = tq.z;
        }
    }
    // read by the next rod update, after the fluid step has streamed these slots
    block_sums(acc, sh, part_slot(a.part_link, a, r, blockIdx.x));
}

// ---------------------------------------------------------------------------
// 6. surrogate jumps: advect the rods with the time-averaged coarse velocity
//    of the canvases before and after the jump, then re-place them
// ---------------------------------------------------------------------------
// centre height that keeps a capsule of axis e off the closed end planes: one
// fluid node between its surface and each plane
__device__ inline double clamp_ends(const RodArgs &a, d3 e, double z) {
    const double ez = fabs(e.z) * a.half + a.radius;
    return fmin(fmax(z, 1.5 + ez), a.nz - 2.5 - ez);
}

__device__ inline void coarse_velocity(const float *c, int D, int H, int W, int ncz, int ncy, int ncx, d3 p, double u[3]) {
    const double q[3] = {p.z / 2.0 - 0.25, p.y / 2.0 - 0.25, p.x / 2.0 - 0.25};
    const int n[3] = {ncz, ncy, ncx};
    int i0[3], i1[3];
    double w[3];
    for (int d = 0; d < 3; ++d) {
        const double v = fmin(fmax(q[d], 0.0), n[d] - 1.0);
        i0[d] = int(floor(v));
        i1[d] = min(i0[d] + 1, n[d] - 1);
        w[d] = v - i0[d];
    }
    u[0] = u[1] = u[2] = 0.0;
    for (int j = 0; j < 8; ++j) {
        const int iz = (j >> 2) ? i1[0] : i0[0], iy = ((j >> 1) & 1) ? i1[1] : i0[1], ix = (j & 1) ? i1[2] : i0[2];
        const double wt = ((j >> 2) ? w[0] : 1.0 - w[0]) * (((j >> 1) & 1) ? w[1] : 1.0 - w[1]) * ((j & 1) ? w[2] : 1.0 - w[2]);
        const float *cc = c + ((int64_t(iz) * H + iy) * W + ix) * 8;
        for (int d = 0; d < 3; ++d) u[d] += wt * double(cc[2 + d]);
    }
}

__global__ void rod_jump_kernel(RodBatch bt, const float *c0, const float *c1, int D, int H, int W, double steps) {
    const RodArgs a = bt.all[0];
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n_rods) return;
    double *rod = a.rods + r * ROD_STRIDE;
    d3 X = ld3(rod + ROD_X);
    double ua[3], ub[3];
    coarse_velocity(c0, D, H, W, a.nz / 2, a.ny / 2, a.nx / 2, X, ua);
    coarse_velocity(c1, D, H, W, a.nz / 2, a.ny / 2, a.nx / 2, X, ub);
    const d3 V = mk(0.5 * (ua[0] + ub[0]), 0.5 * (ua[1] + ub[1]), 0.5 * (ua[2] + ub[2]));
    X = X + steps * V;
    if (a.px) X.x = X.x - a.nx * floor(X.x / a.nx);
    if (a.py) X.y = X.y - a.ny * floor(X.y / a.ny);
    if (a.pz) X.z = X.z - a.nz * floor(X.z / a.nz);
    if (!a.pz) X.z = clamp_ends(a, quat_axis(rod + ROD_Q), X.z);
    st3(rod + ROD_X, X);
    st3(rod + ROD_V, V);
}

// Rods over a jump from their own recent motion: each centre continues
// `factor` times the (minimum-image) displacement it made since x_prev, the
// centres one interval earlier ([n_rods][3]); kept one node off closed end
// planes like the advected jump.  Velocity, orientation and angular momentum
// are kept.
__global__ void rod_drift_kernel(RodBatch bt, const double *x_prev, double factor) {
    const RodArgs a = bt.all[0];
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n_rods) return;
    double *rod = a.rods + r * ROD_STRIDE;
    d3 X = ld3(rod + ROD_X);
    const d3 dX = min_image(X - ld3(x_prev + 3 * r), a);
    X = X + factor * dX;
    if (a.px) X.x = X.x - a.nx * floor(X.x / a.nx);
    if (a.py) X.y = X.y - a.ny * floor(X.y / a.ny);
    if (a.pz) X.z = X.z - a.nz * floor(X.z / a.nz);
    if (!a.pz) X.z = clamp_ends(a, quat_axis(rod + ROD_Q), X.z);
    st3(rod + ROD_X, X);
}

// Rods-only relaxation after the advection of a jump: overlaps the jump made
// (axis segments closer than the contact distance d0 of the excluded-volume
// potential, or an axis end closer than d0_wall to the wall) are removed by
// Jacobi projection, each rod of an overlapping pair moved half the deficit
// along the closest-point direction, orientation kept, until no deficit
// exceeds 1e-6 lattice units or RELAX_IT sweeps are done.  One work-group,
// thread r owns rod r; centres live in LDS.
constexpr int RELAX_IT = 200;

__global__ void __launch_bounds__(LB_MAX_RODS) rod_relax_kernel(RodBatch bt) {
    const RodArgs a = bt.all[0];
    extern __shared__ double rl[];  // [max_rods][6]: centre, axis
    __shared__ int busy;
    const int r = threadIdx.x, n = a.n_rods;
    const bool mine = r < n;
    d3 X = mk(0, 0, 0), e = mk(0, 0, 0);
    if (mine) {
        X = ld3(a.rods + r * ROD_STRIDE + ROD_X);
        e = quat_axis(a.rods + r * ROD_STRIDE + ROD_Q);
        st3(rl + 6 * r, X);
        st3(rl + 6 * r + 3, e);
    }
    const double reach = 2.0 * a.half + a.d0;  // centres farther apart never overlap
    for (int it = 0; it < RELAX_IT; ++it) {
        if (r == 0) busy = 0;
        __syncthreads();
        d3 push = mk(0, 0, 0);
        bool deficit = false;
        if (mine) {
            const d3 pa = X - a.half * e, qa = X + a.half * e;
            for (int s2 = 0; s2 < n; ++s2) {
                if (s2 == r) continue;
                const d3 Xs = ld3(rl + 6 * s2);
                const d3 dx = min_image(Xs - X, a);
                if (dot(dx, dx) >= reach * reach) continue;
                const d3 es = ld3(rl + 6 * s2 + 3);
                const d3 c = X + dx;  // image of s next to r
                d3 ca, cb;
                const double d = seg_seg(pa, qa, c - a.half * es, c + a.half * es, ca, cb);
                if (d >= a.d0 - 1e-6) continue;
                deficit = true;
                d3 nrm;
                if (d > 1e-9) {
                    nrm = (1.0 / d) * (ca - cb);
                } else {
                    const double l = sqrt(dot(dx, dx));
                    nrm = l > 1e-9 ? (-1.0 / l) * dx : mk(0, 0, r > s2 ? 1.0 : -1.0);
                }
                push = push + (0.5 * (a.d0 - d)) * nrm;
            }
            if (a.wall_on) {
                const double h = fmin(pa.z, qa.z) - a.wall_z;
                if (h < a.d0_wall - 1e-6) {
                    deficit = true;
                    push.z += a.d0_wall - h;
                }
            }
        }
        if (deficit) busy = 1;
        __syncthreads();
        const bool again = busy != 0;
        if (mine && again) {
            X = X + push;
            if (a.px) X.x = X.x - a.nx * floor(X.x / a.nx);
            if (a.py) X.y = X.y - a.ny * floor(X.y / a.ny);
            if (a.pz) X.z = X.z - a.nz * floor(X.z / a.nz);
            if (!a.pz) X.z = clamp_ends(a, e, X.z);
            st3(rl + 6 * r, X);
        }
        __syncthreads();
        if (!again) break;
    }
    if (mine) st3(a.rods + r * ROD_STRIDE + ROD_X, X);
}

// every rod node back to fluid, no rod ids (before a re-placement)
__global__ void unrod_kernel(uint8_t *mat, int16_t *rodid, int64_t n) {
    for (int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; p < n; p += int64_t(gridDim.x) * blockDim.x) {
        if ((mat[p] & MAT_ID_MASK) == MAT_ROD) mat[p] = MAT_FLUID;
        rodid[p] = -1;
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <class F>
static hipError_t rods_by_prec(int prec, F &&fn) {
    switch (prec) {
        case LB_F64:
            return fn(static_cast<double *>(nullptr));
        case LB_F32:
            return fn(static_cast<float *>(nullptr));
        case LB_F16DEV:
            return fn(static_cast<_Float16 *>(nullptr));
        case LB_BF16DEV:
            return fn(static_cast<bf16_t *>(nullptr));
        default:
            return hipErrorInvalidValue;
    }
}

static int fill_grid(int64_t n) {
    int64_t g = (n + 255) / 256;
    return int(g > 8192 ? 8192 : (g < 1 ? 1 : g));
}

hipError_t launch_rods_place(int prec, const RodArgs &a, const RodBatch &bt, hipStream_t s) {
    if (a.n_rods == 0) return hipSuccess;
    const int64_t n = int64_t(a.nx) * a.ny * a.nz;
    const dim3 grid(a.nblk, a.n_rods);
    hipLaunchKernelGGL(fill_i32_kernel, dim3(fill_grid(n)), dim3(256), 0, s, a.newid, n, -1);
    hipLaunchKernelGGL(rod_mask_kernel, dim3(2 * a.n_rods), dim3(MB), 0, s, bt);
    return rods_by_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(rod_update_kernel<S>, grid, dim3(RB), 0, s, bt, 1);
        hipLaunchKernelGGL((rod_link_kernel<S, true>), grid, dim3(RB), 0, s, bt, 1);
        return hipGetLastError();
    });
}

hipError_t launch_rods_jump(const RodArgs &a, const RodBatch &bt, const float *c0, const float *c1, int D, int H, int W,
                            double steps, hipStream_t s) {
    if (a.n_rods == 0) return hipSuccess;
    const int64_t n = int64_t(a.nx) * a.ny * a.nz;
    hipLaunchKernelGGL(rod_jump_kernel, dim3((a.n_rods + 63) / 64), dim3(64), 0, s, bt, c0, c1, D, H, W, steps);
    hipLaunchKernelGGL(rod_relax_kernel, dim3(1), dim3(LB_MAX_RODS), size_t(a.n_rods) * 6 * sizeof(double), s, bt);
    hipLaunchKernelGGL(unrod_kernel, dim3(fill_grid(n)), dim3(256), 0, s, a.mat, a.rodid, n);
    return hipGetLastError();
}

hipError_t launch_rods_drift(const RodArgs &a, const RodBatch &bt, const double *x_prev, double factor, hipStream_t s) {
    if (a.n_rods == 0) return hipSuccess;
    const int64_t n = int64_t(a.nx) * a.ny * a.nz;
    hipLaunchKernelGGL(rod_drift_kernel, dim3((a.n_rods + 63) / 64), dim3(64), 0, s, bt, x_prev, factor);
    hipLaunchKernelGGL(rod_relax_kernel, dim3(1), dim3(LB_MAX_RODS), size_t(a.n_rods) * 6 * sizeof(double), s, bt);
    hipLaunchKernelGGL(unrod_kernel, dim3(fill_grid(n)), dim3(256), 0, s, a.mat, a.rodid, n);
    return hipGetLastError();
}

hipError_t launch_rods_link(int prec, const RodArgs &a, const RodBatch &bt, hipStream_t s) {
    if (a.n_rods == 0) return hipSuccess;
    const dim3 grid(a.nblk, a.n_rods);
    return rods_by_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL((rod_link_kernel<S, false>), grid, dim3(RB), 0, s, bt, 0);
        return hipGetLastError();
    });
}

hipError_t launch_rods_sums(const RodArgs &a, double *out, hipStream_t s) {
    hipLaunchKernelGGL(rod_sums_kernel, dim3(1), dim3(64), 0, s, a, out);
    return hipGetLastError();
}

hipError_t launch_rods_step(int prec, const RodBatch &bt, int n_lat, int total_rods, int nblk_max, int max_rods,
                            hipStream_t s) {
    if (total_rods == 0) return hipSuccess;
    const dim3 grid(nblk_max, total_rods);
    return rods_by_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(rod_adhesion_kernel<S>, grid, dim3(RB), 0, s, bt);
        hipLaunchKernelGGL(rod_integrate_kernel, dim3(n_lat), dim3(LB_MAX_RODS), size_t(max_rods) * RS_N * sizeof(double),
                           s, bt);
        // the re-mask, with one work-group per rod more for the neighbour lists
        hipLaunchKernelGGL(rod_mask_kernel, dim3(2 * total_rods), dim3(MB), 0, s, bt);
        hipLaunchKernelGGL(rod_update_kernel<S>, grid, dim3(RB), 0, s, bt, 0);
        hipLaunchKernelGGL((rod_link_kernel<S, true>), grid, dim3(RB), 0, s, bt, 0);
        return hipGetLastError();
    });
}

}  // namespace lbm
