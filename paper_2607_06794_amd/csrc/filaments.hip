// Bead-spring filaments coupled to the Shan-Chen fluid (gfx950).
//
// The paper's nanowires (Methods, filament paragraphs): chains of beads with
// FENE bonds (Eq. 9), excluded volume between all beads (Eq. 10), harmonic
// springs between second neighbours for stiffness (Eq. 11), Lennard-Jones
// cohesion between filaments (Eq. 12), substrate adhesion and load-dependent
// friction, a drag towards the local fluid velocity whose momentum goes back
// to the fluid, a solvation force along the colour gradient, and five bead
// substeps per lattice step.
//
// One filament update, after the fluid step, in five launches:
//   gather   eight lanes per bead: the eight lattice nodes around the bead,
//            their trilinear weights renormalised over fluid nodes, the
//            physical velocity (sum_k j*_k - F/2) / rho and the colour
//            gradient 3 sum_i w_i C(x + c_i) c_i of each node, interpolated;
//   list     one wavefront per bead: non-bonded partners within the
//            interaction range plus a skin, in ascending index order;
//   substeps one launch per substep, one thread per bead: forces from the
//            previous substep's positions, then V and X into the other
//            position slot of the bead record; the impulse the fluid
//            receives summed per bead;
//   spread   one thread per bead adds its impulse times each weight into a
//            fixed-point (2^-50) momentum grid with 64-bit integer atomics:
//            integer addition is exact, so the sums do not depend on order;
//   apply    one thread per (bead, stencil node): the node's owner (the
//            lowest such index, recorded by the spread pass) adds its summed momentum dp to the stored state by the
//            exact-difference rule f*_k += f^eq(rho_k, u_k + dp / rho) -
//            f^eq(rho_k, u_k), which keeps every density and adds dp exactly.
// All bead arithmetic is FP64.
#include <type_traits>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

namespace {

constexpr double FIX_SCALE = FIL_FIX;
constexpr double FIX_INV = 1.0 / FIX_SCALE;

struct v3 {
    double x, y, z;
};
__device__ inline v3 operator+(v3 a, v3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline v3 operator-(v3 a, v3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline v3 operator*(double s, v3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline v3 ld(const double *p) { return {p[0], p[1], p[2]}; }
__device__ inline void st(double *p, v3 v) {
    p[0] = v.x;
    p[1] = v.y;
    p[2] = v.z;
}

__device__ inline double wrap_pos(double x, double box, int per) {
    if (!per) return x;
    // remainder with the sign of the box: fmod, then one shift of negatives
    double r = fmod(x, box);
    if (r != 0.0 && r < 0.0) r += box;
    return r;
}
__device__ inline double min_img(double d, double box, int per) { return per ? d - box * rint(d / box) : d; }
__device__ inline v3 min_image(v3 d, const FilArgs &a) {
    return {min_img(d.x, a.nx, a.px), min_img(d.y, a.ny, a.py), min_img(d.z, a.nz, a.pz)};
}

__device__ inline int wrap_idx(int i, int n) { return ((i % n) + n) % n; }

template <class S>
__device__ inline double popf(const FilArgs &a, const S *f, int k, int i, int64_t n) {
    return static_cast<double>(Codec<S>::dec(f[(int64_t(k) * Q + i) * a.fs + n])) + wgt<double>(i) * a.rho_ref[k];
}

// densities of fluid node n: the density array while it holds the current
// state, else the sum of the populations
template <class S>
__device__ inline void node_rho(const FilArgs &a, const S *f, int64_t n, double rho[2]) {
    if (a.rho_fresh) {
        const typename Codec<S>::C *ro = static_cast<const typename Codec<S>::C *>(a.rho);
        rho[0] = double(ro[n]);
        rho[1] = double(ro[a.fs + n]);
        return;
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) s += popf(a, f, k, i, n);
        rho[k] = s;
    }
}

__device__ inline int64_t node_at(const FilArgs &a, int x, int y, int z) {
    return (int64_t(z) * a.ny + y) * a.nx + x;
}

// neighbour x + c_i of an interior fluid node (closed directions end in
// non-fluid planes, so the neighbour of a fluid node exists)
__device__ inline int64_t nb_of(const FilArgs &a, int x, int y, int z, int i) {
    const int xn = a.px ? wrap_idx(x + cx(i), a.nx) : x + cx(i);
    const int yn = a.py ? wrap_idx(y + cy(i), a.ny) : y + cy(i);
    const int zn = a.pz ? wrap_idx(z + cz(i), a.nz) : z + cz(i);
    return node_at(a, xn, yn, zn);
}

// physical velocity and colour gradient of fluid node (x, y, z)
template <class S>
__device__ void node_fields(const FilArgs &a, const S *f, int x, int y, int z, v3 &u, v3 &gc) {
    const int64_t n = node_at(a, x, y, z);
    double rho[2];
    node_rho(a, f, n, rho);
    // post-collision momentum of both components
    v3 jk[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        jk[k] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const double fi = popf(a, f, k, i, n);
            jk[k] = jk[k] + v3{cx(i) * fi, cy(i) * fi, cz(i) * fi};
        }
    }
    const v3 js = jk[0] + jk[1];
    const double tot = rho[0] + rho[1];
    const double ts = tot > 0.0 ? tot : 1.0;
    const double C0 = (rho[0] - rho[1]) / ts;
    // Shan-Chen force of the stored densities and the lattice colour gradient;
    // the neighbours' materials and stored densities are loaded together (the
    // density array exists on every lattice with filaments; it is used only
    // while it holds the current state)
    uint8_t idn[Q];
    double pn[Q][2];
    {
        const auto *ro = static_cast<const typename Codec<S>::C *>(a.rho);
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int64_t m = nb_of(a, x, y, z, i);
            idn[i] = a.mat[m] & MAT_ID_MASK;
            pn[i][0] = double(ro[m]);
            pn[i][1] = double(ro[a.fs + m]);
        }
    }
    v3 s[2] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    v3 g = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const uint8_t id = idn[i];
        double psi[2], Cn;
        if (id == MAT_FLUID) {
            if (a.rho_fresh) {
                psi[0] = pn[i][0];
                psi[1] = pn[i][1];
            } else {
                node_rho(a, f, nb_of(a, x, y, z, i), psi);
            }
            const double tn = psi[0] + psi[1];
            Cn = (psi[0] - psi[1]) / (tn > 0.0 ? tn : 1.0);
        } else {
            if (id == MAT_GHOST) {
                psi[0] = a.rho_top[0];
                psi[1] = a.rho_top[1];
            } else {
                psi[0] = a.psi_tab[2 * id];
                psi[1] = a.psi_tab[2 * id + 1];
            }
            Cn = C0;
        }
        const double w = wgt<double>(i);
        const v3 c = {double(cx(i)), double(cy(i)), double(cz(i))};
        s[0] = s[0] + (w * psi[1]) * c;  // partner of component A is B
        s[1] = s[1] + (w * psi[0]) * c;
        g = g + (3.0 * w * Cn) * c;
    }
    v3 F = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double gp = -a.G * rho[k];
        F = F + v3{gp * s[k].x + rho[k] * a.g[0], gp * s[k].y + rho[k] * a.g[1], gp * s[k].z + rho[k] * a.g[2]};
    }
    u = {(js.x - 0.5 * F.x) / ts, (js.y - 0.5 * F.y) / ts, (js.z - 0.5 * F.z) / ts};
    gc = g;
}

// ---------------------------------------------------------------------------
// 1. gather: eight lanes per bead, one per stencil node; the weights and the
//    interpolated fields are summed in stencil order through lane shuffles
// ---------------------------------------------------------------------------
template <class S>
__global__ __launch_bounds__(256) void fil_gather_kernel(FilArgs a) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = t >> 3, e = t & 7;
    const int lane0 = (threadIdx.x & 63) & ~7;  // first lane of this bead's group
    const bool act = b < a.n;
    const S *f = static_cast<const S *>(a.f);
    double *rec = a.bead + size_t(act ? b : 0) * FIL_STRIDE;
    const v3 X = ld(rec + FIL_X);
    const double bx = floor(X.x), by = floor(X.y), bz = floor(X.z);
    const double fr[3] = {X.x - bx, X.y - by, X.z - bz};
    const int base[3] = {int(bx), int(by), int(bz)};
    const int dims[3] = {a.nx, a.ny, a.nz}, per[3] = {a.px, a.py, a.pz};
    const int d[3] = {e & 1, (e >> 1) & 1, e >> 2};
    int idx[3];
    bool ok = act;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        idx[q] = base[q] + d[q];
        if (per[q])
            idx[q] = wrap_idx(idx[q], dims[q]);
        else if (idx[q] < 0 || idx[q] >= dims[q])
            ok = false;
    }
    int node = -1;
    double w = 0.0;
    if (ok) {
        const int64_t n = node_at(a, idx[0], idx[1], idx[2]);
        if ((a.mat[n] & MAT_ID_MASK) == MAT_FLUID) {
            node = int(n);
            w = (d[0] ? fr[0] : 1.0 - fr[0]) * (d[1] ? fr[1] : 1.0 - fr[1]) * (d[2] ? fr[2] : 1.0 - fr[2]);
        }
    }
    double wsum = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) wsum += __shfl(w, lane0 + q, 64);
    const int coupled = wsum > 0.0;
    v3 u = {0.0, 0.0, 0.0}, g = {0.0, 0.0, 0.0};
    if (coupled && node >= 0) {
        w = w / wsum;
        const int64_t n = node;
        const uint32_t un = static_cast<uint32_t>(n), row = un / uint32_t(a.nx);
        node_fields(a, f, int(un - row * uint32_t(a.nx)), int(row % uint32_t(a.ny)), int(row / uint32_t(a.ny)), u, g);
    } else {
        node = -1;
        w = 0.0;
    }
    v3 ub = {0.0, 0.0, 0.0}, gb = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const double wq = __shfl(w, lane0 + q, 64);
        const v3 uq = {__shfl(u.x, lane0 + q, 64), __shfl(u.y, lane0 + q, 64), __shfl(u.z, lane0 + q, 64)};
        const v3 gq = {__shfl(g.x, lane0 + q, 64), __shfl(g.y, lane0 + q, 64), __shfl(g.z, lane0 + q, 64)};
        ub = ub + wq * uq;
        gb = gb + wq * gq;
    }
    if (!act) return;
    rec[FIL_W + e] = w;
    a.sten[size_t(b) * 8 + e] = node;
    if (e == 0) {
        st(rec + FIL_U, ub);
        st(rec + FIL_GC, gb);
        rec[FIL_COUPLED] = coupled;
    }
}

// ---------------------------------------------------------------------------
// 2. non-bonded partner lists: every other bead within the range plus the
//    skin, except the chain's own beads at most two apart (their forces are
//    the bonded ones).  One wavefront per bead scans the candidates 64 at a
//    time and appends the hits in ascending order (ballot and prefix count).
// ---------------------------------------------------------------------------
constexpr int LT = 256;

__global__ __launch_bounds__(LT) void fil_list_kernel(FilArgs a, double range2) {
    const int b = blockIdx.x * (LT / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= a.n) return;  // uniform per wavefront
    double *rec = a.bead + size_t(b) * FIL_STRIDE;
    const v3 X = ld(rec + FIL_X);
    if (lane == 0) st(rec + FIL_X0, X);
    const int cb = b / a.per_chain, ib = b % a.per_chain;
    int cnt = 0;
    for (int o0 = 0; o0 < a.n; o0 += 64) {
        const int o = o0 + lane;
        bool hit = false;
        if (o < a.n && o != b && !(o / a.per_chain == cb && abs(o % a.per_chain - ib) <= 2)) {
            const v3 r = min_image(X - ld(a.bead + size_t(o) * FIL_STRIDE + FIL_X), a);
            hit = r.x * r.x + r.y * r.y + r.z * r.z < range2;
        }
        const unsigned long long m = __ballot(hit);
        const int pos = cnt + __popcll(m & ((1ull << lane) - 1ull));
        if (hit && pos < FIL_NBR) a.nbr[size_t(b) * FIL_NBR + pos] = o;
        cnt += __popcll(m);
    }
    if (lane == 0) {
        if (cnt > FIL_NBR) {
            atomicOr(a.status, ST_ROD_LIST);
            cnt = FIL_NBR;
        }
        a.nbr_cnt[b] = cnt;
    }
}

// ---------------------------------------------------------------------------
// 3. one substep per launch, one thread per bead: forces from the positions
//    of the previous substep (src), then V and X (dst), the two position
//    slots of each bead record alternating
// ---------------------------------------------------------------------------
__device__ inline double phi_d(double d, double d0) {
    // d/dd of (d0/d)^12 - 2 (d0/d)^6
    const double q = d0 / d;
    const double q2 = q * q;
    const double x6 = q2 * q2 * q2;
    return 12.0 * (x6 - x6 * x6) / d;
}

__device__ inline double wca_f(double d, const FilArgs &a) { return d <= a.d0 ? -a.eps * phi_d(d, a.d0) : 0.0; }
__device__ inline double fene_f(double d, const FilArgs &a) {
    const double q = d / a.R_m;
    return -a.k_s * d / (1.0 - q * q);
}
__device__ inline double bend_f(double d, const FilArgs &a) { return -a.k_b * (d - 2.0 * a.d0); }
__device__ inline double coh_f(double d, const FilArgs &a) {
    return (a.eps_coh > 0.0 && d > a.d0 && d < a.r_cut) ? -a.eps_coh * phi_d(d, a.d0) : 0.0;
}
__device__ inline double sub_f(double h, const FilArgs &a) {
    return (h > 0.0 && h < a.r_cut_s) ? -a.eps_s * phi_d(h, a.sigma_s) : 0.0;
}

constexpr int ST_TPB = 64;
constexpr int ST_LPB = 8;  // lanes per bead: each takes every eighth partner

__global__ __launch_bounds__(ST_TPB) void fil_substep_kernel(FilArgs a, int src, int first) {
    const int b = (blockIdx.x * ST_TPB + threadIdx.x) / ST_LPB;
    const int ln = threadIdx.x % ST_LPB;
    if (b >= a.n) return;  // uniform per group of ST_LPB lanes (n beads fill whole groups or none)
    const int dst = src == FIL_X ? FIL_XN : FIL_X;
    double *rec = a.bead + size_t(b) * FIL_STRIDE;
    const double dt = 1.0 / a.n_sub;
    const double m = a.mass;
    unsigned flags = 0;
    const v3 X = ld(rec + src);
    const int ch = b / a.per_chain, ib = b % a.per_chain;
    v3 Fi = {0.0, 0.0, 0.0};
    auto pair = [&](v3 Xo, int kind) {
        const v3 r = min_image(X - Xo, a);
        const double d = sqrt(r.x * r.x + r.y * r.y + r.z * r.z);
        double fm = 0.0;
        if (d <= a.d0) fm += wca_f(d, a);
        if (kind == 1) {
            fm += fene_f(d, a);
            if (!(d < a.R_m)) flags |= ST_ROD;
        }
        if (kind == 2) fm += bend_f(d, a);
        if (kind == 3) fm += coh_f(d, a);
        if (fm != 0.0) Fi = Fi + v3{fm * r.x / d, fm * r.y / d, fm * r.z / d};
    };
    // the partners are split over the bead's lanes: lane j takes the bonded
    // partner j (at most four: the chain's beads up to two apart) and the
    // listed partners j, j + 8, ...; the lanes' sums are added with a fixed
    // xor butterfly
    {
        int cnt = 0;
#pragma unroll
        for (int dj = -2; dj <= 2; ++dj) {
            const int j = ib + dj;
            if (dj == 0 || j < 0 || j >= a.per_chain) continue;
            if (cnt == ln) pair(ld(a.bead + size_t(ch * a.per_chain + j) * FIL_STRIDE + src), (dj == -1 || dj == 1) ? 1 : 2);
            ++cnt;
        }
    }
    const int nc = a.nbr_cnt[b];
    for (int q0 = ln; q0 < nc; q0 += 2 * ST_LPB) {
        // two partners per lane and iteration, their loads in flight together
        const int o0 = a.nbr[size_t(b) * FIL_NBR + q0];
        const int q1 = q0 + ST_LPB;
        const int o1 = q1 < nc ? a.nbr[size_t(b) * FIL_NBR + q1] : o0;
        const v3 X0 = ld(a.bead + size_t(o0) * FIL_STRIDE + src), X1 = ld(a.bead + size_t(o1) * FIL_STRIDE + src);
        pair(X0, o0 / a.per_chain == ch ? 0 : 3);
        if (q1 < nc) pair(X1, o1 / a.per_chain == ch ? 0 : 3);
    }
#pragma unroll
    for (int o = 1; o < ST_LPB; o <<= 1) {
        Fi.x += __shfl_xor(Fi.x, o, 64);
        Fi.y += __shfl_xor(Fi.y, o, 64);
        Fi.z += __shfl_xor(Fi.z, o, 64);
    }
    flags |= __shfl_xor(flags, 1, 64) | __shfl_xor(flags, 2, 64) | __shfl_xor(flags, 4, 64);
    if (ln != 0) return;
    if (first) st(rec + FIL_IMP, v3{0.0, 0.0, 0.0});
    v3 Fs = {0.0, 0.0, 0.0};
    const double h = X.z - a.wall_z;
    if (a.wall_on) Fs.z = sub_f(h, a);
    const int coupled = rec[FIL_COUPLED] != 0.0;
    const v3 V = ld(rec + FIL_V);
    const v3 U = ld(rec + FIL_U);
    const v3 Fd = coupled ? (-a.gamma) * (V - U) : v3{0.0, 0.0, 0.0};
    const v3 Fsv = coupled ? a.kappa_s * ld(rec + FIL_GC) : v3{0.0, 0.0, 0.0};
    const v3 Fo = (Fi + Fd) + Fsv;
    v3 Ff = {0.0, 0.0, 0.0};
    if (a.wall_on && h > 0.0 && h < a.r_cut_s) {
        const double fz = Fo.z + fmin(Fs.z, 0.0);
        const double N = fmax(0.0, -fz);
        const double sv = sqrt(V.x * V.x + V.y * V.y);
        if (N > 0.0 && sv > 0.0) {
            const double c = fmin(a.mu * N / sv, m / dt);
            Ff = {-V.x * c, -V.y * c, 0.0};
        }
    }
    const v3 imp = ld(rec + FIL_IMP);
    st(rec + FIL_IMP, imp + dt * ((-1.0) * (Fd + Fsv)));
    // symplectic Euler: V first, X with the new V
    const v3 acc = (Fo + Fs) + Ff;
    const v3 Vn = {V.x + acc.x / m * dt, V.y + acc.y / m * dt, V.z + acc.z / m * dt};
    st(rec + FIL_V, Vn);
    const v3 Xp = {X.x + Vn.x * dt, X.y + Vn.y * dt, X.z + Vn.z * dt};
    st(rec + dst, v3{wrap_pos(Xp.x, a.nx, a.px), wrap_pos(Xp.y, a.ny, a.py), wrap_pos(Xp.z, a.nz, a.pz)});
    if (flags) atomicOr(a.status, flags);
}

// ---------------------------------------------------------------------------
// 4. spread the impulses onto the fixed-point momentum grid
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void fil_spread_kernel(FilArgs a, int last) {
    // eight lanes per bead, lane e on stencil node e; each node's owner for
    // the apply pass is the lowest (bead, e) index that touches it
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = t / 8, e = t % 8;
    if (b >= a.n) return;
    double *rec = a.bead + size_t(b) * FIL_STRIDE;
    if (e == 0) {
        // the last substep's positions become the bead's position; the
        // partner lists hold for moves below half the skin per update
        const v3 X = ld(rec + last);
        if (last != FIL_X) st(rec + FIL_X, X);
        const v3 dd = min_image(X - ld(rec + FIL_X0), a);
        unsigned flags = 0;
        if (dd.x * dd.x + dd.y * dd.y + dd.z * dd.z > 0.25 * a.skin * a.skin) flags |= ST_ROD;
        if (!(X.x == X.x && X.y == X.y && X.z == X.z)) flags |= ST_NAN;
        if (flags) atomicOr(a.status, flags);
    }
    if (rec[FIL_COUPLED] == 0.0) return;
    const int n = a.sten[t];
    if (n < 0) return;
    const double w = rec[FIL_W + e];
    for (int d = 0; d < 3; ++d) {
        const long long q = llrint(w * rec[FIL_IMP + d] * FIX_SCALE);
        atomicAdd(reinterpret_cast<unsigned long long *>(a.grid + int64_t(d) * a.fs + n), static_cast<unsigned long long>(q));
    }
    atomicMin(a.claim + n, t);
}

// ---------------------------------------------------------------------------
// 5. apply the summed momentum by the exact-difference rule
// ---------------------------------------------------------------------------
__device__ inline double feq_i(int i, double rho, v3 u) {
    const double cu = cx(i) * u.x + cy(i) * u.y + cz(i) * u.z;
    const double usq = u.x * u.x + u.y * u.y + u.z * u.z;
    return wgt<double>(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
}

template <class S>
__global__ __launch_bounds__(256) void fil_apply_kernel(FilArgs a) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n * 8) return;
    const int n = a.sten[t];
    if (n < 0) return;
    // only the node's owner (set by the spread pass) applies it, then returns
    // the owner slot and the node's sums to their empty values
    if (a.claim[n] != t) return;
    a.claim[n] = FIL_NO_OWNER;
    long long *g = a.grid;
    const v3 dp = {double(g[n]) * FIX_INV, double(g[a.fs + n]) * FIX_INV, double(g[2 * a.fs + n]) * FIX_INV};
    g[n] = 0;
    g[a.fs + n] = 0;
    g[2 * a.fs + n] = 0;
    S *f = static_cast<S *>(a.f);
    // the node's 38 populations, all loaded before any store (a store through
    // f would otherwise order every later load behind it)
    double fv[2][Q];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int i = 0; i < Q; ++i) fv[k][i] = popf(a, f, k, i, n);
    double rho[2];
    v3 uk[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        double r = 0.0;
        v3 j = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            r += fv[k][i];
            j = j + v3{cx(i) * fv[k][i], cy(i) * fv[k][i], cz(i) * fv[k][i]};
        }
        rho[k] = r;
        uk[k] = r > 0.0 ? v3{j.x / r, j.y / r, j.z / r} : v3{0.0, 0.0, 0.0};
    }
    const double tot = rho[0] + rho[1];
    if (!(tot > 0.0)) return;
    const v3 du = {dp.x / tot, dp.y / tot, dp.z / tot};
    // a node next to a static wall has already handed f*_j to the wall node
    // x + c_j as direction opp(j) (halfway bounce-back of the next pull): the
    // updated value goes there too (the 18 neighbours' materials loaded together)
    const bool near_wall = (a.mat[n] & MAT_NEAR_WALL) != 0;
    const uint32_t un32 = static_cast<uint32_t>(n), row = un32 / uint32_t(a.nx);
    const int x = int(un32 - row * uint32_t(a.nx)), y = int(row % uint32_t(a.ny)), z = int(row / uint32_t(a.ny));
    uint32_t walls = 0;
    if (near_wall) {
        uint8_t mq[Q];
#pragma unroll
        for (int i = 1; i < Q; ++i) mq[i] = a.mat[nb_of(a, x, y, z, i)];
#pragma unroll
        for (int i = 1; i < Q; ++i) walls |= is_static_wall(mq[i] & MAT_ID_MASK) ? 1u << i : 0u;
    }
    // the plane below the reservoir booked the outflow of its stored f* when
    // the fluid step wrote it; the change of that outflow goes to the ledger
    const bool top = a.evap && z == a.nz - 2;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (!(rho[k] > 0.0)) continue;
        const v3 un = uk[k] + du;
        double dout = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int64_t idx = (int64_t(k) * Q + i) * a.fs + n;
            const double v = fv[k][i] + (feq_i(i, rho[k], un) - feq_i(i, rho[k], uk[k]));
            const S sv = Codec<S>::enc(static_cast<typename Codec<S>::C>(v - wgt<double>(i) * a.rho_ref[k]));
            f[idx] = sv;
            // the stored value as the next read of it decodes it
            if (top && cz(i) == 1) dout += (static_cast<double>(Codec<S>::dec(sv)) + wgt<double>(i) * a.rho_ref[k]) - fv[k][i];
            if ((walls >> i) & 1u) f[(int64_t(k) * Q + opp(i)) * a.fs + nb_of(a, x, y, z, i)] = sv;
        }
        if (top && dout != 0.0)
            atomicAdd(reinterpret_cast<unsigned long long *>(a.led + k),
                      static_cast<unsigned long long>(llrint(dout * FIX_SCALE)));
    }
}

template <class F>
static hipError_t fil_by_prec(int prec, F &&fn) {
    switch (prec) {
        case LB_F64:
            return fn(static_cast<double *>(nullptr));
        case LB_F32:
            return fn(static_cast<float *>(nullptr));
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_fil_step(int prec, const FilArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    double range = a.d0;
    if (a.eps_coh > 0.0 && a.r_cut > range) range = a.r_cut;
    range += a.skin;
    return fil_by_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(fil_gather_kernel<S>, dim3((a.n * 8 + 255) / 256), dim3(256), 0, s, a);
        hipLaunchKernelGGL(fil_list_kernel, dim3((a.n + LT / 64 - 1) / (LT / 64)), dim3(LT), 0, s, a, range * range);
        int src = FIL_X;
        for (int sub = 0; sub < a.n_sub; ++sub) {
            hipLaunchKernelGGL(fil_substep_kernel, dim3((a.n * ST_LPB + ST_TPB - 1) / ST_TPB), dim3(ST_TPB), 0, s, a,
                               src, sub == 0 ? 1 : 0);
            src = src == FIL_X ? FIL_XN : FIL_X;
        }
        hipLaunchKernelGGL(fil_spread_kernel, dim3((a.n * 8 + 255) / 256), dim3(256), 0, s, a, src);
        hipLaunchKernelGGL(fil_apply_kernel<S>, dim3((a.n * 8 + 255) / 256), dim3(256), 0, s, a);
        return hipGetLastError();
    });
}

}  // namespace lbm
