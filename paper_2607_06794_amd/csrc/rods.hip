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
// Work decomposition: every per-rod pass runs one work-group per rod over the
// rod's bounding box, and every per-rod sum is a fixed-order block reduction,
// so results do not depend on scheduling.  The integrator is one work-group
// with one thread per rod; each thread sums the pair forces on its own rod.
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
__device__ inline double pair_force(double d, const RodArgs &a) {
    double f = 0.0;
    if (d <= a.d0) f -= a.eps_rep * ljf_d(d, a.d0);
    if (a.eps_att > 0.0 && d > a.d0 && d < a.r_cut) f -= a.eps_att * ljf_d(d, a.d0);
    return f;
}

// closest points of segments [p1, q1], [p2, q2]: stationary point of the
// squared distance if interior, else the best of the four clamped edges
__device__ inline double seg_seg(d3 p1, d3 q1, d3 p2, d3 q2, d3 &c1, d3 &c2) {
    const d3 d1 = q1 - p1, d2 = q2 - p2, r = p1 - p2;
    const double aa = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r), c = dot(d1, r), b = dot(d1, d2);
    double best = 1e300;
    auto tryst = [&](double s, double t) {
        const d3 x1 = p1 + s * d1, x2 = p2 + t * d2;
        const d3 dd = x1 - x2;
        const double v = sqrt(dot(dd, dd));
        if (v < best) {
            best = v;
            c1 = x1;
            c2 = x2;
        }
    };
    const double den = aa * e - b * b;
    if (den > 1e-14 * fmax(aa * e, 1e-300)) {
        const double s = (b * f - c * e) / den, t = (aa * f - b * c) / den;
        if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0) tryst(s, t);
    }
    for (int k = 0; k < 2; ++k) {
        const double s = k;
        const double t = e == 0.0 ? 0.0 : fmin(fmax((b * s + f) / e, 0.0), 1.0);
        tryst(s, t);
    }
    for (int k = 0; k < 2; ++k) {
        const double t = k;
        const double s = aa == 0.0 ? 0.0 : fmin(fmax((b * t - c) / aa, 0.0), 1.0);
        tryst(s, t);
    }
    return best;
}

template <class S>
__device__ inline double decf(const S *f, int64_t idx) {
    return static_cast<double>(Codec<S>::dec(f[idx]));
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
        b.lo[d] = static_cast<int>(floor(c[d] - ext[d])) - margin;
        b.hi[d] = static_cast<int>(ceil(c[d] + ext[d])) + margin;
        // never visit a node twice through the periodic wrap
        if (per[d] && b.hi[d] - b.lo[d] + 1 > n[d]) b.hi[d] = b.lo[d] + n[d] - 1;
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

__device__ inline bool inside_capsule(const double *rod, d3 p, const RodArgs &a) {
    const d3 d = min_image(p - ld3(rod + ROD_X), a);
    const d3 e = quat_axis(rod + ROD_Q);
    const double t = fmin(fmax(dot(d, e), -a.half), a.half);
    const d3 c = d - t * e;
    return dot(c, c) <= a.radius * a.radius;
}

__device__ inline double block_sum_d(double v, double *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < int(blockDim.x >> 6); ++q) s += sh[q];
    __syncthreads();
    return s;
}

constexpr int RB = 256;  // threads per per-rod work-group

}  // namespace

// ---------------------------------------------------------------------------
// 1. reaction to the adhesion force: for fluid x next to rod node y = x + c_i,
//    F_rod += G psi_k(x) w_i psi^s_kbar c_i (psi_k(x) = rho_k(x), the collision
//    invariant of the current post-collision state), torque about X at y
// ---------------------------------------------------------------------------
template <class S>
__global__ void __launch_bounds__(RB) rod_adhesion_kernel(RodArgs a, const S *f) {
    __shared__ double sh[RB / 64];
    double *rod = a.rods + blockIdx.x * ROD_STRIDE;
    const Box b = rod_box(rod, a, 1);
    const int ex = b.hi[0] - b.lo[0] + 1, ey = b.hi[1] - b.lo[1] + 1, ez = b.hi[2] - b.lo[2] + 1;
    const int64_t nbox = int64_t(ex) * ey * ez;
    const int r = blockIdx.x;
    const d3 X = ld3(rod + ROD_X);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t m = threadIdx.x; m < nbox; m += RB) {
        int x = b.lo[0] + int(m % ex), y = b.lo[1] + int((m / ex) % ey), z = b.lo[2] + int(m / (int64_t(ex) * ey));
        const double px = x, py = y, pz = z;  // unwrapped position near the rod
        if (!wrap_coord(x, a.nx, a.px) || !wrap_coord(y, a.ny, a.py) || !wrap_coord(z, a.nz, a.pz)) continue;
        const int64_t n = (int64_t(z) * a.ny + y) * a.nx + x;
        if ((a.mat[n] & MAT_ID_MASK) != MAT_FLUID) continue;
        bool any = false;
        for (int i = 1; i < Q; ++i) {
            int xx = x + cx(i), yy = y + cy(i), zz = z + cz(i);
            if (!wrap_coord(xx, a.nx, a.px) || !wrap_coord(yy, a.ny, a.py) || !wrap_coord(zz, a.nz, a.pz)) continue;
            any |= a.rodid[(int64_t(zz) * a.ny + yy) * a.nx + xx] == r;
        }
        if (!any) continue;
        double rho[2];
        for (int k = 0; k < 2; ++k) {
            double s = 0.0;
            for (int j = 0; j < Q; ++j) s += decf(f, (k * Q + j) * a.fs + n) + wgt<double>(j) * a.rho_ref[k];
            rho[k] = s;
        }
        for (int i = 1; i < Q; ++i) {
            int xx = x + cx(i), yy = y + cy(i), zz = z + cz(i);
            if (!wrap_coord(xx, a.nx, a.px) || !wrap_coord(yy, a.ny, a.py) || !wrap_coord(zz, a.nz, a.pz)) continue;
            if (a.rodid[(int64_t(zz) * a.ny + yy) * a.nx + xx] != r) continue;
            const double g = a.G * wgt<double>(i) * (rho[0] * a.psi_rod[1] + rho[1] * a.psi_rod[0]);
            const d3 fr = mk(g * cx(i), g * cy(i), g * cz(i));
            const d3 arm = min_image(mk(px + cx(i), py + cy(i), pz + cz(i)) - X, a);
            const d3 tq = cross(arm, fr);
            acc[0] += fr.x;
            acc[1] += fr.y;
            acc[2] += fr.z;
            acc[3] += tq.x;
            acc[4] += tq.y;
            acc[5] += tq.z;
        }
    }
    for (int q = 0; q < 6; ++q) {
        const double v = block_sum_d(acc[q], sh);
        if (threadIdx.x == 0) rod[ROD_FA + q] = v;
    }
    if (threadIdx.x == 0) {
        // the slots filled by the last link pass have now been streamed: book their mass
        rod[ROD_SOLID] += rod[ROD_PEND];
        rod[ROD_SOLID + 1] += rod[ROD_PEND + 1];
        rod[ROD_PEND] = 0.0;
        rod[ROD_PEND + 1] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// 2. rigid-body substeps (one work-group, one thread per rod)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) rod_integrate_kernel(RodArgs a) {
    const int nr = a.n_rods;
    const double dt = 1.0 / a.n_sub;
    for (int r = threadIdx.x; r < nr; r += blockDim.x) {
        double *rod = a.rods + r * ROD_STRIDE;
        for (int q = 0; q < 3; ++q) rod[ROD_XOLD + q] = rod[ROD_X + q];
        for (int q = 0; q < 4; ++q) rod[ROD_QOLD + q] = rod[ROD_Q + q];
    }
    for (int sub = 0; sub < a.n_sub; ++sub) {
        __syncthreads();
        // contact forces at the positions of this substep
        for (int r = threadIdx.x; r < nr; r += blockDim.x) {
            const double *ra = a.rods + r * ROD_STRIDE;
            const d3 Xa = ld3(ra + ROD_X), ea = quat_axis(ra + ROD_Q);
            const d3 pa = Xa - a.half * ea, qa = Xa + a.half * ea;
            d3 F = mk(0, 0, 0), T = mk(0, 0, 0);
            const double reach = 2.0 * a.half + fmax(a.d0, a.eps_att > 0.0 ? a.r_cut : a.d0);
            for (int s = 0; s < nr; ++s) {
                if (s == r) continue;
                const double *rb = a.rods + s * ROD_STRIDE;
                const d3 Xb = ld3(rb + ROD_X);
                const d3 dx = min_image(Xb - Xa, a);
                if (dot(dx, dx) >= reach * reach) continue;
                const d3 shift = dx - (Xb - Xa);
                const d3 eb = quat_axis(rb + ROD_Q);
                const d3 pb = Xb - a.half * eb + shift, qb = Xb + a.half * eb + shift;
                d3 ca, cb;
                const double d = seg_seg(pa, qa, pb, qb, ca, cb);
                if (d <= 0.0) continue;
                const double fm = pair_force(d, a);
                if (fm == 0.0) continue;
                const d3 fv = (fm / d) * (ca - cb);
                F = F + fv;
                T = T + cross(ca - Xa, fv);
            }
            if (a.wall_on) {
                const d3 low = pa.z <= qa.z ? pa : qa;
                const double h = low.z - a.wall_z;
                if (h > 0.0 && h <= a.d0_wall) {
                    const d3 fw = mk(0, 0, -a.eps_wall * ljf_d(h, a.d0_wall));
                    F = F + fw;
                    T = T + cross(low - Xa, fw);
                }
            }
            double *rw = a.rods + r * ROD_STRIDE;
            st3(rw + ROD_FC, F);
            st3(rw + ROD_TC, T);
        }
        __syncthreads();
        for (int r = threadIdx.x; r < nr; r += blockDim.x) {
            double *rod = a.rods + r * ROD_STRIDE;
            const d3 F = ld3(rod + ROD_FS) + ld3(rod + ROD_FA) + ld3(rod + ROD_FC);
            const d3 T = ld3(rod + ROD_TS) + ld3(rod + ROD_TA) + ld3(rod + ROD_TC);
            d3 V = ld3(rod + ROD_V) + (dt / a.mass) * F;
            d3 X = ld3(rod + ROD_X) + dt * V;
            const d3 L = ld3(rod + ROD_L) + dt * T;
            st3(rod + ROD_V, V);
            st3(rod + ROD_L, L);
            const d3 w = omega_of(rod, a);  // uses the new L and the current q
            const double wn = sqrt(dot(w, w));
            if (wn > 0.0) {
                const double h = 0.5 * wn * dt;
                const double sh = sin(h) / wn;
                const double dq[4] = {cos(h), sh * w.x, sh * w.y, sh * w.z};
                const double *q = rod + ROD_Q;
                double qn[4] = {dq[0] * q[0] - dq[1] * q[1] - dq[2] * q[2] - dq[3] * q[3],
                                dq[0] * q[1] + dq[1] * q[0] + dq[2] * q[3] - dq[3] * q[2],
                                dq[0] * q[2] - dq[1] * q[3] + dq[2] * q[0] + dq[3] * q[1],
                                dq[0] * q[3] + dq[1] * q[2] - dq[2] * q[1] + dq[3] * q[0]};
                const double nn = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
                for (int c = 0; c < 4; ++c) rod[ROD_Q + c] = qn[c] / nn;
            }
            if (a.px) X.x = X.x - a.nx * floor(X.x / a.nx);
            if (a.py) X.y = X.y - a.ny * floor(X.y / a.ny);
            if (a.pz) X.z = X.z - a.nz * floor(X.z / a.nz);
            st3(rod + ROD_X, X);
        }
    }
    __syncthreads();
    // a rod may move less than one node per step (the re-mask relies on it)
    for (int r = threadIdx.x; r < nr; r += blockDim.x) {
        double *rod = a.rods + r * ROD_STRIDE;
        const d3 dX = min_image(ld3(rod + ROD_X) - ld3(rod + ROD_XOLD), a);
        const d3 e0 = quat_axis(rod + ROD_QOLD), e1 = quat_axis(rod + ROD_Q);
        const d3 de = e1 - e0;
        const double tip = sqrt(dot(dX, dX)) + (a.half + a.radius) * sqrt(dot(de, de));
        if (!(tip < 0.9)) atomicOr(a.status, ST_ROD);
    }
}

// ---------------------------------------------------------------------------
// 3. new occupancy of every rod (newid has been filled with -1)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(RB) rod_mask_kernel(RodArgs a) {
    const double *rod = a.rods + blockIdx.x * ROD_STRIDE;
    const Box b = rod_box(rod, a, 0);
    const int ex = b.hi[0] - b.lo[0] + 1, ey = b.hi[1] - b.lo[1] + 1, ez = b.hi[2] - b.lo[2] + 1;
    const int64_t nbox = int64_t(ex) * ey * ez;
    for (int64_t m = threadIdx.x; m < nbox; m += RB) {
        int x = b.lo[0] + int(m % ex), y = b.lo[1] + int((m / ex) % ey), z = b.lo[2] + int(m / (int64_t(ex) * ey));
        if (!inside_capsule(rod, mk(x, y, z), a)) continue;
        if (!wrap_coord(x, a.nx, a.px) || !wrap_coord(y, a.ny, a.py) || !wrap_coord(z, a.nz, a.pz)) {
            atomicOr(a.status, ST_ROD);
            continue;
        }
        const int64_t n = (int64_t(z) * a.ny + y) * a.nx + x;
        if ((a.mat[n] & MAT_ID_MASK) != MAT_FLUID && (a.mat[n] & MAT_ID_MASK) != MAT_ROD) {
            atomicOr(a.status, ST_ROD);  // a rod ran into a wall or the reservoir
            continue;
        }
        a.newid[n] = static_cast<int16_t>(blockIdx.x);
    }
}

__global__ void fill_i16_kernel(int16_t *p, int64_t n, int16_t v) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------
// 4. cover / uncover (init = 1: place the rods without bookkeeping)
// ---------------------------------------------------------------------------
template <class S>
__global__ void __launch_bounds__(RB) rod_update_kernel(RodArgs a, S *f, int init) {
    __shared__ double sh[RB / 64];
    double *rod = a.rods + blockIdx.x * ROD_STRIDE;
    const int r = blockIdx.x;
    const Box b = rod_box(rod, a, 1);  // covers the old position too (moves < 1 node)
    const int ex = b.hi[0] - b.lo[0] + 1, ey = b.hi[1] - b.lo[1] + 1, ez = b.hi[2] - b.lo[2] + 1;
    const int64_t nbox = int64_t(ex) * ey * ez;
    const d3 X = ld3(rod + ROD_X);
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // momentum[3], torque[3], mass[2]
    for (int64_t m = threadIdx.x; m < nbox; m += RB) {
        int x = b.lo[0] + int(m % ex), y = b.lo[1] + int((m / ex) % ey), z = b.lo[2] + int(m / (int64_t(ex) * ey));
        const double px = x, py = y, pz = z;
        if (!wrap_coord(x, a.nx, a.px) || !wrap_coord(y, a.ny, a.py) || !wrap_coord(z, a.nz, a.pz)) continue;
        const int64_t n = (int64_t(z) * a.ny + y) * a.nx + x;
        const int16_t oldid = a.rodid[n], newid = a.newid[n];
        const bool cover = newid == r && oldid != r;
        const bool uncover = oldid == r && newid != r;
        if (!cover && !uncover) continue;
        const d3 arm = min_image(mk(px, py, pz) - X, a);
        if (cover) {
            if (!init) {
                d3 mom = mk(0, 0, 0);
                for (int k = 0; k < 2; ++k) {
                    double s = 0.0;
                    d3 jk = mk(0, 0, 0);
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
        } else {
            // uncovered: f = f^eq(rho_bar, u_b), rho_bar = mean over neighbours
            // that are fluid before and after the move
            double rb[2] = {0.0, 0.0};
            int cnt = 0;
            bool near_wall = false;
            for (int i = 1; i < Q; ++i) {
                int xx = x + cx(i), yy = y + cy(i), zz = z + cz(i);
                if (!wrap_coord(xx, a.nx, a.px) || !wrap_coord(yy, a.ny, a.py) || !wrap_coord(zz, a.nz, a.pz)) continue;
                const int64_t q = (int64_t(zz) * a.ny + yy) * a.nx + xx;
                const uint8_t mq = a.mat[q] & MAT_ID_MASK;
                near_wall |= is_static_wall(mq);
                if (mq == MAT_FLUID && a.rodid[q] < 0 && a.newid[q] < 0) {
                    for (int k = 0; k < 2; ++k) {
                        double s = 0.0;
                        for (int j = 0; j < Q; ++j) s += decf(f, (k * Q + j) * a.fs + q) + wgt<double>(j) * a.rho_ref[k];
                        rb[k] += s;
                    }
                    ++cnt;
                }
            }
            if (cnt) {
                rb[0] /= cnt;
                rb[1] /= cnt;
            }
            const d3 ub = velocity_at(rod, mk(px, py, pz), a);
            const double usq = dot(ub, ub);
            d3 mom = mk(0, 0, 0);
            for (int k = 0; k < 2; ++k) {
                for (int i = 0; i < Q; ++i) {
                    const double cu = cx(i) * ub.x + cy(i) * ub.y + cz(i) * ub.z;
                    const double feq = wgt<double>(i) * rb[k] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
                    f[(k * Q + i) * a.fs + n] = Codec<S>::enc(typename Codec<S>::C(feq - wgt<double>(i) * a.rho_ref[k]));
                }
                acc[6 + k] -= rb[k];
                mom = mom + rb[k] * ub;
            }
            const d3 tq = cross(arm, mom);
            acc[0] -= mom.x;
            acc[1] -= mom.y;
            acc[2] -= mom.z;
            acc[3] -= tq.x;
            acc[4] -= tq.y;
            acc[5] -= tq.z;
            a.mat[n] = MAT_FLUID | (near_wall ? MAT_NEAR_WALL : 0);
        }
    }
    double tot[8];
    for (int q = 0; q < 8; ++q) tot[q] = block_sum_d(acc[q], sh);
    if (threadIdx.x == 0 && !init) {
        for (int q = 0; q < 3; ++q) rod[ROD_V + q] += tot[q] / a.mass;
        for (int q = 0; q < 3; ++q) rod[ROD_L + q] += tot[3 + q];
        rod[ROD_SOLID] += tot[6];
        rod[ROD_SOLID + 1] += tot[7];
    }
}

// commit the new occupancy of rod r (after every block has read the old one)
__global__ void __launch_bounds__(RB) rod_commit_kernel(RodArgs a) {
    const double *rod = a.rods + blockIdx.x * ROD_STRIDE;
    const int r = blockIdx.x;
    const Box b = rod_box(rod, a, 1);
    const int ex = b.hi[0] - b.lo[0] + 1, ey = b.hi[1] - b.lo[1] + 1, ez = b.hi[2] - b.lo[2] + 1;
    const int64_t nbox = int64_t(ex) * ey * ez;
    for (int64_t m = threadIdx.x; m < nbox; m += RB) {
        int x = b.lo[0] + int(m % ex), y = b.lo[1] + int((m / ex) % ey), z = b.lo[2] + int(m / (int64_t(ex) * ey));
        if (!wrap_coord(x, a.nx, a.px) || !wrap_coord(y, a.ny, a.py) || !wrap_coord(z, a.nz, a.pz)) continue;
        const int64_t n = (int64_t(z) * a.ny + y) * a.nx + x;
        if (a.rodid[n] == r || a.newid[n] == r) a.rodid[n] = a.newid[n];
    }
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
// 5. moving bounce-back slots for the next pull, and the momentum they carry
// ---------------------------------------------------------------------------
template <class S>
__global__ void __launch_bounds__(RB) rod_link_kernel(RodArgs a, S *f) {
    __shared__ double sh[RB / 64];
    double *rod = a.rods + blockIdx.x * ROD_STRIDE;
    const int r = blockIdx.x;
    const Box b = rod_box(rod, a, 1);
    const int ex = b.hi[0] - b.lo[0] + 1, ey = b.hi[1] - b.lo[1] + 1, ez = b.hi[2] - b.lo[2] + 1;
    const int64_t nbox = int64_t(ex) * ey * ez;
    const d3 X = ld3(rod + ROD_X);
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // dP[3], dT[3], mass[2]
    for (int64_t m = threadIdx.x; m < nbox; m += RB) {
        int x = b.lo[0] + int(m % ex), y = b.lo[1] + int((m / ex) % ey), z = b.lo[2] + int(m / (int64_t(ex) * ey));
        const double px = x, py = y, pz = z;
        if (!wrap_coord(x, a.nx, a.px) || !wrap_coord(y, a.ny, a.py) || !wrap_coord(z, a.nz, a.pz)) continue;
        const int64_t n = (int64_t(z) * a.ny + y) * a.nx + x;
        if ((a.mat[n] & MAT_ID_MASK) != MAT_FLUID) continue;
        bool any = false;
        for (int i = 1; i < Q; ++i) {
            int xx = x - cx(i), yy = y - cy(i), zz = z - cz(i);
            if (!wrap_coord(xx, a.nx, a.px) || !wrap_coord(yy, a.ny, a.py) || !wrap_coord(zz, a.nz, a.pz)) continue;
            any |= a.rodid[(int64_t(zz) * a.ny + yy) * a.nx + xx] == r;
        }
        if (!any) continue;
        double rho[2];
        for (int k = 0; k < 2; ++k) {
            double s = 0.0;
            for (int j = 0; j < Q; ++j) s += decf(f, (k * Q + j) * a.fs + n) + wgt<double>(j) * a.rho_ref[k];
            rho[k] = s;
        }
        for (int i = 1; i < Q; ++i) {
            int xx = x - cx(i), yy = y - cy(i), zz = z - cz(i);
            if (!wrap_coord(xx, a.nx, a.px) || !wrap_coord(yy, a.ny, a.py) || !wrap_coord(zz, a.nz, a.pz)) continue;
            const int64_t s = (int64_t(zz) * a.ny + yy) * a.nx + xx;
            if (a.rodid[s] != r) continue;
            const d3 ci = mk(cx(i), cy(i), cz(i));
            const d3 xb = mk(px - 0.5 * cx(i), py - 0.5 * cy(i), pz - 0.5 * cz(i));
            const d3 ub = velocity_at(rod, xb, a);
            const d3 arm = min_image(xb - X, a);
            d3 dp = mk(0, 0, 0);
            for (int k = 0; k < 2; ++k) {
                const double fo = decf(f, (k * Q + opp(i)) * a.fs + n) + wgt<double>(opp(i)) * a.rho_ref[k];
                const double add = 2.0 * wgt<double>(i) * rho[k] * dot(ci, ub) * 3.0;
                const double fin = fo + add;
                f[(k * Q + i) * a.fs + s] = Codec<S>::enc(typename Codec<S>::C(fin - wgt<double>(i) * a.rho_ref[k]));
                dp = dp - (fo + fin) * ci;
                acc[6 + k] -= add;
            }
            const d3 tq = cross(arm, dp);
            acc[0] += dp.x;
            acc[1] += dp.y;
            acc[2] += dp.z;
            acc[3] += tq.x;
            acc[4] += tq.y;
            acc[5] += tq.z;
        }
    }
    double tot[8];
    for (int q = 0; q < 8; ++q) tot[q] = block_sum_d(acc[q], sh);
    if (threadIdx.x == 0) {
        for (int q = 0; q < 6; ++q) rod[ROD_FS + q] = tot[q];
        // booked once the next fluid step has streamed these slots
        rod[ROD_PEND] = tot[6];
        rod[ROD_PEND + 1] = tot[7];
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

hipError_t launch_rods_place(int prec, const RodArgs &a, void *f, hipStream_t s) {
    if (a.n_rods == 0) return hipSuccess;
    const int64_t n = int64_t(a.nx) * a.ny * a.nz;
    hipLaunchKernelGGL(fill_i16_kernel, dim3(fill_grid(n)), dim3(256), 0, s, a.newid, n, int16_t(-1));
    hipLaunchKernelGGL(rod_mask_kernel, dim3(a.n_rods), dim3(RB), 0, s, a);
    hipError_t e = rods_by_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(rod_update_kernel<S>, dim3(a.n_rods), dim3(RB), 0, s, a, static_cast<S *>(f), 1);
        hipLaunchKernelGGL(rod_commit_kernel, dim3(a.n_rods), dim3(RB), 0, s, a);
        hipLaunchKernelGGL(rod_link_kernel<S>, dim3(a.n_rods), dim3(RB), 0, s, a, static_cast<S *>(f));
        return hipGetLastError();
    });
    return e;
}

hipError_t launch_rods_sums(const RodArgs &a, double *out, hipStream_t s) {
    hipLaunchKernelGGL(rod_sums_kernel, dim3(1), dim3(64), 0, s, a, out);
    return hipGetLastError();
}

hipError_t launch_rods_step(int prec, const RodArgs &a, void *f, hipStream_t s) {
    if (a.n_rods == 0) return hipSuccess;
    const int64_t n = int64_t(a.nx) * a.ny * a.nz;
    hipError_t e = rods_by_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(rod_adhesion_kernel<S>, dim3(a.n_rods), dim3(RB), 0, s, a, static_cast<const S *>(f));
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rod_integrate_kernel, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(fill_i16_kernel, dim3(fill_grid(n)), dim3(256), 0, s, a.newid, n, int16_t(-1));
    hipLaunchKernelGGL(rod_mask_kernel, dim3(a.n_rods), dim3(RB), 0, s, a);
    return rods_by_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(rod_update_kernel<S>, dim3(a.n_rods), dim3(RB), 0, s, a, static_cast<S *>(f), 0);
        hipLaunchKernelGGL(rod_commit_kernel, dim3(a.n_rods), dim3(RB), 0, s, a);
        hipLaunchKernelGGL(rod_link_kernel<S>, dim3(a.n_rods), dim3(RB), 0, s, a, static_cast<S *>(f));
        return hipGetLastError();
    });
}

}  // namespace lbm
