// Colour-gradient D3Q19 step for gfx950 (the paper's fluid model; Methods,
// "Fluid-filament simulation method"): per component BGK towards the
// equilibrium of the common velocity (Eqs. 1-3), the capillary force of a
// continuum-surface formulation from the curvature of the colour field
// C = (rho_1 - rho_2) / (rho_1 + rho_2), weighted by the density fractions and
// applied before the collision (Guo's forcing), then recolouring; wetting by
// a ghost colour in the solid layer and wall normals from the voxel geometry,
// the interface normal turned to the wall's contact angle.
//
// The curvature needs the colour two nodes out, so the step runs as three
// passes over SoA arrays (thread per node, x fastest, coalesced):
//   1. colour:  pull the 38 populations of each fluid node, C into an array;
//               then each static wall node's ghost colour, the w-weighted
//               mean C of its fluid neighbours, into the same array;
//   2. normal:  grad C from the neighbours' C (ghost colours on walls),
//               unit normal with the contact-angle correction next to walls,
//               n and |grad C| into four arrays;
//   3. collide: pull again, moments, curvature from the neighbours' normals,
//               CSF force, Guo-forced BGK per component, recolouring, store,
//               and hand the bounce-back values to the wall nodes.
// Passes 2 and 3 read their stencils from L2 (each value is used by 19
// threads of neighbouring rows).  HBM traffic per fluid node: the populations
// read twice and written once plus the colour and normal arrays.
#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

namespace {

__device__ inline int wrapc(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// neighbour x + d of a node along one axis: wrapped in a periodic direction;
// in a closed one, false when outside the lattice
__device__ inline bool step_axis(int &v, int d, int n, int per) {
    v += d;
    if (per) {
        v = wrapc(v, n);
        return true;
    }
    return v >= 0 && v < n;
}

template <class S>
__device__ inline typename Codec<S>::C load_pop(const CGArgs &a, const S *f, int k, int i, int64_t node) {
    using C = typename Codec<S>::C;
    return Codec<S>::dec(f[(int64_t(k) * Q + i) * a.fs + node]) + wgt<C>(i) * C(a.rho_ref[k]);
}

// the 38 post-streaming populations of fluid node (x, y, z): f_i(x) =
// f*_i(x - c_i); wall nodes hold the bounce-back values handed to them
template <class S>
__device__ inline void pull(const CGArgs &a, int x, int y, int z, typename Codec<S>::C (&fv)[2][Q]) {
    const S *f = static_cast<const S *>(a.fsrc);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        // fluid nodes never sit on a closed end plane, so x - c_i is inside
        const int xs = a.px ? wrapc(x - cx(i), a.nx) : x - cx(i);
        const int ys = a.py ? wrapc(y - cy(i), a.ny) : y - cy(i);
        const int zs = a.pz ? wrapc(z - cz(i), a.nz) : z - cz(i);
        const int64_t src = (int64_t(zs) * a.ny + ys) * a.nx + xs;
#pragma unroll
        for (int k = 0; k < 2; ++k) fv[k][i] = load_pop<S>(a, f, k, i, src);
    }
}

__device__ inline void decode(int64_t n, const CGArgs &a, int &x, int &y, int &z) {
    x = int(n % a.nx);
    const int64_t r = n / a.nx;
    y = int(r % a.ny);
    z = int(r / a.ny);
}

// ---- pass 1: colour of every fluid node -----------------------------------
template <class S>
__global__ void __launch_bounds__(256) cg_colour_kernel(CGArgs a) {
    using C = typename Codec<S>::C;
    const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (n >= a.nodes) return;
    if ((a.mat[n] & MAT_ID_MASK) != MAT_FLUID) return;
    int x, y, z;
    decode(n, a, x, y, z);
    C fv[2][Q];
    pull<S>(a, x, y, z, fv);
    C r0 = C(0), r1 = C(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        r0 += fv[0][i];
        r1 += fv[1][i];
    }
    const C rt = r0 + r1;
    static_cast<C *>(a.colour)[n] = rt > C(0) ? (r0 - r1) / rt : C(0);
}

// ---- pass 1b: ghost colour of the static wall nodes: the w-weighted mean C
// of each wall node's fluid neighbours (0 without any), stored in the colour
// array so that the normal pass reads one value per neighbour
template <class C>
__global__ void __launch_bounds__(256) cg_ghost_kernel(CGArgs a) {
    const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (n >= a.nodes) return;
    if (!is_static_wall(a.mat[n] & MAT_ID_MASK)) return;
    int x, y, z;
    decode(n, a, x, y, z);
    C *col = static_cast<C *>(a.colour);
    C num = C(0), den = C(0);
#pragma unroll
    for (int j = 1; j < Q; ++j) {
        int vx = x, vy = y, vz = z;
        if (!step_axis(vx, cx(j), a.nx, a.px) || !step_axis(vy, cy(j), a.ny, a.py) || !step_axis(vz, cz(j), a.nz, a.pz))
            continue;
        const int64_t v = (int64_t(vz) * a.ny + vy) * a.nx + vx;
        if ((a.mat[v] & MAT_ID_MASK) == MAT_FLUID) {
            num += wgt<C>(j) * col[v];
            den += wgt<C>(j);
        }
    }
    col[n] = den > C(0) ? num / den : C(0);
}

// colour seen at node q: C on fluid nodes, the ghost colour on static wall
// nodes, 0 elsewhere
template <class C>
__device__ inline C colour_at(const CGArgs &a, int qx, int qy, int qz) {
    const int64_t q = (int64_t(qz) * a.ny + qy) * a.nx + qx;
    const uint8_t m = a.mat[q] & MAT_ID_MASK;
    return (m == MAT_FLUID || is_static_wall(m)) ? static_cast<const C *>(a.colour)[q] : C(0);
}

// ---- pass 2: interface normal ---------------------------------------------
template <class C>
__global__ void __launch_bounds__(256) cg_normal_kernel(CGArgs a) {
    const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (n >= a.nodes) return;
    C *nrm = static_cast<C *>(a.normal);
    const uint8_t mb = a.mat[n];
    C nv[3] = {C(0), C(0), C(0)}, mag = C(0);
    if ((mb & MAT_ID_MASK) == MAT_FLUID) {
        int x, y, z;
        decode(n, a, x, y, z);
        // grad C = (1 / c_s^2) sum_i w_i C(x + c_i) c_i
        C g[3] = {C(0), C(0), C(0)};
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int qx = a.px ? wrapc(x + cx(i), a.nx) : x + cx(i);
            const int qy = a.py ? wrapc(y + cy(i), a.ny) : y + cy(i);
            const int qz = a.pz ? wrapc(z + cz(i), a.nz) : z + cz(i);
            const C v = wgt<C>(i) * colour_at<C>(a, qx, qy, qz);
            if (cx(i)) g[0] += cx(i) * v;
            if (cy(i)) g[1] += cy(i) * v;
            if (cz(i)) g[2] += cz(i) * v;
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) g[d] *= C(3);
        mag = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        if (mag > C(a.grad_eps)) {
#pragma unroll
            for (int d = 0; d < 3; ++d) nv[d] = g[d] / mag;
            if (mb & MAT_NEAR_WALL) {
                // wall normal from the solid neighbours (into the fluid) and
                // their w-weighted mean cos(theta)
                C s[3] = {C(0), C(0), C(0)}, ws = C(0), cts = C(0);
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    const int qx = a.px ? wrapc(x + cx(i), a.nx) : x + cx(i);
                    const int qy = a.py ? wrapc(y + cy(i), a.ny) : y + cy(i);
                    const int qz = a.pz ? wrapc(z + cz(i), a.nz) : z + cz(i);
                    const uint8_t mq = a.mat[(int64_t(qz) * a.ny + qy) * a.nx + qx] & MAT_ID_MASK;
                    if (is_static_wall(mq)) {
                        const C w = wgt<C>(i);
                        s[0] += w * C(cx(i));
                        s[1] += w * C(cy(i));
                        s[2] += w * C(cz(i));
                        ws += w;
                        cts += w * C(a.cos_theta[mq]);
                    }
                }
                const C sn = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
                if (ws > C(0) && sn > C(0)) {
                    const C nw[3] = {-s[0] / sn, -s[1] / sn, -s[2] / sn};
                    const C ct = cts / ws;
                    const C dot = nv[0] * nw[0] + nv[1] * nw[1] + nv[2] * nw[2];
                    C t[3] = {nv[0] - dot * nw[0], nv[1] - dot * nw[1], nv[2] - dot * nw[2]};
                    const C tm = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
                    if (tm > C(1e-12)) {
                        const C st = sqrt(fmax(C(1) - ct * ct, C(0)));
#pragma unroll
                        for (int d = 0; d < 3; ++d) nv[d] = -ct * nw[d] + st * (t[d] / tm);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) nrm[d * a.fs + n] = nv[d];
    nrm[3 * a.fs + n] = mag;
}

// ---- pass 3: force, collision, recolouring ---------------------------------
template <class S>
__global__ void __launch_bounds__(256) cg_collide_kernel(CGArgs a) {
    using C = typename Codec<S>::C;
    const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (n >= a.nodes) return;
    const uint8_t mb = a.mat[n];
    if ((mb & MAT_ID_MASK) != MAT_FLUID) return;
    const unsigned known = *a.status;  // status bits already raised before this launch
    int x, y, z;
    decode(n, a, x, y, z);
    C fv[2][Q];
    pull<S>(a, x, y, z, fv);
    // moments (Eq. 3)
    C rho[2], j[3] = {C(0), C(0), C(0)};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        C s = C(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            s += fv[k][i];
            if (cx(i)) j[0] += cx(i) * fv[k][i];
            if (cy(i)) j[1] += cy(i) * fv[k][i];
            if (cz(i)) j[2] += cz(i) * fv[k][i];
        }
        rho[k] = s;
    }
    const C rt = rho[0] + rho[1];
    const C irt = rt > C(0) ? C(1) / rt : C(1);
    // curvature kappa = -div n; a neighbour without a normal of its own (not
    // fluid, or |grad C| at or below the threshold) enters with this node's
    const C *nrm = static_cast<const C *>(a.normal);
    const C n0[3] = {nrm[n], nrm[a.fs + n], nrm[2 * a.fs + n]};
    const C mag = nrm[3 * a.fs + n];
    C div = C(0);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int qx = a.px ? wrapc(x + cx(i), a.nx) : x + cx(i);
        const int qy = a.py ? wrapc(y + cy(i), a.ny) : y + cy(i);
        const int qz = a.pz ? wrapc(z + cz(i), a.nz) : z + cz(i);
        const int64_t q = (int64_t(qz) * a.ny + qy) * a.nx + qx;
        const bool def = (a.mat[q] & MAT_ID_MASK) == MAT_FLUID && nrm[3 * a.fs + q] > C(a.grad_eps);
        C d = C(0);
        if (cx(i)) d += cx(i) * (def ? nrm[q] : n0[0]);
        if (cy(i)) d += cy(i) * (def ? nrm[a.fs + q] : n0[1]);
        if (cz(i)) d += cz(i) * (def ? nrm[2 * a.fs + q] : n0[2]);
        div += wgt<C>(i) * d;
    }
    const C kappa = C(-3) * div;
    // CSF force F = (sigma / 2) kappa |grad C| n plus the body force
    C F[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) F[d] = C(0.5) * C(a.sigma) * kappa * mag * n0[d] + rt * C(a.g[d]);
    // common velocity with the half-force shift
    C u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = (j[d] + C(0.5) * F[d]) * irt;
    const C usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    {
        unsigned st = 0;
        if (!(rt > C(0))) st |= ST_RHO;
        if (!(usq <= C(0.09))) st |= (usq != usq) ? ST_NAN : ST_SPEED;
        post_status(a.status, known, st);
    }
    const C uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    // colour-blind post-collision populations: per component BGK towards
    // f^eq(rho_k, u) plus Guo's source with F_k = (rho_k / rho) F, summed
    C tot[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const C cu = C(cx(i)) * u[0] + C(cy(i)) * u[1] + C(cz(i)) * u[2];
        const C cF = C(cx(i)) * F[0] + C(cy(i)) * F[1] + C(cz(i)) * F[2];
        const C w = wgt<C>(i);
        const C shape = C(1) + C(3) * cu + C(4.5) * cu * cu - C(1.5) * usq;
        const C src = w * (C(3) * (cF - uF) + C(9) * cu * cF);
        C sum = C(0);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const C om = C(a.omega[k]);
            const C feq = w * rho[k] * shape;
            sum += fv[k][i] - (fv[k][i] - feq) * om + (C(1) - C(0.5) * om) * (rho[k] * irt) * src;
        }
        tot[i] = sum;
    }
    // recolouring: proportional share plus +- beta (rho_1 rho_2 / rho) w_i cos phi_i
    const C seg = C(a.beta) * rho[0] * rho[1] * irt;
    const C fr0 = rho[0] * irt, fr1 = rho[1] * irt;
    S *dst = static_cast<S *>(a.fdst);
    const bool near_wall = (mb & MAT_NEAR_WALL) != 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        C cphi = C(0);
        if (i > 0) {
            const C cn = C(cx(i)) * n0[0] + C(cy(i)) * n0[1] + C(cz(i)) * n0[2];
            cphi = i <= 6 ? cn : cn * C(0.70710678118654752440);
        }
        const C w = wgt<C>(i);
        const C o0 = fr0 * tot[i] + seg * w * cphi;
        const C o1 = fr1 * tot[i] - seg * w * cphi;
        const S e0 = Codec<S>::enc(o0 - w * C(a.rho_ref[0]));
        const S e1 = Codec<S>::enc(o1 - w * C(a.rho_ref[1]));
        dst[int64_t(i) * a.fs + n] = e0;
        dst[(int64_t(Q) + i) * a.fs + n] = e1;
        if (near_wall && i > 0) {
            // halfway bounce-back: the wall node x + c_i holds f*_i(x) as
            // direction opp(i) for the next pull
            int qx = x, qy = y, qz = z;
            if (step_axis(qx, cx(i), a.nx, a.px) && step_axis(qy, cy(i), a.ny, a.py) &&
                step_axis(qz, cz(i), a.nz, a.pz)) {
                const int64_t q = (int64_t(qz) * a.ny + qy) * a.nx + qx;
                if (is_static_wall(a.mat[q] & MAT_ID_MASK)) {
                    dst[int64_t(opp(i)) * a.fs + q] = e0;
                    dst[(int64_t(Q) + opp(i)) * a.fs + q] = e1;
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_cg_step(int prec, const CGArgs &a, hipStream_t s) {
    const dim3 grid(unsigned((a.nodes + 255) / 256)), block(256);
    switch (prec) {
        case LB_F64:
            hipLaunchKernelGGL(cg_colour_kernel<double>, grid, block, 0, s, a);
            hipLaunchKernelGGL(cg_ghost_kernel<double>, grid, block, 0, s, a);
            hipLaunchKernelGGL(cg_normal_kernel<double>, grid, block, 0, s, a);
            hipLaunchKernelGGL(cg_collide_kernel<double>, grid, block, 0, s, a);
            return hipGetLastError();
        case LB_F32:
            hipLaunchKernelGGL(cg_colour_kernel<float>, grid, block, 0, s, a);
            hipLaunchKernelGGL(cg_ghost_kernel<float>, grid, block, 0, s, a);
            hipLaunchKernelGGL(cg_normal_kernel<float>, grid, block, 0, s, a);
            hipLaunchKernelGGL(cg_collide_kernel<float>, grid, block, 0, s, a);
            return hipGetLastError();
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace lbm
