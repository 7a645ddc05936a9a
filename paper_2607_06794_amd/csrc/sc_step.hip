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
// is in LDS.  Densities therefore never travel through HBM: every population
// is read once and written once, the ring re-reads hit L2.
//
// Boundaries inside the same pass:
//  * static walls (halfway bounce-back): a fluid node next to a wall writes
//    f*_j(x) into the wall node's slot of direction opp(j), so the next pull
//    is branch-free;
//  * the reservoir plane z = nz-1: the plane below it takes w_i rho_top_k for
//    the directions pulled from the reservoir and books the outflow of its
//    stored f*(t) towards the reservoir into a
//    per-tile FP64 ledger slot (deterministic: each tile owns its slot);
//  * rod nodes: their slots are written by the rod link kernel.
#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

namespace {

__device__ inline int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
__device__ inline int wrapmod(int v, int n) {
    int r = v % n;
    return r < 0 ? r + n : r;
}

// Per-node source offsets: o[0] = coordinate - 1, o[1] = coordinate, o[2] = + 1
struct NodeIdx {
    uint32_t xo[3];
    uint32_t yo[3];  // already multiplied by nx
    bool valid;
};

__device__ inline NodeIdx make_node(int x, int y, const StepArgs &a) {
    NodeIdx n;
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
    const int xm = a.px ? wrap1(x - 1, a.nx) : max(x - 1, 0);
    const int xp = a.px ? wrap1(x + 1, a.nx) : min(x + 1, a.nx - 1);
    const int ym = a.py ? wrap1(y - 1, a.ny) : max(y - 1, 0);
    const int yp = a.py ? wrap1(y + 1, a.ny) : min(y + 1, a.ny - 1);
    n.xo[0] = xm;
    n.xo[1] = x;
    n.xo[2] = xp;
    n.yo[0] = static_cast<uint32_t>(ym) * a.nx;
    n.yo[1] = static_cast<uint32_t>(y) * a.nx;
    n.yo[2] = static_cast<uint32_t>(yp) * a.nx;
    return n;
}

// Pull the 19 population deviations d_i = f_i - w_i rho_ref of component k at
// node n on the plane with offsets zo; directions pulled from the reservoir
// plane take w_i (rho_top_k - rho_ref_k).
template <class S, class C>
__device__ inline void pull_devs(const S *__restrict__ f, int64_t fs, int k, const NodeIdx &n,
                                 const uint32_t zo[3], bool top_rule, C top_dev_k, C v[Q]) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const uint32_t src = zo[1 - cz(i)] + n.yo[1 - cy(i)] + n.xo[1 - cx(i)];
        if (cz(i) == -1 && top_rule) {
            v[i] = wgt<C>(i) * top_dev_k;
        } else {
            v[i] = Codec<S>::dec(f[static_cast<int64_t>(k * Q + i) * fs + src]);
        }
    }
}

template <class C>
__device__ inline C wave_sum(C v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace

template <class S, int TY, int NPT, bool TAU1>
__global__ void __launch_bounds__(64 * (TY / NPT)) sc_step_kernel(StepArgs a) {
    using C = typename Codec<S>::C;
    constexpr int TX = 64;
    constexpr int RY = TY / NPT;
    constexpr int NT = TX * RY;
    constexpr int HX = TX + 2, HY = TY + 2, PL = HX * HY;
    constexpr int NH = 2 * HX + 2 * TY;
    constexpr int NHPT = (NH + NT - 1) / NT;
    constexpr int NW = NT / 64;

    __shared__ C ring[4][2][PL];
    __shared__ double red[NW][2];

    // ---- tile of this work-group; consecutive tiles stay on one XCD
    const int nblk = gridDim.x;
    int b = blockIdx.x;
    if ((nblk & 7) == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
    const int tx = b % a.ntx;
    const int ty = (b / a.ntx) % a.nty;
    const int tz = b / (a.ntx * a.nty);
    const int x0 = tx * TX, y0 = ty * TY;
    const int z0 = tz * a.zchunk;
    const int z1 = min(z0 + a.zchunk, a.nz);
    if (z0 >= a.nz) return;  // uniform per block

    const int tid = threadIdx.x;
    const int lx = tid & 63;
    const int ly = tid >> 6;
    const S *__restrict__ fsrc = static_cast<const S *>(a.fsrc);
    S *__restrict__ fdst = static_cast<S *>(a.fdst);
    const uint32_t nxy = static_cast<uint32_t>(a.nx) * a.ny;

    // constants in compute precision; rref is the storage reference density
    // (0 for the FP64 form), populations travel as d_i = f_i - w_i rref
    const C G = C(a.G);
    const C rref[2] = {C(a.rho_ref[0]), C(a.rho_ref[1])};
    const C rtop[2] = {C(a.rho_top[0]), C(a.rho_top[1])};
    const C tdev[2] = {C(a.rho_top[0] - a.rho_ref[0]), C(a.rho_top[1] - a.rho_ref[1])};
    const C om[2] = {C(a.omega[0]), C(a.omega[1])};
    const C ta[2] = {C(a.tau[0]), C(a.tau[1])};
    const C gb[3] = {C(a.g[0]), C(a.g[1]), C(a.g[2])};

    // ---- owned interior nodes and ring (halo) nodes of this thread
    NodeIdx own[NPT];
    bool own_fin[NPT];
    int own_ring[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
        const int yy = ly + r * RY;
        own[r] = make_node(x0 + lx, y0 + yy, a);
        own_fin[r] = (x0 + lx < a.nx) && (y0 + yy < a.ny);
        own_ring[r] = (yy + 1) * HX + (lx + 1);
    }
    NodeIdx hal[NHPT];
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

    // moments of the owned nodes: current plane and next plane
    C cur_rho[NPT][2], cur_drho[NPT][2], cur_j[NPT][2][3];
    C nxt_rho[NPT][2], nxt_drho[NPT][2], nxt_j[NPT][2][3];
    C cur_f[TAU1 ? 1 : NPT][TAU1 ? 1 : 2][TAU1 ? 1 : Q];
    C nxt_f[TAU1 ? 1 : NPT][TAU1 ? 1 : 2][TAU1 ? 1 : Q];
    uint8_t cur_m[NPT], nxt_m[NPT];

    // psi of a node given its material byte and densities
    auto psi_of = [&](uint8_t m, int k, C rho) -> C {
        const uint8_t id = m & MAT_ID_MASK;
        if (id == MAT_FLUID) return rho;
        if (id == MAT_GHOST) return rtop[k];
        return C(a.psi_s[id][k]);
    };

    // fill the ring slot of plane z (and the owned moments when own_out)
    auto fill_plane = [&](int z, bool keep) {
        const int slot = z & 3;
        bool zvalid;
        int zz = z;
        if (a.pz) {
            zz = wrap1(z, a.nz);
            zvalid = true;
        } else {
            zvalid = (z >= 0 && z < a.nz);
        }
        zz = min(max(zz, 0), a.nz - 1);
        const int zm = a.pz ? wrap1(zz - 1, a.nz) : max(zz - 1, 0);
        const int zp = a.pz ? wrap1(zz + 1, a.nz) : min(zz + 1, a.nz - 1);
        const uint32_t zo[3] = {zm * nxy, zz * nxy, zp * nxy};
        const bool top_rule = a.evap && (zz == a.nz - 2);
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            const NodeIdx &n = own[r];
            const bool v = zvalid && n.valid;
            const uint8_t m = v ? a.mat[zo[1] + n.yo[1] + n.xo[1]] : uint8_t(MAT_ID_MASK);
            C rho[2] = {C(0), C(0)}, drho[2] = {C(0), C(0)};
            C j[2][3] = {{C(0), C(0), C(0)}, {C(0), C(0), C(0)}};
            if (v && (m & MAT_ID_MASK) == MAT_FLUID) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    C fv[Q];
                    pull_devs<S, C>(fsrc, a.fs, k, n, zo, top_rule, tdev[k], fv);
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
                    drho[k] = s;
                    rho[k] = rref[k] + s;
                    j[k][0] = jx;
                    j[k][1] = jy;
                    j[k][2] = jz;
                    if constexpr (!TAU1) {
                        if (keep) {
#pragma unroll
                            for (int i = 0; i < Q; ++i) nxt_f[r][k][i] = fv[i];
                        }
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
            const NodeIdx &n = hal[mm];
            const bool v = zvalid && n.valid;
            const uint8_t m = v ? a.mat[zo[1] + n.yo[1] + n.xo[1]] : uint8_t(MAT_ID_MASK);
            C rho[2] = {C(0), C(0)};
            if (v && (m & MAT_ID_MASK) == MAT_FLUID) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    C fv[Q];
                    pull_devs<S, C>(fsrc, a.fs, k, n, zo, top_rule, tdev[k], fv);
                    C s = C(0);
#pragma unroll
                    for (int i = 0; i < Q; ++i) s += fv[i];
                    rho[k] = rref[k] + s;
                }
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

    // prologue: planes z0-1 (psi only) and z0 (psi + moments)
    fill_plane(z0 - 1, false);
    fill_plane(z0, true);
    shift_next();

    for (int z = z0; z < z1; ++z) {
        fill_plane(z + 1, true);
        __syncthreads();

        const int sm = (z - 1) & 3, s0 = z & 3, sp = (z + 1) & 3;
        const uint32_t zoff = static_cast<uint32_t>(z) * nxy;
        const bool ledger_plane = a.evap && (z == a.nz - 2);
        double led[2] = {0.0, 0.0};
        unsigned st = 0;

#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            if (!own_fin[r] || (cur_m[r] & MAT_ID_MASK) != MAT_FLUID) continue;
            const int rc = own_ring[r];
            const C rho[2] = {cur_rho[r][0], cur_rho[r][1]};
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
            const C usq_chk = up[0] * up[0] + up[1] * up[1] + up[2] * up[2];
            if (!(rho[0] + rho[1] > C(0))) st |= ST_RHO;
            if (!(usq_chk <= C(0.09))) st |= (usq_chk != usq_chk) ? ST_NAN : ST_SPEED;

            const uint32_t idx = zoff + own[r].yo[1] + own[r].xo[1];
            const bool near_wall = (cur_m[r] & MAT_NEAR_WALL) != 0;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                C ue[3];
                const bool ok = rho[k] >= C(1e-12);
                const C rk = ok ? ta[k] / rho[k] : C(0);
#pragma unroll
                for (int d = 0; d < 3; ++d) ue[d] = up[d] + F[k][d] * rk;
                const C usq = ue[0] * ue[0] + ue[1] * ue[1] + ue[2] * ue[2];
                const C dr = cur_drho[r][k];
                C fstar[Q];
                C deq_sum = C(0);
#pragma unroll
                for (int ii = 1; ii <= Q; ++ii) {
                    const int i = ii % Q;  // directions 1..18 first, the rest direction last
                    // Eq. 2 as a deviation: f_i^eq - w_i rref = w_i (rho - rref) + w_i rho [3 c.u + 9/2 (c.u)^2 - 3/2 u^2].
                    // The rest population is the remainder so that sum_i f_i^eq = rho holds up to one
                    // rounding: the rounded weights do not sum to one, and using them for all 19
                    // directions would drift the mass by a fixed factor every step.
                    const C cu = C(cx(i)) * ue[0] + C(cy(i)) * ue[1] + C(cz(i)) * ue[2];
                    C deq;
                    if (i != 0) {
                        deq = wgt<C>(i) * dr + wgt<C>(i) * rho[k] * (C(3) * cu + C(4.5) * cu * cu - C(1.5) * usq);
                        deq_sum += deq;
                    } else {
                        deq = dr - deq_sum;
                    }
                    C ds;
                    if constexpr (TAU1) {
                        ds = deq;  // Eq. 1 with tau = 1: f* = f^eq
                    } else {
                        ds = cur_f[r][k][i] - (cur_f[r][k][i] - deq) * om[k];
                    }
                    fstar[i] = ds;
                    fdst[static_cast<int64_t>(k * Q + i) * a.fs + idx] = Codec<S>::enc(ds);
                }
                if (ledger_plane) {
                    // this step's streaming moves the node's stored f*_i(t) with c_iz = +1
                    // into the reservoir and pulls w_i rho_top_k out of it
                    double outflow = 0.0, inflow = 0.0;
#pragma unroll
                    for (int i = 0; i < Q; ++i) {
                        if (cz(i) == 1)
                            outflow += double(Codec<S>::dec(fsrc[static_cast<int64_t>(k * Q + i) * a.fs + idx])) +
                                       wgt<double>(i) * a.rho_ref[k];
                        if (cz(i) == -1) inflow += wgt<double>(i) * a.rho_top[k];
                    }
                    led[k] += outflow - inflow;
                }
                if (near_wall) {
                    // halfway bounce-back: hand f*_j(x) to the wall node x + c_j as
                    // direction opp(j) (w_j = w_opp(j), so the deviation carries over)
                    const uint32_t zo3[3] = {
                        static_cast<uint32_t>(a.pz ? wrap1(z - 1, a.nz) : max(z - 1, 0)) * nxy, zoff,
                        static_cast<uint32_t>(a.pz ? wrap1(z + 1, a.nz) : min(z + 1, a.nz - 1)) * nxy};
#pragma unroll
                    for (int jd = 1; jd < Q; ++jd) {
                        const uint32_t nb = zo3[1 + cz(jd)] + own[r].yo[1 + cy(jd)] + own[r].xo[1 + cx(jd)];
                        if (is_static_wall(a.mat[nb] & MAT_ID_MASK))
                            fdst[static_cast<int64_t>(k * Q + opp(jd)) * a.fs + nb] = Codec<S>::enc(fstar[jd]);
                    }
                }
            }
        }
        if (st) atomicOr(a.status, st);

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
}

int tiles_xy(int nx, int ny, int tile_y) { return ((nx + 63) / 64) * ((ny + tile_y - 1) / tile_y); }

template <class S, int TY, int NPT, bool TAU1>
static hipError_t launch_one(const StepArgs &a, hipStream_t s) {
    const int nblk = a.ntx * a.nty * a.nzc;
    hipLaunchKernelGGL((sc_step_kernel<S, TY, NPT, TAU1>), dim3(nblk), dim3(64 * (TY / NPT)), 0, s, a);
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
