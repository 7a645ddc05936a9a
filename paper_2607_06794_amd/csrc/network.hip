// Resistor network of a deposit (Methods, electrical characterisation,
// Eqs. 15-18): beads joined below a cutoff distance with conductance 1/r,
// potentials from Kirchhoff's current law between two electrodes along x,
// node currents and the current leaving the source.
//
// The network is small next to the lattice (a few thousand beads per
// deposit), so the solve is latency-bound, not bandwidth-bound:
//  * neighbours: one thread per bead scans every bead through LDS tiles in
//    index order (a deterministic, ascending neighbour list per bead);
//  * Kirchhoff: a Jacobi-preconditioned conjugate-gradient solve in one
//    work-group -- the search direction in LDS (up to NET_LDS_P beads), the
//    other vectors in L2; each iteration costs one sparse product and two
//    work-group reductions in a fixed order, and the loop is bounded by the
//    caller's iteration limit.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lbm.h"
#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

// Fixed scratch of lb_kirchhoff_noalloc: the workspace of a network of up to
// LB_NET_NOALLOC_MAX_BEADS beads, one copy per GPU for the life of the
// process.  Host code never uses this name as an address (on the host it is a
// stand-in symbol); net_static_scratch() returns the device address.
static __device__ __align__(256) char net_scratch[net_workspace_bytes(LB_NET_NOALLOC_MAX_BEADS)];

hipError_t net_static_scratch(void **ptr, size_t *bytes) {
    constexpr int MAX_DEV = 64;
    static std::mutex mu;
    static void *addr[MAX_DEV] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(net_scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = sizeof(net_scratch);
    return hipSuccess;
}

void net_carve(NetArgs &a, void *ws) {
    const size_t nn = size_t(a.n);
    char *w = static_cast<char *>(ws);
    // doubles first (8-byte aligned from the 256-byte aligned base), then the ints
    a.g = reinterpret_cast<double *>(w);
    w += nn * NET_DEG * sizeof(double);
    a.diag = reinterpret_cast<double *>(w);
    a.r = a.diag + nn;
    a.z = a.r + nn;
    a.p = a.z + nn;
    a.q = a.p + nn;
    a.out = a.q + nn;
    w += 5 * nn * sizeof(double) + 8 * sizeof(double);
    a.nbr = reinterpret_cast<int *>(w);
    a.deg = a.nbr + nn * NET_DEG;
    a.cls = a.deg + nn;
    a.cnt = a.cls + nn;
}

namespace {

constexpr int NET_TB = 256;   // threads per work-group of the neighbour scan
constexpr int NET_CG = 1024;  // threads of the solve's single work-group

__device__ inline int net_class(double x, const NetArgs &a) { return x < a.x_src ? 1 : (x > a.x_snk ? 2 : 0); }

// every thread gets the work-group sum of v[q]: xor butterfly per
// wavefront, then the wavefront sums added in order
template <int NV>
__device__ inline void wg_sum(double (&v)[NV], double *sh) {
#pragma unroll
    for (int q = 0; q < NV; ++q)
#pragma unroll
        for (int s = 32; s > 0; s >>= 1) v[q] += __shfl_xor(v[q], s, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();  // earlier readers of sh are done
    if (l == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) sh[q * (NET_CG / 64) + w] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double t = 0.0;
        for (int k = 0; k < NET_CG / 64; ++k) t += sh[q * (NET_CG / 64) + k];
        v[q] = t;
    }
}

// beads j != i with 0 < r_ij^2 < r_c^2, ascending j; deg may exceed
// NET_DEG (only the first NET_DEG are stored; the host reports the excess)
__global__ void __launch_bounds__(NET_TB) net_edges_kernel(NetArgs a) {
    __shared__ double tile[NET_TB * 3];
    const int i = blockIdx.x * NET_TB + int(threadIdx.x);
    const bool own = i < a.n;
    const double px = own ? a.pos[3 * i] : 0.0, py = own ? a.pos[3 * i + 1] : 0.0, pz = own ? a.pos[3 * i + 2] : 0.0;
    int k = 0;
    for (int j0 = 0; j0 < a.n; j0 += NET_TB) {
        const int j = j0 + int(threadIdx.x);
        __syncthreads();
        if (j < a.n) {
            tile[3 * threadIdx.x] = a.pos[3 * j];
            tile[3 * threadIdx.x + 1] = a.pos[3 * j + 1];
            tile[3 * threadIdx.x + 2] = a.pos[3 * j + 2];
        }
        __syncthreads();
        const int m = min(NET_TB, a.n - j0);
        if (own) {
            for (int q = 0; q < m; ++q) {
                const double dx = tile[3 * q] - px, dy = tile[3 * q + 1] - py, dz = tile[3 * q + 2] - pz;
                // (dx^2 + dy^2) + dz^2 without contraction: the edge decision
                // is taken exactly as stated
                const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
                if (r2 > 0.0 && r2 < a.rc2) {
                    if (k < NET_DEG) {
                        a.nbr[size_t(i) * NET_DEG + k] = j0 + q;
                        a.g[size_t(i) * NET_DEG + k] = 1.0 / sqrt(r2);
                    }
                    ++k;
                }
            }
        }
    }
    if (own) a.deg[i] = k;
}

// Networks of up to NET_LDS_P beads keep the search direction p in LDS for
// the whole solve: the sparse product reads p at every neighbour, and from
// LDS that read no longer waits on the load of the neighbour's index from L2.
constexpr int NET_LDS_P = 16384;

// potentials (Jacobi-preconditioned CG on the free beads; the electrode beads
// are fixed), then Eq. 15's node currents and the current leaving the source
template <bool LP>
__global__ void __launch_bounds__(NET_CG) net_solve_kernel(NetArgs a) {
    __shared__ double sh[4 * (NET_CG / 64)];
    extern __shared__ double lds_p[];
    double *P = LP ? lds_p : a.p;
    const int n = a.n;
    if (threadIdx.x == 0) {
        for (int q = 0; q < 4; ++q) a.cnt[q] = 0;
    }
    __syncthreads();
    // set-up: x0 = 0 on the free beads, r0 = b = sum over source neighbours of G dV
    double s0[2] = {0.0, 0.0};  // r.z, r.r
    int maxdeg = 0, nsrc = 0, nsnk = 0, dsum = 0;
    for (int i = threadIdx.x; i < n; i += NET_CG) {
        const int ci = net_class(a.pos[3 * i], a);
        const int d = a.deg[i], dk = min(d, NET_DEG);
        double dg = 0.0, b = 0.0;
        for (int k = 0; k < dk; ++k) {
            const int j = a.nbr[size_t(i) * NET_DEG + k];
            const double gk = a.g[size_t(i) * NET_DEG + k];
            dg += gk;
            if (net_class(a.pos[3 * j], a) == 1) b += gk * a.dV;
        }
        a.cls[i] = ci;
        const bool fr = ci == 0;
        const double r = fr ? b : 0.0;
        const double z = (fr && dg > 0.0) ? r / dg : 0.0;
        a.diag[i] = dg;
        a.V[i] = ci == 1 ? a.dV : 0.0;
        a.r[i] = r;
        a.z[i] = z;
        P[i] = z;
        s0[0] += r * z;
        s0[1] += r * r;
        maxdeg = max(maxdeg, d);
        nsrc += ci == 1;
        nsnk += ci == 2;
        dsum += dk;  // the stored edges (a degree above NET_DEG is rejected)
    }
    atomicMax(&a.cnt[0], maxdeg);
    atomicAdd(&a.cnt[1], nsrc);
    atomicAdd(&a.cnt[2], nsnk);
    atomicAdd(&a.cnt[3], dsum);
    wg_sum(s0, sh);  // its barriers also publish cls
    double rz = s0[0], rr = s0[1];
    const double bb = s0[1], stop2 = a.tol * a.tol * bb;
    int it = 0;
    while (it < a.max_iter && rr > stop2) {
        // q = A p on the free beads (p is zero on the electrode beads)
        double pq[1] = {0.0};
        for (int i = threadIdx.x; i < n; i += NET_CG) {
            double q = 0.0;
            if (a.cls[i] == 0) {
                const int dk = min(a.deg[i], NET_DEG);
                const int *nb = a.nbr + size_t(i) * NET_DEG;
                const double *gi = a.g + size_t(i) * NET_DEG;
                double off = 0.0;
                int k = 0;
                // four edges' index and conductance loads in flight at a time,
                // added in edge order
                for (; k + 4 <= dk; k += 4) {
                    const int j0 = nb[k], j1 = nb[k + 1], j2 = nb[k + 2], j3 = nb[k + 3];
                    const double g0 = gi[k], g1 = gi[k + 1], g2 = gi[k + 2], g3 = gi[k + 3];
                    off += g0 * P[j0];
                    off += g1 * P[j1];
                    off += g2 * P[j2];
                    off += g3 * P[j3];
                }
                for (; k < dk; ++k) off += gi[k] * P[nb[k]];
                q = a.diag[i] * P[i] - off;
            }
            a.q[i] = q;
            pq[0] += P[i] * q;
        }
        wg_sum(pq, sh);
        if (!(pq[0] > 0.0)) break;  // same value in every thread
        const double alpha = rz / pq[0];
        double s1[2] = {0.0, 0.0};
        for (int i = threadIdx.x; i < n; i += NET_CG) {
            if (a.cls[i] != 0) continue;
            const double r = a.r[i] - alpha * a.q[i];
            const double dg = a.diag[i];
            const double z = dg > 0.0 ? r / dg : 0.0;
            a.V[i] += alpha * P[i];
            a.r[i] = r;
            a.z[i] = z;
            s1[0] += r * z;
            s1[1] += r * r;
        }
        wg_sum(s1, sh);
        const double beta = rz > 0.0 ? s1[0] / rz : 0.0;
        rz = s1[0];
        rr = s1[1];
        for (int i = threadIdx.x; i < n; i += NET_CG)
            if (a.cls[i] == 0) P[i] = a.z[i] + beta * P[i];
        __syncthreads();  // the next product reads every bead's p
        ++it;
    }
    __syncthreads();  // every potential written
    // Eq. 15 and the current leaving the source electrode
    double st[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += NET_CG) {
        const int ci = a.cls[i];
        const int dk = min(a.deg[i], NET_DEG);
        const double Vi = a.V[i];
        double s = 0.0;
        for (int k = 0; k < dk; ++k) {
            const int j = a.nbr[size_t(i) * NET_DEG + k];
            const double e = a.g[size_t(i) * NET_DEG + k] * (Vi - a.V[j]);
            s += fabs(e);
            if (ci == 1 && a.cls[j] != 1) st[0] += e;
        }
        a.I[i] = 0.5 * s;
    }
    wg_sum(st, sh);
    if (threadIdx.x == 0) {
        a.out[0] = st[0];
        a.out[1] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
        a.out[2] = double(it);
    }
}

// bead j of rod r: X + t e, t from -h to +h in nb - 1 equal steps
__global__ void rod_beads_kernel(const double *rods, int n_rods, int nb, double half, double *pos) {
    const int t = blockIdx.x * blockDim.x + int(threadIdx.x);
    if (t >= n_rods * nb) return;
    const int r = t / nb, j = t - r * nb;
    const double *rod = rods + size_t(r) * ROD_STRIDE;
    const double w = rod[ROD_Q], x = rod[ROD_Q + 1], y = rod[ROD_Q + 2], z = rod[ROD_Q + 3];
    const double e[3] = {2.0 * (x * z + w * y), 2.0 * (y * z - w * x), 1.0 - 2.0 * (x * x + y * y)};
    const double s = -half + 2.0 * half * j / (nb - 1);
#pragma unroll
    for (int d = 0; d < 3; ++d) pos[3 * size_t(t) + d] = rod[ROD_X + d] + s * e[d];
}

}  // namespace

hipError_t launch_net_edges(const NetArgs &a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(net_edges_kernel, dim3((a.n + NET_TB - 1) / NET_TB), dim3(NET_TB), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_net_solve(const NetArgs &a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    if (a.n <= NET_LDS_P)
        hipLaunchKernelGGL(net_solve_kernel<true>, dim3(1), dim3(NET_CG), size_t(a.n) * sizeof(double), s, a);
    else
        hipLaunchKernelGGL(net_solve_kernel<false>, dim3(1), dim3(NET_CG), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_rod_beads(const double *rods, int n_rods, int nb, double half, double *pos, hipStream_t s) {
    const int n = n_rods * nb;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(rod_beads_kernel, dim3((n + 255) / 256), dim3(256), 0, s, rods, n_rods, nb, half, pos);
    return hipGetLastError();
}

}  // namespace lbm
