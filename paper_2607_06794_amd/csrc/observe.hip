// Droplet and deposit observables (gfx950).
//
// Droplet shape: colour C = (rho_A - rho_B) / (rho_A + rho_B) on fluid nodes
// (liquid C > 0).  One thread per (x, y) column scans down from the top for
// the topmost wet node and interpolates the C = 0 crossing above it (column
// height above the wall surface z = 1/2); the droplet height is the largest
// column height.  The footprint half-lengths are the runs of C > 0 on the
// first fluid plane through the given centre, ends interpolated at C = 0, and
// the contact angles follow from the spherical-cap relation
// theta = 2 atan(h / r) (Results, drying dynamics: h, r_x, r_y, theta_x,
// theta_y; the paper leaves the extraction open).
//
// Deposit statistics of the rods (Methods, structural characterisation):
// beads evenly spaced along each axis segment and the segments between them;
// g^b (Eq. 14) = bead count over the mean bead count per bin, S_x^b (Eq. 13)
// = mean of 2 cos^2(zeta) - 1 over the segments whose midpoints fall in the
// bin; axial profiles bin x inside a central strip in y, transverse profiles
// bin y inside a central strip in x.  Per-bin sums run over rods and segments
// in index order, so they are deterministic.
//
// Contact graph (Methods, electrical network model): rods connect when their
// axis segments are closer than r_c; clusters by synchronous minimum-label
// propagation over a shared-memory adjacency bitmap (labels converge to the
// smallest rod index of each cluster); a cluster spans when it reaches both
// x < x_src and x > x_snk.
#include <math.h>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

namespace {

template <class S>
__device__ inline double colour_at(const S *f, int64_t fs, const uint8_t *mat, int64_t n, double r0, double r1) {
    if ((mat[n] & MAT_ID_MASK) != MAT_FLUID) return NAN;
    double rho[2];
    const double rr[2] = {r0, r1};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) s += double(Codec<S>::dec(f[(k * Q + i) * fs + n])) + wgt<double>(i) * rr[k];
        rho[k] = s;
    }
    const double tot = rho[0] + rho[1];
    return tot > 0.0 ? (rho[0] - rho[1]) / tot : NAN;
}

template <class S>
__global__ void column_height_kernel(ObsArgs o, const S *f) {
    const int64_t ncol = int64_t(o.nx) * o.ny;
    for (int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; c < ncol; c += int64_t(gridDim.x) * blockDim.x) {
        const int x = int(c % o.nx), y = int(c / o.nx);
        double h = 0.0, above = NAN;
        int wet = 0;
        bool found = false;
        for (int z = o.nz - 1; z >= 0; --z) {
            const double cz = colour_at(f, o.fs, o.mat, int64_t(z) * ncol + c, o.rho_ref[0], o.rho_ref[1]);
            if (cz > 0.0) {
                ++wet;
                if (!found && z >= 1) {
                    found = true;
                    const double frac = (z + 1 < o.nz && !isnan(above)) ? cz / (cz - above) : 0.5;
                    h = (double(z) + frac) - 0.5;
                }
            }
            above = cz;
            if (z == 1) {
                if (y == o.iy) o.line_x[x] = cz;
                if (x == o.ix) o.line_y[y] = cz;
            }
        }
        o.col_h[c] = h;
        o.col_wet[c] = wet;
    }
}

__device__ double run_half_length(const double *line, int n, int centre) {
    if (!(line[centre] > 0.0)) return 0.0;
    int lo = centre, hi = centre;
    while (lo - 1 >= 0 && line[lo - 1] > 0.0) --lo;
    while (hi + 1 < n && line[hi + 1] > 0.0) ++hi;
    double left = lo - 0.5, right = hi + 0.5;
    if (lo - 1 >= 0 && !isnan(line[lo - 1])) left = lo - line[lo] / (line[lo] - line[lo - 1]);
    if (hi + 1 < n && !isnan(line[hi + 1])) right = hi + line[hi] / (line[hi] - line[hi + 1]);
    return 0.5 * (right - left);
}

__global__ void __launch_bounds__(1024) shape_final_kernel(ObsArgs o) {
    __shared__ double smax[16];
    __shared__ long long swet[16];
    const int64_t ncol = int64_t(o.nx) * o.ny;
    double hm = 0.0;
    long long wet = 0;
    for (int64_t c = threadIdx.x; c < ncol; c += blockDim.x) {
        hm = fmax(hm, o.col_h[c]);
        wet += o.col_wet[c];
    }
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) {
        hm = fmax(hm, __shfl_xor(hm, s, 64));
        wet += __shfl_xor(wet, s, 64);
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) {
        smax[w] = hm;
        swet[w] = wet;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < int(blockDim.x >> 6); ++q) {
            hm = fmax(hm, smax[q]);
            wet += swet[q];
        }
        const double rx = run_half_length(o.line_x, o.nx, o.ix);
        const double ry = run_half_length(o.line_y, o.ny, o.iy);
        o.out[0] = hm;
        o.out[1] = rx;
        o.out[2] = ry;
        o.out[3] = rx > 0.0 ? 2.0 * atan2(hm, rx) : 0.0;
        o.out[4] = ry > 0.0 ? 2.0 * atan2(hm, ry) : 0.0;
        o.out[5] = double(wet);
    }
}

// ---------------------------------------------------------------------------
// deposit profiles
// ---------------------------------------------------------------------------
__device__ inline double min_img1(double d, double box, int per) { return per ? d - box * rint(d / box) : d; }
__device__ inline double wrap1d(double v, double n) { return v - n * floor(v / n); }
__device__ inline int bin_of(double v, double n, int nb) {
    const int b = int(floor(wrap1d(v, n) * nb / n));
    return b < nb - 1 ? b : nb - 1;
}
__device__ inline void rod_axis(const double *q, double e[3]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    e[0] = 2.0 * (x * z + w * y);
    e[1] = 2.0 * (y * z - w * x);
    e[2] = 1.0 - 2.0 * (x * x + y * y);
}

// one work-group; thread r bins rod r's beads and segments, then thread b
// sums bin b over rods and segments in index order
__global__ void __launch_bounds__(LB_MAX_RODS) deposit_kernel(DepArgs d) {
    const int r = threadIdx.x;
    const double nx = d.nx, ny = d.ny;
    if (r < d.n_rods) {
        const double *rod = d.rods + r * ROD_STRIDE;
        double e[3];
        rod_axis(rod + ROD_Q, e);
        double X[3] = {rod[ROD_X], rod[ROD_X + 1], rod[ROD_X + 2]};
        // mirror image at the droplet centre (the rod is symmetric end to end)
        if (d.mirror_x) {
            X[0] = 2.0 * d.xc - X[0];
            e[0] = -e[0];
        }
        if (d.mirror_y) {
            X[1] = 2.0 * d.yc - X[1];
            e[1] = -e[1];
        }
        int16_t *bx = d.bins + size_t(r) * DEP_NB * 4;
        int16_t *by = bx + DEP_NB, *sx = by + DEP_NB, *sy = sx + DEP_NB;
        double prev[3] = {0, 0, 0};
        for (int j = 0; j < d.nb; ++j) {
            const double t = -d.half + 2.0 * d.half * j / (d.nb - 1);
            const double p[3] = {X[0] + t * e[0], X[1] + t * e[1], X[2] + t * e[2]};
            const bool ax = fabs(min_img1(p[1] - d.yc, ny, d.py)) <= 0.5 * d.strip_y;
            const bool tr = fabs(min_img1(p[0] - d.xc, nx, d.px)) <= 0.5 * d.strip_x;
            bx[j] = ax ? int16_t(bin_of(p[0], nx, d.nbx)) : int16_t(-1);
            by[j] = tr ? int16_t(bin_of(p[1], ny, d.nby)) : int16_t(-1);
            if (j > 0) {
                const double m[3] = {0.5 * (prev[0] + p[0]), 0.5 * (prev[1] + p[1]), 0.5 * (prev[2] + p[2])};
                const bool max_in = fabs(min_img1(m[1] - d.yc, ny, d.py)) <= 0.5 * d.strip_y;
                const bool mtr = fabs(min_img1(m[0] - d.xc, nx, d.px)) <= 0.5 * d.strip_x;
                sx[j - 1] = max_in ? int16_t(bin_of(m[0], nx, d.nbx)) : int16_t(-1);
                sy[j - 1] = mtr ? int16_t(bin_of(m[1], ny, d.nby)) : int16_t(-1);
            }
            prev[0] = p[0];
            prev[1] = p[1];
            prev[2] = p[2];
        }
        d.sval[r] = 2.0 * e[0] * e[0] - 1.0;
    }
    __syncthreads();
    // bins: threads [0, nbx) axial, [nbx, nbx + nby) transverse
    const int t = threadIdx.x;
    const bool axial = t < d.nbx;
    const int b = axial ? t : t - d.nbx;
    if (t < d.nbx + d.nby) {
        long long cnt = 0, nseg = 0;
        double ssum = 0.0;
        for (int q = 0; q < d.n_rods; ++q) {
            const int16_t *bx = d.bins + size_t(q) * DEP_NB * 4;
            const int16_t *beadb = axial ? bx : bx + DEP_NB;
            const int16_t *segb = axial ? bx + 2 * DEP_NB : bx + 3 * DEP_NB;
            for (int j = 0; j < d.nb; ++j) cnt += beadb[j] == b;
            for (int j = 0; j + 1 < d.nb; ++j)
                if (segb[j] == b) {
                    ssum += d.sval[q];
                    ++nseg;
                }
        }
        double *out = d.out + (axial ? 0 : 3 * DEP_MAXBIN);
        out[b] = double(cnt);
        out[DEP_MAXBIN + b] = nseg > 0 ? ssum / double(nseg) : 0.0;
        out[2 * DEP_MAXBIN + b] = double(nseg);
    }
}

// ---------------------------------------------------------------------------
// contact graph
// ---------------------------------------------------------------------------
struct v3 {
    double x, y, z;
};
__device__ inline v3 operator+(v3 a, v3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline v3 operator-(v3 a, v3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline v3 operator*(double s, v3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline double vdot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// distance between segments [p1, q1], [p2, q2]: the stationary point of the
// squared distance if interior, else the best clamped edge
__device__ double seg_dist(v3 p1, v3 q1, v3 p2, v3 q2) {
    const v3 d1 = q1 - p1, d2 = q2 - p2, r = p1 - p2;
    const double a = vdot(d1, d1), e = vdot(d2, d2), f = vdot(d2, r), c = vdot(d1, r), b = vdot(d1, d2);
    double best = 1e300;
    auto tryst = [&](double s, double t) {
        const v3 dd = (p1 + s * d1) - (p2 + t * d2);
        best = fmin(best, sqrt(vdot(dd, dd)));
    };
    const double den = a * e - b * b;
    if (den > 1e-14 * fmax(a * e, 1e-300)) {
        const double s = (b * f - c * e) / den, t = (a * f - b * c) / den;
        if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0) tryst(s, t);
    }
    for (int k = 0; k < 2; ++k) tryst(k, e == 0.0 ? 0.0 : fmin(fmax((b * k + f) / e, 0.0), 1.0));
    for (int k = 0; k < 2; ++k) tryst(a == 0.0 ? 0.0 : fmin(fmax((b * k - c) / a, 0.0), 1.0), k);
    return best;
}

__global__ void __launch_bounds__(LB_MAX_RODS) graph_kernel(DepArgs d) {
    constexpr int W = LB_MAX_RODS / 64;
    __shared__ unsigned long long adj[LB_MAX_RODS][W];
    __shared__ int lab[2][LB_MAX_RODS];
    __shared__ int size[LB_MAX_RODS];
    __shared__ int edges, largest, spanning;
    __shared__ int changed[2];
    const int n = d.n_rods, a = threadIdx.x;
    for (int w = 0; w < W; ++w) adj[a][w] = 0ull;
    lab[0][a] = a;
    size[a] = 0;
    if (a == 0) edges = largest = spanning = changed[0] = changed[1] = 0;
    __syncthreads();
    const double box[3] = {double(d.nx), double(d.ny), double(d.nz)};
    const int per[3] = {d.px, d.py, d.pz};
    if (a < n) {
        const double *ra = d.rods + a * ROD_STRIDE;
        double ea[3];
        rod_axis(ra + ROD_Q, ea);
        const v3 Xa = {ra[ROD_X], ra[ROD_X + 1], ra[ROD_X + 2]}, Ea = {ea[0], ea[1], ea[2]};
        const v3 pa = Xa - d.half * Ea, qa = Xa + d.half * Ea;
        for (int b = a + 1; b < n; ++b) {
            const double *rb = d.rods + b * ROD_STRIDE;
            double eb[3];
            rod_axis(rb + ROD_Q, eb);
            const double dx[3] = {min_img1(rb[ROD_X] - ra[ROD_X], box[0], per[0]),
                                  min_img1(rb[ROD_X + 1] - ra[ROD_X + 1], box[1], per[1]),
                                  min_img1(rb[ROD_X + 2] - ra[ROD_X + 2], box[2], per[2])};
            const v3 Xb = Xa + v3{dx[0], dx[1], dx[2]}, Eb = {eb[0], eb[1], eb[2]};
            if (seg_dist(pa, qa, Xb - d.half * Eb, Xb + d.half * Eb) < d.r_contact) {
                atomicOr(&adj[a][b >> 6], 1ull << (b & 63));
                atomicOr(&adj[b][a >> 6], 1ull << (a & 63));
                atomicAdd(&edges, 1);
            }
        }
    }
    __syncthreads();
    // synchronous minimum-label propagation; the change flag is double
    // buffered so that every thread reads the same value before it is reset
    int cur = 0;
    for (int it = 0; it <= n; ++it) {
        const int par = it & 1;
        int m = lab[cur][a];
        if (a < n)
            for (int w = 0; w < W; ++w) {
                unsigned long long bits = adj[a][w];
                while (bits) {
                    const int b = w * 64 + __builtin_ctzll(bits);
                    bits &= bits - 1;
                    m = min(m, lab[cur][b]);
                }
            }
        lab[cur ^ 1][a] = m;
        if (m != lab[cur][a]) changed[par] = 1;
        __syncthreads();
        const bool go = changed[par] != 0;
        if (a == 0) changed[par ^ 1] = 0;
        __syncthreads();
        cur ^= 1;
        if (!go) break;
    }
    if (a < n) atomicAdd(&size[lab[cur][a]], 1);
    __syncthreads();
    if (a < n && lab[cur][a] == a) {
        atomicMax(&largest, size[a]);
        double lo = 1e300, hi = -1e300;
        for (int b = 0; b < n; ++b) {
            if (lab[cur][b] != a) continue;
            const double *rb = d.rods + b * ROD_STRIDE;
            double eb[3];
            rod_axis(rb + ROD_Q, eb);
            lo = fmin(lo, rb[ROD_X] - d.half * fabs(eb[0]));
            hi = fmax(hi, rb[ROD_X] + d.half * fabs(eb[0]));
        }
        if (lo < d.x_src && hi > d.x_snk) atomicOr(&spanning, 1);
    }
    __syncthreads();
    if (a < n) d.labels[a] = lab[cur][a];
    if (a == 0) {
        d.graph[0] = n;
        d.graph[1] = edges;
        d.graph[2] = largest;
        d.graph[3] = spanning;
    }
}

__global__ void rod_map_kernel(const uint8_t *mat, int nx, int ny, int nz, int32_t *map) {
    const int64_t ncol = int64_t(nx) * ny;
    for (int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; c < ncol; c += int64_t(gridDim.x) * blockDim.x) {
        int cnt = 0;
        for (int z = 0; z < nz; ++z) cnt += (mat[int64_t(z) * ncol + c] & MAT_ID_MASK) == MAT_ROD;
        map[c] = cnt;
    }
}

int grid_cols(int64_t ncol) {
    const int64_t g = (ncol + 255) / 256;
    return int(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

// Shan-Chen equation of state at probe nodes: p = c_s^2 (rho_A + rho_B) +
// G c_s^2 psi_A psi_B with psi = rho on fluid nodes; NaN at non-fluid probes
template <class S>
__global__ void pressure_probe_kernel(const S *f, int64_t fs, const uint8_t *mat, int nx, int ny, int nz, double r0,
                                      double r1, double G, const int *xyz, int n, double *out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int x = xyz[3 * q], y = xyz[3 * q + 1], z = xyz[3 * q + 2];
    const int64_t node = (int64_t(z) * ny + y) * nx + x;
    if ((mat[node] & MAT_ID_MASK) != MAT_FLUID) {
        out[q] = __builtin_nan("");
        return;
    }
    const double rr[2] = {r0, r1};
    double rho[2];
    for (int k = 0; k < 2; ++k) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i) s += double(Codec<S>::dec(f[(k * Q + i) * fs + node])) + wgt<double>(i) * rr[k];
        rho[k] = s;
    }
    out[q] = (rho[0] + rho[1]) / 3.0 + G / 3.0 * rho[0] * rho[1];
}

hipError_t launch_droplet(int prec, const void *f, const ObsArgs &o, hipStream_t s) {
    const int64_t ncol = int64_t(o.nx) * o.ny;
    hipError_t e;
    switch (prec) {
        case LB_F64:
            hipLaunchKernelGGL(column_height_kernel<double>, dim3(grid_cols(ncol)), dim3(256), 0, s, o,
                               static_cast<const double *>(f));
            break;
        case LB_F32:
            hipLaunchKernelGGL(column_height_kernel<float>, dim3(grid_cols(ncol)), dim3(256), 0, s, o,
                               static_cast<const float *>(f));
            break;
        case LB_F16DEV:
            hipLaunchKernelGGL(column_height_kernel<_Float16>, dim3(grid_cols(ncol)), dim3(256), 0, s, o,
                               static_cast<const _Float16 *>(f));
            break;
        case LB_BF16DEV:
            hipLaunchKernelGGL(column_height_kernel<bf16_t>, dim3(grid_cols(ncol)), dim3(256), 0, s, o,
                               static_cast<const bf16_t *>(f));
            break;
        default:
            return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(shape_final_kernel, dim3(1), dim3(1024), 0, s, o);
    return hipGetLastError();
}

// one image's profiles into the ensemble sums: Eq. 14 normalises the bead
// counts by their mean over the bins (summed in bin order by one thread);
// Eq. 13's bin means enter only where the image has segments
__global__ void __launch_bounds__(2 * DEP_MAXBIN) deposit_accumulate_kernel(const double *out, int nbx, int nby,
                                                                           double *acc) {
    __shared__ double mean[2];
    if (threadIdx.x < 2) {
        const int d = threadIdx.x, nb = d ? nby : nbx;
        const double *cnt = out + d * 3 * DEP_MAXBIN;
        double t = 0.0;
        for (int b = 0; b < nb; ++b) t += cnt[b];
        mean[d] = t / nb;
    }
    __syncthreads();
    const int d = threadIdx.x >= DEP_MAXBIN, b = threadIdx.x - d * DEP_MAXBIN;
    if (b >= (d ? nby : nbx)) return;
    const double *o = out + d * 3 * DEP_MAXBIN;
    const double nseg = o[2 * DEP_MAXBIN + b];
    acc[d * DEP_MAXBIN + b] += mean[d] > 0.0 ? o[b] / mean[d] : 0.0;
    acc[(2 + d) * DEP_MAXBIN + b] += nseg > 0.0 ? o[DEP_MAXBIN + b] : 0.0;
    acc[(4 + d) * DEP_MAXBIN + b] += nseg > 0.0 ? 1.0 : 0.0;
    acc[(6 + d) * DEP_MAXBIN + b] += nseg;
}

__global__ void __launch_bounds__(2 * DEP_MAXBIN) deposit_finish_kernel(const double *acc, int nbx, int nby,
                                                                       int images, double *out) {
    const int d = threadIdx.x >= DEP_MAXBIN, b = threadIdx.x - d * DEP_MAXBIN;
    if (b >= (d ? nby : nbx)) return;
    const double c = acc[(4 + d) * DEP_MAXBIN + b];
    double *o = out + d * 3 * DEP_MAXBIN;
    o[b] = acc[d * DEP_MAXBIN + b] / images;
    o[DEP_MAXBIN + b] = c > 0.0 ? acc[(2 + d) * DEP_MAXBIN + b] / c : 0.0;
    o[2 * DEP_MAXBIN + b] = acc[(6 + d) * DEP_MAXBIN + b];
}

hipError_t launch_deposit_accumulate(const DepArgs &d, double *acc, hipStream_t s) {
    hipLaunchKernelGGL(deposit_kernel, dim3(1), dim3(LB_MAX_RODS), 0, s, d);
    hipLaunchKernelGGL(deposit_accumulate_kernel, dim3(1), dim3(2 * DEP_MAXBIN), 0, s, d.out, d.nbx, d.nby, acc);
    return hipGetLastError();
}

hipError_t launch_deposit_finish(const double *acc, int nbx, int nby, int images, double *out, hipStream_t s) {
    hipLaunchKernelGGL(deposit_finish_kernel, dim3(1), dim3(2 * DEP_MAXBIN), 0, s, acc, nbx, nby, images, out);
    return hipGetLastError();
}

hipError_t launch_deposit(const DepArgs &d, hipStream_t s) {
    hipLaunchKernelGGL(deposit_kernel, dim3(1), dim3(LB_MAX_RODS), 0, s, d);
    hipLaunchKernelGGL(graph_kernel, dim3(1), dim3(LB_MAX_RODS), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_rod_map(const uint8_t *mat, int nx, int ny, int nz, int32_t *map, hipStream_t s) {
    hipLaunchKernelGGL(rod_map_kernel, dim3(grid_cols(int64_t(nx) * ny)), dim3(256), 0, s, mat, nx, ny, nz, map);
    return hipGetLastError();
}

hipError_t launch_pressure(int prec, const void *f, int64_t fs, const uint8_t *mat, int nx, int ny, int nz,
                           const double rref[2], double G, const int *xyz, int n, double *out, hipStream_t s) {
    const dim3 grid((n + 255) / 256);
    switch (prec) {
        case LB_F64:
            hipLaunchKernelGGL(pressure_probe_kernel<double>, grid, dim3(256), 0, s, static_cast<const double *>(f), fs,
                               mat, nx, ny, nz, rref[0], rref[1], G, xyz, n, out);
            break;
        case LB_F32:
            hipLaunchKernelGGL(pressure_probe_kernel<float>, grid, dim3(256), 0, s, static_cast<const float *>(f), fs, mat,
                               nx, ny, nz, rref[0], rref[1], G, xyz, n, out);
            break;
        case LB_F16DEV:
            hipLaunchKernelGGL(pressure_probe_kernel<_Float16>, grid, dim3(256), 0, s, static_cast<const _Float16 *>(f),
                               fs, mat, nx, ny, nz, rref[0], rref[1], G, xyz, n, out);
            break;
        case LB_BF16DEV:
            hipLaunchKernelGGL(pressure_probe_kernel<bf16_t>, grid, dim3(256), 0, s, static_cast<const bf16_t *>(f), fs,
                               mat, nx, ny, nz, rref[0], rref[1], G, xyz, n, out);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lbm
