// Auxiliary kernels of liblbm: initial populations, wall flags, bounce-back
// slot fill, FP64 export and FP64 observables reductions.
#include <type_traits>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

namespace {

// f*(t = 0) = w_i rho_k on fluid nodes (the fluid at rest), stored as the
// deviation w_i (rho_k - rref_k) rounded once from FP64; slots of non-fluid
// nodes start at zero deviation and are filled by slot_fill_kernel.
template <class S>
__global__ void init_pop_kernel(S *f, int64_t fs, const double *rho, const uint8_t *mat, int64_t n, double r0,
                                double r1) {
    using C = typename Codec<S>::C;
    const double rr[2] = {r0, r1};
    for (int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; p < n; p += int64_t(gridDim.x) * blockDim.x) {
        const bool fl = (mat[p] & MAT_ID_MASK) == MAT_FLUID;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const double rk = fl ? rho[k * n + p] : rr[k];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const double d = wgt<double>(i) * (rk - rr[k]);
                f[(k * Q + i) * fs + p] = Codec<S>::enc(C(d));
            }
        }
    }
}

// evaporation sink: liquid fluid nodes (rho_A > rho_B, FP64 sums of the
// stored populations) per column into chunk slot 0 of h; slots 1 .. nz-1
// cleared, so that any z-chunk count of the next step reads the full height
template <class S>
__global__ void sink_heights_kernel(const S *f, int64_t fs, const uint8_t *mat, int nx, int ny, int nz, double r0,
                                    double r1, int32_t *h) {
    const int64_t nxy = int64_t(nx) * ny;
    const double rr[2] = {r0, r1};
    for (int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; c < nxy; c += int64_t(gridDim.x) * blockDim.x) {
        int cnt = 0;
        for (int z = 0; z < nz; ++z) {
            const int64_t p = z * nxy + c;
            if (z) h[p] = 0;
            if ((mat[p] & MAT_ID_MASK) != MAT_FLUID) continue;
            double rho[2];
            for (int k = 0; k < 2; ++k) {
                double sum = 0.0;
                for (int i = 0; i < Q; ++i) sum += double(Codec<S>::dec(f[(k * Q + i) * fs + p])) + wgt<double>(i) * rr[k];
                rho[k] = sum;
            }
            cnt += rho[0] > rho[1] ? 1 : 0;
        }
        h[c] = cnt;
    }
}

__device__ inline int wrapc(int v, int n, int per) {
    if (per) return v < 0 ? v + n : (v >= n ? v - n : v);
    return min(max(v, 0), n - 1);
}

// mark fluid nodes that have a static-wall neighbour
__global__ void flags_kernel(uint8_t *mat, int nx, int ny, int nz, int px, int py, int pz) {
    const int64_t n = int64_t(nx) * ny * nz;
    for (int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; p < n; p += int64_t(gridDim.x) * blockDim.x) {
        uint8_t m = mat[p] & MAT_ID_MASK;
        if (m == MAT_FLUID) {
            const int x = p % nx, y = (p / nx) % ny, z = p / (int64_t(nx) * ny);
            bool near = false;
            for (int j = 1; j < Q; ++j) {
                const int xx = wrapc(x + cx(j), nx, px), yy = wrapc(y + cy(j), ny, py), zz = wrapc(z + cz(j), nz, pz);
                const uint8_t q = mat[(int64_t(zz) * ny + yy) * nx + xx] & MAT_ID_MASK;
                near |= is_static_wall(q);
            }
            if (near) m |= MAT_NEAR_WALL;
        }
        mat[p] = (mat[p] & MAT_ID_MASK) | (m & MAT_NEAR_WALL);
    }
}

// bounce-back slots for the current state: wall node x + c_j gets f*_j(x) as direction opp(j)
template <class S>
__global__ void slot_fill_kernel(S *f, int64_t fs, const uint8_t *mat, int nx, int ny, int nz, int px, int py,
                                 int pz) {
    const int64_t n = int64_t(nx) * ny * nz;
    for (int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; p < n; p += int64_t(gridDim.x) * blockDim.x) {
        if (!(mat[p] & MAT_NEAR_WALL)) continue;
        const int x = p % nx, y = (p / nx) % ny, z = p / (int64_t(nx) * ny);
        for (int j = 1; j < Q; ++j) {
            const int xx = wrapc(x + cx(j), nx, px), yy = wrapc(y + cy(j), ny, py), zz = wrapc(z + cz(j), nz, pz);
            const int64_t q = (int64_t(zz) * ny + yy) * nx + xx;
            if (!is_static_wall(mat[q] & MAT_ID_MASK)) continue;
            // opposite directions share the weight, hence the deviation offset:
            // the stored value is copied unchanged
            for (int k = 0; k < 2; ++k) f[(k * Q + opp(j)) * fs + q] = f[(k * Q + j) * fs + p];
        }
    }
}

template <class S>
__global__ void export_kernel(const S *f, int64_t fs, const uint8_t *mat, int64_t n, double r0, double r1,
                              double *rho_out, double *f_out) {
    const double rr[2] = {r0, r1};
    for (int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; p < n; p += int64_t(gridDim.x) * blockDim.x) {
        const bool fl = (mat[p] & MAT_ID_MASK) == MAT_FLUID;
        for (int k = 0; k < 2; ++k) {
            double s = 0.0;
            for (int i = 0; i < Q; ++i) {
                const double v = fl ? double(Codec<S>::dec(f[(k * Q + i) * fs + p])) + wgt<double>(i) * rr[k] : 0.0;
                s += v;
                if (f_out) f_out[(k * Q + i) * n + p] = v;
            }
            if (rho_out) rho_out[k * n + p] = s;
        }
    }
}

__device__ inline double block_sum(double v, double *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < int(blockDim.x >> 6); ++q) s += sh[q];
    return s;
}
__device__ inline double block_max(double v, double *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < int(blockDim.x >> 6); ++q) s = fmax(s, sh[q]);
    return s;
}

// pass 1: per-block FP64 partials [block][OBS_FIELDS]
template <class S>
__global__ void __launch_bounds__(256) obs_partial_kernel(const S *f, int64_t fs, const uint8_t *mat, int64_t n,
                                                          double r0, double r1, double *partials) {
    __shared__ double sh[4];
    const double rr[2] = {r0, r1};
    double acc[OBS_FIELDS];
    for (int q = 0; q < OBS_FIELDS; ++q) acc[q] = 0.0;
    for (int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; p < n; p += int64_t(gridDim.x) * blockDim.x) {
        if ((mat[p] & MAT_ID_MASK) != MAT_FLUID) continue;
        double rho[2], j[3] = {0, 0, 0};
        for (int k = 0; k < 2; ++k) {
            double s = 0.0;
            for (int i = 0; i < Q; ++i) {
                const double v = double(Codec<S>::dec(f[(k * Q + i) * fs + p])) + wgt<double>(i) * rr[k];
                s += v;
                j[0] += cx(i) * v;
                j[1] += cy(i) * v;
                j[2] += cz(i) * v;
            }
            rho[k] = s;
        }
        acc[0] += rho[0];
        acc[1] += rho[1];
        acc[4] += j[0];
        acc[5] += j[1];
        acc[6] += j[2];
        const double tot = rho[0] + rho[1];
        const double j2 = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
        if (tot > 0) {
            acc[7] = fmax(acc[7], sqrt(j2) / tot);
            acc[8] += 0.5 * j2 / tot;
        }
        acc[9] += 1.0;
    }
    for (int q = 0; q < OBS_FIELDS; ++q) {
        const double v = (q == 7) ? block_max(acc[q], sh) : block_sum(acc[q], sh);
        if (threadIdx.x == 0) partials[blockIdx.x * OBS_FIELDS + q] = v;
    }
}

// fold the per-tile ledger slots into the carry (fixed order) and clear them
__global__ void fold_ledger_kernel(double *ledger_part, int nslots, double *carry) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s0 = carry[0], s1 = carry[1];
    for (int t = 0; t < nslots; ++t) {
        s0 += ledger_part[2 * t];
        s1 += ledger_part[2 * t + 1];
        ledger_part[2 * t] = 0.0;
        ledger_part[2 * t + 1] = 0.0;
    }
    carry[0] = s0;
    carry[1] = s1;
}

// pass 2: one block sums the partials in a fixed order (deterministic)
__global__ void obs_final_kernel(const double *partials, int nblocks, const double *ledger_part, int nledger,
                                 const double *carry, double *result) {
    if (threadIdx.x != 0) return;
    double r[OBS_FIELDS];
    for (int q = 0; q < OBS_FIELDS; ++q) r[q] = 0.0;
    for (int b = 0; b < nblocks; ++b)
        for (int q = 0; q < OBS_FIELDS; ++q) {
            const double v = partials[b * OBS_FIELDS + q];
            r[q] = (q == 7) ? fmax(r[q], v) : r[q] + v;
        }
    r[2] = carry[0];
    r[3] = carry[1];
    for (int t = 0; t < nledger; ++t) {
        r[2] += ledger_part[2 * t];
        r[3] += ledger_part[2 * t + 1];
    }
    for (int q = 0; q < OBS_FIELDS; ++q) result[q] = r[q];
}

int grid_for(int64_t n, int bs) {
    int64_t g = (n + bs - 1) / bs;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return int(g);
}

}  // namespace

template <class F>
static hipError_t by_prec(int prec, F &&fn) {
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

hipError_t launch_init_populations(int prec, void *f, int64_t fs, const double *rho, const uint8_t *mat, int64_t n,
                                   const double rho_ref[2], hipStream_t s) {
    return by_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(init_pop_kernel<S>, dim3(grid_for(n, 256)), dim3(256), 0, s, static_cast<S *>(f), fs, rho,
                           mat, n, rho_ref[0], rho_ref[1]);
        return hipGetLastError();
    });
}

hipError_t launch_flags(uint8_t *mat, int nx, int ny, int nz, const int per[3], hipStream_t s) {
    const int64_t n = int64_t(nx) * ny * nz;
    hipLaunchKernelGGL(flags_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, mat, nx, ny, nz, per[0], per[1], per[2]);
    return hipGetLastError();
}

hipError_t launch_slot_fill(int prec, void *f, int64_t fs, const uint8_t *mat, int nx, int ny, int nz,
                            const int per[3], hipStream_t s) {
    const int64_t n = int64_t(nx) * ny * nz;
    return by_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(slot_fill_kernel<S>, dim3(grid_for(n, 256)), dim3(256), 0, s, static_cast<S *>(f), fs, mat,
                           nx, ny, nz, per[0], per[1], per[2]);
        return hipGetLastError();
    });
}

hipError_t launch_export(int prec, const void *f, int64_t fs, const uint8_t *mat, int64_t n, const double rho_ref[2],
                         double *rho_out, double *f_out, hipStream_t s) {
    return by_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(export_kernel<S>, dim3(grid_for(n, 256)), dim3(256), 0, s, static_cast<const S *>(f), fs,
                           mat, n, rho_ref[0], rho_ref[1], rho_out, f_out);
        return hipGetLastError();
    });
}

hipError_t launch_sink_heights(int prec, const void *f, int64_t fs, const uint8_t *mat, int nx, int ny, int nz,
                               const double rho_ref[2], int32_t *h, hipStream_t s) {
    const int64_t nxy = int64_t(nx) * ny;
    return by_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(sink_heights_kernel<S>, dim3(grid_for(nxy, 256)), dim3(256), 0, s, static_cast<const S *>(f),
                           fs, mat, nx, ny, nz, rho_ref[0], rho_ref[1], h);
        return hipGetLastError();
    });
}

hipError_t launch_fold_ledger(double *ledger_part, int nslots, double *carry, hipStream_t s) {
    hipLaunchKernelGGL(fold_ledger_kernel, dim3(1), dim3(64), 0, s, ledger_part, nslots, carry);
    return hipGetLastError();
}

hipError_t launch_observables(int prec, const void *f, int64_t fs, const uint8_t *mat, int64_t n,
                              const double rho_ref[2], const double *ledger_part, int nledger,
                              const double *ledger_carry, double *partials, int nblocks, double *result,
                              hipStream_t s) {
    hipError_t e = by_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(obs_partial_kernel<S>, dim3(nblocks), dim3(256), 0, s, static_cast<const S *>(f), fs, mat,
                           n, rho_ref[0], rho_ref[1], partials);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(obs_final_kernel, dim3(1), dim3(64), 0, s, partials, nblocks, ledger_part, nledger,
                       ledger_carry, result);
    return hipGetLastError();
}

}  // namespace lbm
