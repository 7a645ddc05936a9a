// Learned surrogate (gfx950): restriction of the lattice state to a coarse
// canvas, prolongation and lift back to populations, and the training and
// inference kernels of a 3-D convolutional U-Net.
//
// Convolutions are implicit GEMMs on BF16 MFMA (32 x 32 x 8, FP32
// accumulation).  Tensors are channels-last, [D][H][W][C], C a multiple of 8.
//   forward  y[p, o]  = b[o] + sum_{t, c} x[p + o_t, c] w[t, c, o]
//            M = positions, N = output channels, K = 27 x input channels
//   dgrad    dx[q, c] = sum_{t, o} g[q - o_t, o] w[t, c, o],  g = dy (y > 0)
//            M = positions, N = input channels, K = 27 x output channels
//   wgrad    dw[t, c, o] += sum_p x[p + o_t, c] g[p, o]
//            per tap: M = input channels, N = output channels, K = positions
// A work-group of four wavefronts computes a 64 x 64 output tile, each
// wavefront a 32 x 32 block; K advances in steps of 32 staged through LDS.
// The decoder's inputs are read in place: channels [0, c1) from the coarser
// level through nearest-neighbour upsampling, [c1, c1 + c2) from the skip.
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

__device__ inline uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return static_cast<uint16_t>(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

constexpr int TM = 64, TN = 64, TK = 32;
constexpr int LDA = TK + 8;   // A tile row stride (elements)
constexpr int LDB = TN + 8;   // B tile row stride
constexpr int NTH = 256;

__device__ inline void tap_offset(int t, int &dz, int &dy, int &dx) {
    dz = t / 9 - 1;
    dy = (t / 3) % 3 - 1;
    dx = t % 3 - 1;
}

// 8 consecutive channels [c, c + 8) of the (virtual) input at full-resolution
// position (qd, qh, qw); zeros outside the volume or past cin
__device__ inline void load_in8(const ConvArgs &a, int qd, int qh, int qw, int c, uint16_t out[8]) {
    const int cin = a.c1 + a.c2;
    bool ok = qd >= 0 && qd < a.D && qh >= 0 && qh < a.H && qw >= 0 && qw < a.W && c < cin;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (ok) {
        if (c < a.c1) {
            int64_t idx;
            if (a.up1)
                idx = (int64_t(qd >> 1) * (a.H >> 1) + (qh >> 1)) * (a.W >> 1) + (qw >> 1);
            else
                idx = (int64_t(qd) * a.H + qh) * a.W + qw;
            v = *reinterpret_cast<const uint4 *>(a.x1 + idx * a.c1 + c);
        } else {
            const int64_t idx = (int64_t(qd) * a.H + qh) * a.W + qw;
            v = *reinterpret_cast<const uint4 *>(a.x2 + idx * a.c2 + (c - a.c1));
        }
    }
    const uint16_t *s = reinterpret_cast<const uint16_t *>(&v);
#pragma unroll
    for (int j = 0; j < 8; ++j) out[j] = s[j];
}

// 8 consecutive channels of g = dy (y > 0) (or dy without the ReLU) at p
__device__ inline void load_g8(const ConvArgs &a, const float *dy, int64_t p, int o, bool valid, uint16_t out[8]) {
    if (!valid || o >= a.cout) {
#pragma unroll
        for (int j = 0; j < 8; ++j) out[j] = 0;
        return;
    }
    const float4 g0 = *reinterpret_cast<const float4 *>(dy + p * a.cout + o);
    const float4 g1 = *reinterpret_cast<const float4 *>(dy + p * a.cout + o + 4);
    float g[8] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
    if (a.relu) {
        const uint4 yv = *reinterpret_cast<const uint4 *>(a.y + p * a.cout + o);
        const uint16_t *ys = reinterpret_cast<const uint16_t *>(&yv);
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (!(bf2f(ys[j]) > 0.0f)) g[j] = 0.0f;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) out[j] = f2bf(g[j]);
}

// one 32 x 32 x 32 step of a wavefront from LDS: A[m][k] at sa + m * lda + k
// (or transposed: sa + k * lda + m), B[k][n] at sb + k * ldb + n
template <bool AT>
__device__ inline void mma_step(const uint16_t *sa, int lda, const uint16_t *sb, int ldb, v16f &acc) {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int kk = 0; kk < TK; kk += 8) {
        v4s av, bv;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = kk + 4 * (l >> 5) + i;
            av[i] = AT ? short(sa[k * lda + (l & 31)]) : short(sa[(l & 31) * lda + k]);
            bv[i] = short(sb[k * ldb + (l & 31)]);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
    }
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NTH) conv_fwd_kernel(ConvArgs a) {
    __shared__ uint16_t As[TM * LDA];
    __shared__ uint16_t Bs[TK * LDB];
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
    const int64_t P = int64_t(a.D) * a.H * a.W;
    const int64_t p0 = int64_t(blockIdx.x) * TM;
    const int o0 = blockIdx.y * TN;
    const int cin = a.c1 + a.c2;
    const int m0 = (wv >> 1) * 32, n0 = (wv & 1) * 32;
    v16f acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
    // this thread's A row and B row
    const int ar = tid >> 2, ac = (tid & 3) * 8;
    const int64_t pa = p0 + ar;
    const bool arow = pa < P;
    const int aw = int(pa % a.W), ah = int((pa / a.W) % a.H), ad = int(pa / (int64_t(a.W) * a.H));
    const int br = tid >> 3, bc = (tid & 7) * 8;
    for (int t = 0; t < 27; ++t) {
        int dz, dy, dx;
        tap_offset(t, dz, dy, dx);
        for (int c0 = 0; c0 < cin; c0 += TK) {
            uint16_t va[8];
            if (arow)
                load_in8(a, ad + dz, ah + dy, aw + dx, c0 + ac, va);
            else
#pragma unroll
                for (int j = 0; j < 8; ++j) va[j] = 0;
#pragma unroll
            for (int j = 0; j < 8; ++j) As[ar * LDA + ac + j] = va[j];
            uint4 wb = make_uint4(0, 0, 0, 0);
            if (c0 + br < cin && o0 + bc < a.cout)
                wb = *reinterpret_cast<const uint4 *>(a.w + (int64_t(t) * cin + c0 + br) * a.cout + o0 + bc);
            const uint16_t *wbs = reinterpret_cast<const uint16_t *>(&wb);
#pragma unroll
            for (int j = 0; j < 8; ++j) Bs[br * LDB + bc + j] = wbs[j];
            __syncthreads();
            mma_step<false>(As + m0 * LDA, LDA, Bs + n0, LDB, acc);
            __syncthreads();
        }
    }
    // D element i of lane l: row 8 (i / 4) + 4 (l / 32) + i % 4, column l % 32
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int64_t p = p0 + m0 + 8 * (i >> 2) + 4 * (l >> 5) + (i & 3);
        const int o = o0 + n0 + (l & 31);
        if (p >= P || o >= a.cout) continue;
        float v = acc[i] + (a.b ? a.b[o] : 0.0f);
        if (a.relu) v = fmaxf(v, 0.0f);
        if (a.y) a.y[p * a.cout + o] = f2bf(v);
        if (a.yf) a.yf[p * a.cout + o] = v;
    }
}

// ---------------------------------------------------------------------------
// input gradient
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NTH) conv_dgrad_kernel(ConvArgs a, const float *dy, float *dx) {
    __shared__ uint16_t As[TM * LDA];
    __shared__ uint16_t Bs[TK * LDB];
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
    const int64_t P = int64_t(a.D) * a.H * a.W;
    const int64_t q0 = int64_t(blockIdx.x) * TM;
    const int c0n = blockIdx.y * TN;  // input-channel tile
    const int cin = a.c1 + a.c2;
    const int m0 = (wv >> 1) * 32, n0 = (wv & 1) * 32;
    v16f acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
    const int ar = tid >> 2, ac = (tid & 3) * 8;
    const int64_t qa = q0 + ar;
    const bool arow = qa < P;
    const int aw = int(qa % a.W), ah = int((qa / a.W) % a.H), ad = int(qa / (int64_t(a.W) * a.H));
    // B tile rows are output channels k, columns input channels n: thread loads
    // 8 output channels of one input channel and scatters them down a column
    const int bn = tid >> 2, bk = (tid & 3) * 8;
    for (int t = 0; t < 27; ++t) {
        int dz, dyy, dxx;
        tap_offset(t, dz, dyy, dxx);
        const int sd = ad - dz, sh = ah - dyy, sw = aw - dxx;
        const bool in = arow && sd >= 0 && sd < a.D && sh >= 0 && sh < a.H && sw >= 0 && sw < a.W;
        const int64_t ps = (int64_t(sd) * a.H + sh) * a.W + sw;
        for (int o0 = 0; o0 < a.cout; o0 += TK) {
            uint16_t va[8];
            load_g8(a, dy, ps, o0 + ac, in, va);
#pragma unroll
            for (int j = 0; j < 8; ++j) As[ar * LDA + ac + j] = va[j];
            uint4 wb = make_uint4(0, 0, 0, 0);
            if (c0n + bn < cin && o0 + bk < a.cout)
                wb = *reinterpret_cast<const uint4 *>(a.w + (int64_t(t) * cin + c0n + bn) * a.cout + o0 + bk);
            const uint16_t *wbs = reinterpret_cast<const uint16_t *>(&wb);
#pragma unroll
            for (int j = 0; j < 8; ++j) Bs[(bk + j) * LDB + bn] = wbs[j];
            __syncthreads();
            mma_step<false>(As + m0 * LDA, LDA, Bs + n0, LDB, acc);
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int64_t q = q0 + m0 + 8 * (i >> 2) + 4 * (l >> 5) + (i & 3);
        const int c = c0n + n0 + (l & 31);
        if (q < P && c < cin) dx[q * cin + c] = acc[i];
    }
}

// ---------------------------------------------------------------------------
// weight gradient (accumulated with FP32 atomics over position chunks)
// ---------------------------------------------------------------------------
constexpr int WG_CHUNK = 2048;  // positions per work-group

__global__ void __launch_bounds__(NTH) conv_wgrad_kernel(ConvArgs a, const float *dy, float *dw) {
    __shared__ uint16_t Xs[TK * LDB];  // [position][input channel]
    __shared__ uint16_t Gs[TK * LDB];  // [position][output channel]
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
    const int64_t P = int64_t(a.D) * a.H * a.W;
    const int cin = a.c1 + a.c2;
    const int ntile_o = (a.cout + TN - 1) / TN;
    const int ci0 = (blockIdx.y / ntile_o) * TM, o0 = (blockIdx.y % ntile_o) * TN;
    const int t = blockIdx.z;
    int dz, dyy, dxx;
    tap_offset(t, dz, dyy, dxx);
    const int m0 = (wv >> 1) * 32, n0 = (wv & 1) * 32;
    v16f acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
    const int r = tid >> 3, cc = (tid & 7) * 8;
    const int64_t pbeg = int64_t(blockIdx.x) * WG_CHUNK;
    const int64_t pend = min(P, pbeg + WG_CHUNK);
    for (int64_t pk = pbeg; pk < pend; pk += TK) {
        const int64_t p = pk + r;
        const bool valid = p < pend;
        const int pw = int(p % a.W), ph = int((p / a.W) % a.H), pd = int(p / (int64_t(a.W) * a.H));
        uint16_t vx[8], vg[8];
        if (valid)
            load_in8(a, pd + dz, ph + dyy, pw + dxx, ci0 + cc, vx);
        else
#pragma unroll
            for (int j = 0; j < 8; ++j) vx[j] = 0;
        load_g8(a, dy, p, o0 + cc, valid, vg);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            Xs[r * LDB + cc + j] = vx[j];
            Gs[r * LDB + cc + j] = vg[j];
        }
        __syncthreads();
        // A[m = input channel][k = position] is Xs transposed
        mma_step<true>(Xs + m0, LDB, Gs + n0, LDB, acc);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int c = ci0 + m0 + 8 * (i >> 2) + 4 * (l >> 5) + (i & 3);
        const int o = o0 + n0 + (l & 31);
        if (c < cin && o < a.cout) atomicAdd(dw + (int64_t(t) * cin + c) * a.cout + o, acc[i]);
    }
}

// bias gradient: db[o] += sum_p g[p, o]; thread per (chunk, channel)
__global__ void conv_bgrad_kernel(ConvArgs a, const float *dy, float *db) {
    const int64_t P = int64_t(a.D) * a.H * a.W;
    const int o = threadIdx.x;
    if (o >= a.cout) return;
    const int64_t pbeg = int64_t(blockIdx.x) * WG_CHUNK, pend = min(P, pbeg + WG_CHUNK);
    float s = 0.0f;
    for (int64_t p = pbeg; p < pend; ++p) {
        float g = dy[p * a.cout + o];
        if (a.relu && !(bf2f(a.y[p * a.cout + o]) > 0.0f)) g = 0.0f;
        s += g;
    }
    atomicAdd(db + o, s);
}

// ---------------------------------------------------------------------------
// pooling and the gradient plumbing of the U-Net
// ---------------------------------------------------------------------------
// y[q, c] = mean of the 8 children of q (BF16 in, BF16 out)
__global__ void pool2_kernel(const uint16_t *x, int D, int H, int W, int C, uint16_t *y) {
    const int64_t Pc = int64_t(D / 2) * (H / 2) * (W / 2);
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < Pc * C; e += int64_t(gridDim.x) * blockDim.x) {
        const int c = int(e % C);
        const int64_t q = e / C;
        const int qw = int(q % (W / 2)), qh = int((q / (W / 2)) % (H / 2)), qd = int(q / (int64_t(W / 2) * (H / 2)));
        float s = 0.0f;
        for (int j = 0; j < 8; ++j) {
            const int64_t p = (int64_t(2 * qd + (j >> 2)) * H + 2 * qh + ((j >> 1) & 1)) * W + 2 * qw + (j & 1);
            s += bf2f(x[p * C + c]);
        }
        y[e] = f2bf(s * 0.125f);
    }
}

// g[p, c] = gc[parent(p), c] / 8 (+ skip[p, off + c] when skip is given)
__global__ void pool2_back_kernel(const float *gc, const float *skip, int skip_stride, int skip_off, int D, int H,
                                  int W, int C, float *g) {
    const int64_t P = int64_t(D) * H * W;
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < P * C; e += int64_t(gridDim.x) * blockDim.x) {
        const int c = int(e % C);
        const int64_t p = e / C;
        const int pw = int(p % W), ph = int((p / W) % H), pd = int(p / (int64_t(W) * H));
        const int64_t q = (int64_t(pd >> 1) * (H >> 1) + (ph >> 1)) * (W >> 1) + (pw >> 1);
        float v = gc[q * C + c] * 0.125f;
        if (skip) v += skip[p * skip_stride + skip_off + c];
        g[e] = v;
    }
}

// gc[q, c] = sum over the 8 children p of q of g[p, c] (g row stride `stride`)
__global__ void up2_back_kernel(const float *g, int stride, int C, int D, int H, int W, float *gc) {
    const int64_t Pc = int64_t(D / 2) * (H / 2) * (W / 2);
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < Pc * C; e += int64_t(gridDim.x) * blockDim.x) {
        const int c = int(e % C);
        const int64_t q = e / C;
        const int qw = int(q % (W / 2)), qh = int((q / (W / 2)) % (H / 2)), qd = int(q / (int64_t(W / 2) * (H / 2)));
        float s = 0.0f;
        for (int j = 0; j < 8; ++j) {
            const int64_t p = (int64_t(2 * qd + (j >> 2)) * H + 2 * qh + ((j >> 1) & 1)) * W + 2 * qw + (j & 1);
            s += g[p * stride + c];
        }
        gc[e] = s;
    }
}

__global__ void fill_f32_kernel(float *p, int64_t n, float v) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------
// loss in channel-normalised units: pred = xin[:, 0:6] + s * out[:, 0:6],
// e_c = (pred_c - tgt_c) / s_c, loss = masked mean of e^2 over the six
// channels + lam (relative rho_A mass error)^2; tensors [P][8] FP32, mask =
// xin[:, 6]
// ---------------------------------------------------------------------------
constexpr int LOSS_BLOCKS = 256;

__global__ void __launch_bounds__(256) loss_partial_kernel(const float *out, const float *xin, const float *tgt, int64_t P,
                                                           ChanScale sc, double *part) {
    __shared__ double sh[4][4];
    double s[4] = {0, 0, 0, 0};  // sum mask, sum mask tgt_A, sum mask (pred_A - tgt_A), sum mask e^2
    for (int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; p < P; p += int64_t(gridDim.x) * blockDim.x) {
        const float m = xin[p * 8 + 6];
        if (m == 0.0f) continue;
        double sq = 0.0;
        for (int c = 0; c < 6; ++c) {
            const double d = (double(xin[p * 8 + c]) + double(sc.s[c]) * double(out[p * 8 + c]) - double(tgt[p * 8 + c])) /
                             double(sc.s[c]);
            sq += d * d;
        }
        s[0] += m;
        s[1] += m * double(tgt[p * 8]);
        s[2] += m * (double(xin[p * 8]) + double(sc.s[0]) * double(out[p * 8]) - double(tgt[p * 8]));
        s[3] += m * sq;
    }
    for (int q = 0; q < 4; ++q) {
        double v = s[q];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = sh[0][threadIdx.x] + sh[1][threadIdx.x] +
                                                            sh[2][threadIdx.x] + sh[3][threadIdx.x];
}

// totals in a fixed order; res = sum mask, sum mask tgt_A, mass error, loss
__global__ void loss_total_kernel(const double *part, int nb, double lam, double *res) {
    if (threadIdx.x != 0) return;
    double s[4] = {0, 0, 0, 0};
    for (int b = 0; b < nb; ++b)
        for (int q = 0; q < 4; ++q) s[q] += part[b * 4 + q];
    const double me = s[1] != 0.0 ? s[2] / s[1] : 0.0;
    res[0] = s[0];
    res[1] = s[1];
    res[2] = me;
    res[3] = (s[0] > 0.0 ? s[3] / (6.0 * s[0]) : 0.0) + lam * me * me;
}

__global__ void loss_grad_kernel(const float *out, const float *xin, const float *tgt, int64_t P, ChanScale sc,
                                 double lam, const double *res, float *grad) {
    const double n = res[0], mt = res[1], me = res[2];
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < P * 8; e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t p = e >> 3;
        const int c = int(e & 7);
        const float m = xin[p * 8 + 6];
        double g = 0.0;
        if (c < 6 && m != 0.0f && n > 0.0) {
            const double sc_c = sc.s[c];
            const double d = (double(xin[e]) + sc_c * double(out[e]) - double(tgt[e])) / sc_c;
            g = 2.0 * m * d / (6.0 * n);
            if (c == 0 && mt != 0.0) g += 2.0 * lam * me * m * sc_c / mt;
        }
        grad[e] = float(g);
    }
}

// per-channel sums of mask (y - x)^2 and of the mask over one pair of canvases
__global__ void __launch_bounds__(256) moments_kernel(const float *x, const float *y, int64_t P, double *part) {
    __shared__ double sh[4][7];
    double s[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; p < P; p += int64_t(gridDim.x) * blockDim.x) {
        const double m = x[p * 8 + 6];
        if (m == 0.0) continue;
        for (int c = 0; c < 6; ++c) {
            const double d = double(y[p * 8 + c]) - double(x[p * 8 + c]);
            s[c] += m * d * d;
        }
        s[6] += m;
    }
    for (int q = 0; q < 7; ++q) {
        double v = s[q];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 7) part[blockIdx.x * 7 + threadIdx.x] = sh[0][threadIdx.x] + sh[1][threadIdx.x] +
                                                            sh[2][threadIdx.x] + sh[3][threadIdx.x];
}

__global__ void moments_total_kernel(const double *part, int nb, double *res) {
    if (threadIdx.x != 0) return;
    double s[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int b = 0; b < nb; ++b)
        for (int q = 0; q < 7; ++q) s[q] += part[b * 7 + q];
    for (int q = 0; q < 7; ++q) res[q] = s[q];
}

// ---------------------------------------------------------------------------
// Adam on FP32 master parameters, with the BF16 copy the kernels read
// ---------------------------------------------------------------------------
__global__ void adam_kernel(float *p, const float *g, float *m, float *v, uint16_t *pb, int64_t n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pi;
        if (pb) pb[i] = f2bf(pi);
    }
}

// prediction of the network: pred[:, 0:6] = xin[:, 0:6] + s * out[:, 0:6], the rest
// copied from the input; also the BF16 copy (next input of a rollout)
__global__ void residual_kernel(const float *out, const float *xin, int64_t P, ChanScale sc, float *pred,
                                uint16_t *predb) {
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < P * 8; e += int64_t(gridDim.x) * blockDim.x) {
        const int c = int(e & 7);
        const float v = c < 6 ? xin[e] + sc.s[c] * out[e] : xin[e];
        if (pred) pred[e] = v;
        if (predb) predb[e] = f2bf(v);
    }
}

__global__ void to_bf16_kernel(const float *x, int64_t n, uint16_t *y) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        y[i] = f2bf(x[i]);
}

// ---------------------------------------------------------------------------
// restriction and lift
//
// Both work with the physical velocity u = (j + F/2) / rho of the method
// (Eq. 5 force F, velocity shift of the collision).  The stored state is the
// collision output f*, whose momentum is j* = j + F for equal relaxation
// times, so a restriction reads u = (j* - F/2) / rho with F from the stored
// densities, and a lift writes f*_k = f^eq(rho_k, u - F/(2 rho) + tau_k F_k /
// rho_k) with F from the lifted densities.  The force needs psi of the
// neighbours: a first pass writes psi_k of every node to scratch.
// ---------------------------------------------------------------------------
__device__ inline double psi_solid(const SurLattice &L, uint8_t m, int k) {
    return L.psi_tab[2 * (m & MAT_ID_MASK) + k];
}

// F_k = -G psi_k(x) sum_i w_i psi_kbar(x + c_i) c_i + rho_k g at fluid node
// (x, y, z) with densities rho (= psi on fluid); neighbours beyond a closed
// end plane count as 0 (fluid nodes never reach them: the end planes are solid)
__device__ inline void force_at(const SurLattice &L, int x, int y, int z, const double rho[2], double F[2][3]) {
    const int64_t n_all = int64_t(L.nx) * L.ny * L.nz;
    double s[2][3] = {{0, 0, 0}, {0, 0, 0}};
    for (int i = 1; i < Q; ++i) {
        int xx = x + cx(i), yy = y + cy(i), zz = z + cz(i);
        if (L.px) xx = (xx + L.nx) % L.nx;
        if (L.py) yy = (yy + L.ny) % L.ny;
        if (L.pz) zz = (zz + L.nz) % L.nz;
        if (xx < 0 || xx >= L.nx || yy < 0 || yy >= L.ny || zz < 0 || zz >= L.nz) continue;
        const int64_t m = (int64_t(zz) * L.ny + yy) * L.nx + xx;
        for (int k = 0; k < 2; ++k) {
            const double v = wgt<double>(i) * L.psi[(1 - k) * n_all + m];
            s[k][0] += v * cx(i);
            s[k][1] += v * cy(i);
            s[k][2] += v * cz(i);
        }
    }
    for (int k = 0; k < 2; ++k)
        for (int d = 0; d < 3; ++d) F[k][d] = -L.G * rho[k] * s[k][d] + rho[k] * L.g[d];
}

// psi_k of the stored state: rho_k on fluid nodes, the material's value elsewhere
template <class S>
__global__ void psi_state_kernel(const S *f, SurLattice L) {
    const int64_t n_all = int64_t(L.nx) * L.ny * L.nz;
    for (int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; n < n_all; n += int64_t(gridDim.x) * blockDim.x) {
        const uint8_t m = L.mat[n];
        for (int k = 0; k < 2; ++k) {
            double v;
            if ((m & MAT_ID_MASK) == MAT_FLUID) {
                v = 0.0;
                for (int i = 0; i < Q; ++i) v += double(Codec<S>::dec(f[(k * Q + i) * L.fs + n])) + wgt<double>(i) * L.rref[k];
            } else {
                v = psi_solid(L, m, k);
            }
            L.psi[k * n_all + n] = v;
        }
    }
}

template <class S>
__global__ void restrict_kernel(const S *f, SurLattice L, int D, int H, int W, float *outf, uint16_t *outb) {
    const int64_t P = int64_t(D) * H * W;
    const int nx = L.nx, ny = L.ny, nz = L.nz;
    for (int64_t c = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; c < P; c += int64_t(gridDim.x) * blockDim.x) {
        const int qx = int(c % W), qy = int((c / W) % H), qz = int(c / (int64_t(W) * H));
        float cell[8] = {0.03f, 1.0f, 0, 0, 0, 0, 0, 0};
        if (2 * qz + 1 < nz && 2 * qy + 1 < ny && 2 * qx + 1 < nx) {
            double rho[2] = {0, 0}, mom[3] = {0, 0, 0};
            int nf = 0, nrod = 0;
            for (int j = 0; j < 8; ++j) {
                const int z = 2 * qz + (j >> 2), y = 2 * qy + ((j >> 1) & 1), x = 2 * qx + (j & 1);
                const int64_t n = (int64_t(z) * ny + y) * nx + x;
                const uint8_t m = L.mat[n] & MAT_ID_MASK;
                nrod += m == MAT_ROD;
                if (m != MAT_FLUID) continue;
                ++nf;
                double r[2] = {0, 0};
                for (int k = 0; k < 2; ++k)
                    for (int i = 0; i < Q; ++i) {
                        const double v = double(Codec<S>::dec(f[(k * Q + i) * L.fs + n])) + wgt<double>(i) * L.rref[k];
                        r[k] += v;
                        mom[0] += v * cx(i);
                        mom[1] += v * cy(i);
                        mom[2] += v * cz(i);
                    }
                double F[2][3];
                force_at(L, x, y, z, r, F);
                for (int d = 0; d < 3; ++d) mom[d] -= 0.5 * (F[0][d] + F[1][d]);
                rho[0] += r[0];
                rho[1] += r[1];
            }
            double out[8] = {0, 0, 0, 0, 0, nrod / 8.0, 1.0, nf / 8.0};
            if (nf) {
                out[0] = rho[0] / nf;
                out[1] = rho[1] / nf;
                const double tot = rho[0] + rho[1];
                if (tot > 0.0)
                    for (int d = 0; d < 3; ++d) out[2 + d] = mom[d] / tot;
            }
            for (int q = 0; q < 8; ++q) cell[q] = float(out[q]);
        }
        for (int q = 0; q < 8; ++q) {
            if (outf) outf[c * 8 + q] = cell[q];
            if (outb) outb[c * 8 + q] = f2bf(cell[q]);
        }
    }
}

__device__ inline void lerp_index(int x, int nc, int &i0, int &i1, double &w) {
    double c = x / 2.0 - 0.25;
    c = fmin(fmax(c, 0.0), nc - 1.0);
    i0 = int(floor(c));
    i1 = min(i0 + 1, nc - 1);
    w = c - i0;
}

// prolonged (rho_A, rho_B, u) at fine node (x, y, z): trilinear over the
// corner cells that hold fluid (channel 7 > 0), renormalised; else the plain
// mean of the fluid-holding cells of the 4 x 4 x 4 block around them; else
// gas at rest
__device__ inline void prolong_at(const float *coarse, int H, int W, int ncz, int ncy, int ncx, int x, int y, int z,
                                  double a[5]) {
    int z0, z1, y0, y1, x0, x1;
    double wz, wy, wx;
    lerp_index(z, ncz, z0, z1, wz);
    lerp_index(y, ncy, y0, y1, wy);
    lerp_index(x, ncx, x0, x1, wx);
    for (int q = 0; q < 5; ++q) a[q] = 0.0;
    double wsum = 0.0;
    for (int j = 0; j < 8; ++j) {
        const int iz = (j >> 2) ? z1 : z0, iy = ((j >> 1) & 1) ? y1 : y0, ix = (j & 1) ? x1 : x0;
        const double fz = (j >> 2) ? wz : 1.0 - wz, fy = ((j >> 1) & 1) ? wy : 1.0 - wy, fx = (j & 1) ? wx : 1.0 - wx;
        const float *cc = coarse + ((int64_t(iz) * H + iy) * W + ix) * 8;
        if (!(cc[7] > 0.0f)) continue;
        const double wt = fz * fy * fx;
        for (int q = 0; q < 5; ++q) a[q] += wt * double(cc[q]);
        wsum += wt;
    }
    if (wsum > 0.0) {
        for (int q = 0; q < 5; ++q) a[q] /= wsum;
        return;
    }
    int cnt = 0;
    for (int iz = z0 - 1; iz <= z0 + 2; ++iz)
        for (int iy = y0 - 1; iy <= y0 + 2; ++iy)
            for (int ix = x0 - 1; ix <= x0 + 2; ++ix) {
                if (iz < 0 || iz >= ncz || iy < 0 || iy >= ncy || ix < 0 || ix >= ncx) continue;
                const float *cc = coarse + ((int64_t(iz) * H + iy) * W + ix) * 8;
                if (!(cc[7] > 0.0f)) continue;
                for (int q = 0; q < 5; ++q) a[q] += double(cc[q]);
                ++cnt;
            }
    if (cnt) {
        for (int q = 0; q < 5; ++q) a[q] /= cnt;
    } else {
        a[0] = 0.03;
        a[1] = 1.0;
    }
}

// psi_k of the lifted state: prolonged rho_k on fluid nodes, the material's value elsewhere
__global__ void psi_lift_kernel(const float *coarse, int H, int W, SurLattice L) {
    const int64_t n_all = int64_t(L.nx) * L.ny * L.nz;
    for (int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; n < n_all; n += int64_t(gridDim.x) * blockDim.x) {
        const uint8_t m = L.mat[n];
        double v[2];
        if ((m & MAT_ID_MASK) == MAT_FLUID) {
            const int x = int(n % L.nx), y = int((n / L.nx) % L.ny), z = int(n / (int64_t(L.nx) * L.ny));
            double a[5];
            prolong_at(coarse, H, W, L.nz / 2, L.ny / 2, L.nx / 2, x, y, z, a);
            v[0] = a[0];
            v[1] = a[1];
        } else {
            v[0] = psi_solid(L, m, 0);
            v[1] = psi_solid(L, m, 1);
        }
        L.psi[n] = v[0];
        L.psi[n_all + n] = v[1];
    }
}

template <class S>
__global__ void lift_kernel(const float *coarse, int H, int W, SurLattice L, S *f) {
    const int64_t n_all = int64_t(L.nx) * L.ny * L.nz;
    for (int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; n < n_all; n += int64_t(gridDim.x) * blockDim.x) {
        if ((L.mat[n] & MAT_ID_MASK) != MAT_FLUID) continue;
        const int x = int(n % L.nx), y = int((n / L.nx) % L.ny), z = int(n / (int64_t(L.nx) * L.ny));
        double a[5];
        prolong_at(coarse, H, W, L.nz / 2, L.ny / 2, L.nx / 2, x, y, z, a);
        const double rho[2] = {a[0], a[1]};
        double F[2][3];
        force_at(L, x, y, z, rho, F);
        const double tot = rho[0] + rho[1];
        double up[3];
        for (int d = 0; d < 3; ++d) up[d] = a[2 + d] - 0.5 * (F[0][d] + F[1][d]) / tot;
        for (int k = 0; k < 2; ++k) {
            double u[3];
            const bool ok = rho[k] >= 1e-12;  // no shift for a vanishing component
            for (int d = 0; d < 3; ++d) u[d] = ok ? up[d] + L.tau[k] * F[k][d] / rho[k] : up[d];
            const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            for (int i = 0; i < Q; ++i) {
                const double cu = cx(i) * u[0] + cy(i) * u[1] + cz(i) * u[2];
                const double feq = wgt<double>(i) * rho[k] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
                f[(k * Q + i) * L.fs + n] = Codec<S>::enc(typename Codec<S>::C(feq - wgt<double>(i) * L.rref[k]));
            }
        }
    }
}

int grid_for(int64_t n) {
    const int64_t g = (n + 255) / 256;
    return int(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

}  // namespace

hipError_t launch_conv_fwd(const ConvArgs &a, hipStream_t s) {
    const int64_t P = int64_t(a.D) * a.H * a.W;
    hipLaunchKernelGGL(conv_fwd_kernel, dim3(unsigned((P + TM - 1) / TM), (a.cout + TN - 1) / TN), dim3(NTH), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_conv_dgrad(const ConvArgs &a, const float *dy, float *dx, hipStream_t s) {
    const int64_t P = int64_t(a.D) * a.H * a.W;
    const int cin = a.c1 + a.c2;
    hipLaunchKernelGGL(conv_dgrad_kernel, dim3(unsigned((P + TM - 1) / TM), (cin + TN - 1) / TN), dim3(NTH), 0, s, a, dy,
                       dx);
    return hipGetLastError();
}

hipError_t launch_conv_wgrad(const ConvArgs &a, const float *dy, float *dw, float *db, hipStream_t s) {
    const int64_t P = int64_t(a.D) * a.H * a.W;
    const int cin = a.c1 + a.c2;
    const unsigned nchunk = unsigned((P + WG_CHUNK - 1) / WG_CHUNK);
    const int tiles = ((cin + TM - 1) / TM) * ((a.cout + TN - 1) / TN);
    hipLaunchKernelGGL(conv_wgrad_kernel, dim3(nchunk, tiles, 27), dim3(NTH), 0, s, a, dy, dw);
    if (db) hipLaunchKernelGGL(conv_bgrad_kernel, dim3(nchunk), dim3(256), 0, s, a, dy, db);
    return hipGetLastError();
}

hipError_t launch_pool2(const uint16_t *x, int D, int H, int W, int C, uint16_t *y, hipStream_t s) {
    hipLaunchKernelGGL(pool2_kernel, dim3(grid_for(int64_t(D / 2) * (H / 2) * (W / 2) * C)), dim3(256), 0, s, x, D, H, W,
                       C, y);
    return hipGetLastError();
}

hipError_t launch_pool2_back(const float *gc, const float *skip, int skip_stride, int skip_off, int D, int H, int W,
                             int C, float *g, hipStream_t s) {
    hipLaunchKernelGGL(pool2_back_kernel, dim3(grid_for(int64_t(D) * H * W * C)), dim3(256), 0, s, gc, skip, skip_stride,
                       skip_off, D, H, W, C, g);
    return hipGetLastError();
}

hipError_t launch_up2_back(const float *g, int stride, int C, int D, int H, int W, float *gc, hipStream_t s) {
    hipLaunchKernelGGL(up2_back_kernel, dim3(grid_for(int64_t(D / 2) * (H / 2) * (W / 2) * C)), dim3(256), 0, s, g, stride,
                       C, D, H, W, gc);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t s) {
    hipLaunchKernelGGL(fill_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *x, int64_t n, uint16_t *y, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, y);
    return hipGetLastError();
}

hipError_t launch_residual(const float *out, const float *xin, int64_t P, const ChanScale &sc, float *pred,
                           uint16_t *predb, hipStream_t s) {
    hipLaunchKernelGGL(residual_kernel, dim3(grid_for(P * 8)), dim3(256), 0, s, out, xin, P, sc, pred, predb);
    return hipGetLastError();
}

hipError_t launch_loss(const float *out, const float *xin, const float *tgt, int64_t P, const ChanScale &sc, double lam,
                       double *part, double *res, float *grad, hipStream_t s) {
    hipLaunchKernelGGL(loss_partial_kernel, dim3(LOSS_BLOCKS), dim3(256), 0, s, out, xin, tgt, P, sc, part);
    hipLaunchKernelGGL(loss_total_kernel, dim3(1), dim3(64), 0, s, part, LOSS_BLOCKS, lam, res);
    if (grad)
        hipLaunchKernelGGL(loss_grad_kernel, dim3(grid_for(P * 8)), dim3(256), 0, s, out, xin, tgt, P, sc, lam, res, grad);
    return hipGetLastError();
}

hipError_t launch_moments(const float *x, const float *y, int64_t P, double *part, double *res, hipStream_t s) {
    hipLaunchKernelGGL(moments_kernel, dim3(LOSS_BLOCKS), dim3(256), 0, s, x, y, P, part);
    hipLaunchKernelGGL(moments_total_kernel, dim3(1), dim3(64), 0, s, part, LOSS_BLOCKS, res);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, uint16_t *pb, int64_t n, int step, float lr, float b1,
                       float b2, float eps, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, float(step)), c2 = 1.0f - powf(b2, float(step));
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, g, m, v, pb, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

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

hipError_t launch_restrict(int prec, const void *f, const SurLattice &L, int D, int H, int W, float *outf,
                           uint16_t *outb, hipStream_t s) {
    const int gn = grid_for(int64_t(L.nx) * L.ny * L.nz), gc = grid_for(int64_t(D) * H * W);
    return by_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        const S *fs = static_cast<const S *>(f);
        hipLaunchKernelGGL(psi_state_kernel<S>, dim3(gn), dim3(256), 0, s, fs, L);
        hipLaunchKernelGGL(restrict_kernel<S>, dim3(gc), dim3(256), 0, s, fs, L, D, H, W, outf, outb);
        return hipGetLastError();
    });
}

hipError_t launch_lift(int prec, const float *coarse, int D, int H, int W, const SurLattice &L, void *f, hipStream_t s) {
    (void)D;
    const int gn = grid_for(int64_t(L.nx) * L.ny * L.nz);
    return by_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(psi_lift_kernel, dim3(gn), dim3(256), 0, s, coarse, H, W, L);
        hipLaunchKernelGGL(lift_kernel<S>, dim3(gn), dim3(256), 0, s, coarse, H, W, L, static_cast<S *>(f));
        return hipGetLastError();
    });
}

}  // namespace lbm
