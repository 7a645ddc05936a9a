// Learned surrogate (gfx950): restriction of the lattice state to a coarse
// canvas, prolongation and lift back to populations, and the training and
// inference kernels of a 3-D convolutional U-Net.
//
// Convolutions are implicit GEMMs on BF16 MFMA (32 x 32 x 16, FP32
// accumulation).  Tensors are channels-last, [D][H][W][C], C a multiple of 8.
//   forward  y[p, o]  = b[o] + sum_{t, c} x[p + o_t, c] w[t, c, o]
//            M = positions, N = output channels, K = 27 x input channels
//   dgrad    dx[q, c] = sum_{t, o} g[q - o_t, o] w[t, c, o],  g = dy (y > 0)
//            M = positions, N = input channels, K = 27 x output channels
//   wgrad    dw[t, c, o] += sum_p x[p + o_t, c] g[p, o]
//            M = 27 x input channels, N = output channels, K = positions
// A work-group of four wavefronts computes a 256 x 32, 128 x 64 or 128 x 128
// tile (chosen by N), each wavefront 64 x 32 or 64 x 64; K advances in steps
// of 32 through two LDS buffers.
// The decoder's inputs are read in place: channels [0, c1) from the coarser
// level through nearest-neighbour upsampling, [c1, c1 + c2) from the skip.
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

__device__ inline uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return static_cast<uint16_t>(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }


// ---------------------------------------------------------------------------
// forward and input gradient: one implicit GEMM, C[M][N] = sum_k A[M][k] B[k][N]
//   forward: M = positions p, N = output channels o, k = (tap t, input channel c),
//            A[p][k] = x[p + o_t][c], B[k][o] = wt[o][t][c] (packed weights)
//   dgrad:   M = positions q, N = input channels c, k = (tap t, output channel o),
//            A[q][k] = g[q - o_t][o], B[k][c] = w[t][c][o]
// Both operands sit in LDS K-contiguous per row ([row][BK + 8], 80-byte rows,
// conflict-free 16-byte reads), so every MFMA operand is one 128-bit LDS
// read: lane l takes row l % 32, k = 8 (l / 32) .. + 7 of a 32 x 32 x 16
// block.  K advances by BK = 32 per stage through two LDS buffers; the global
// loads of stage s + 1 are in flight while stage s computes, one barrier per
// stage.  TPR threads share an A row (4 / TPR k-groups of 8 channels each);
// the row's coordinates and its 27-bit mask of in-volume taps are computed
// once, so a stage costs each thread a few integer operations per load.
// ---------------------------------------------------------------------------
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
constexpr int BK = 32, LDK = BK + 8;

// bit t set when tap t of (d, h, w) lies inside the volume
__device__ inline unsigned tap_mask(int d, int h, int w, int D, int H, int W) {
    const unsigned mz = 2u | (d > 0 ? 1u : 0u) | (d < D - 1 ? 4u : 0u);
    const unsigned my = 2u | (h > 0 ? 1u : 0u) | (h < H - 1 ? 4u : 0u);
    const unsigned mx = 2u | (w > 0 ? 1u : 0u) | (w < W - 1 ? 4u : 0u);
    unsigned m = 0;
#pragma unroll
    for (int t = 0; t < 27; ++t)
        if ((mz >> (t / 9)) & (my >> ((t / 3) % 3)) & (mx >> (t % 3)) & 1u) m |= 1u << t;
    return m;
}

template <int BM, int BN, int WM, int WN, bool DGRAD>
__global__ void __launch_bounds__(256) conv_gemm_kernel(ConvArgs a, const uint16_t *g, float *dx, float *acc_out) {
    static_assert(WM * WN == 4, "four wavefronts");
    constexpr int MB = BM / WM / 32, NB = BN / WN / 32;
    static_assert(MB >= 1 && NB >= 1 && MB * WM * 32 == BM && NB * WN * 32 == BN, "tile shape");
    constexpr int TPR = 256 / BM, GPT = 4 / TPR;  // threads per A row, k-groups per thread
    constexpr int BLD = BN * 4;                    // B loads (16 bytes) per stage
    constexpr int BLT = BLD >= 256 ? BLD / 256 : 1;
    __shared__ __attribute__((aligned(16))) uint16_t As[2][BM * LDK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN * LDK];

    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
    const int P = a.D * a.H * a.W;
    const int HW = a.H * a.W;
    const int cin = a.c1 + a.c2;
    const int N = DGRAD ? cin : a.cout;   // columns of C
    const int kc = DGRAD ? a.cout : cin;  // channels per tap along k
    const int Kd = 27 * kc;
    const int m0 = blockIdx.x * BM;
    const int n0 = blockIdx.y * BN;
    const int wm = (wv / WN) * MB * 32, wn = (wv % WN) * NB * 32;

    // ---- this thread's A row and its k-groups
    // rows tid % BM; the k-groups (tid / BM) * GPT .. are the same for a whole
    // wavefront, so its tap and channel bookkeeping is scalar
    const int ar = tid % BM, ag0 = __builtin_amdgcn_readfirstlane((tid / BM) * GPT);
    const int p = m0 + ar;
    const bool prow = p < P;
    const int pw = p % a.W, ph = (p / a.W) % a.H, pd = p / HW;
    unsigned tmask = prow ? tap_mask(pd, ph, pw, a.D, a.H, a.W) : 0u;
    // split-K: work-group z of gridDim.z takes stages [s0, s1) and adds its
    // partial sums (no bias or ReLU) into acc_out (forward) or dx (dgrad)
    const int nst_all = (Kd + BK - 1) / BK;
    const int s0 = int(int64_t(nst_all) * blockIdx.z / gridDim.z);
    const int s1 = int(int64_t(nst_all) * (blockIdx.z + 1) / gridDim.z);
    const bool split = gridDim.z > 1;
    int gt[GPT], gc[GPT];  // tap and channel of each k-group at the current stage
#pragma unroll
    for (int j = 0; j < GPT; ++j) {
        gt[j] = (s0 * BK + 8 * (ag0 + j)) / kc;
        gc[j] = (s0 * BK + 8 * (ag0 + j)) % kc;
    }
    const int H2 = a.H >> 1, W2 = a.W >> 1;

    // ---- B: BN rows x 4 k-groups per stage
    int bn[BLT], bgi[BLT], bt[BLT], bc[BLT];
    bool bon[BLT];
#pragma unroll
    for (int j = 0; j < BLT; ++j) {
        const int idx = tid + 256 * j;
        bn[j] = idx >> 2;
        bgi[j] = idx & 3;
        bon[j] = idx < BLD && n0 + bn[j] < N;
        bt[j] = (s0 * BK + 8 * bgi[j]) / kc;
        bc[j] = (s0 * BK + 8 * bgi[j]) % kc;
    }

    // Loads are unconditional (an invalid one reads a safe address) and the
    // zero fill happens at the LDS store, so no load waits on another.
    uint4 ra[GPT], rb[BLT];
    bool aok[GPT], bok[BLT];
    const uint16_t *asafe = DGRAD ? g : a.x1;
    auto load = [&](int k0) {
#pragma unroll
        for (int j = 0; j < GPT; ++j) {
            const int t = gt[j], c = gc[j];
            const bool ok = prow && (k0 + 8 * (ag0 + j) < Kd) && ((tmask >> (DGRAD ? 26 - t : t)) & 1u);
            const int dz = t / 9 - 1, dyy = (t / 3) % 3 - 1, dxx = t % 3 - 1;
            const uint16_t *src;
            if (DGRAD) {
                src = g + (p - (dz * HW + dyy * a.W + dxx)) * a.cout + c;
            } else if (c < a.c1) {
                if (a.up1) {
                    const int q = (((pd + dz) >> 1) * H2 + ((ph + dyy) >> 1)) * W2 + ((pw + dxx) >> 1);
                    src = a.x1 + q * a.c1 + c;
                } else {
                    src = a.x1 + (p + dz * HW + dyy * a.W + dxx) * a.c1 + c;
                }
            } else {
                src = a.x2 + (p + dz * HW + dyy * a.W + dxx) * a.c2 + (c - a.c1);
            }
            ra[j] = *reinterpret_cast<const uint4 *>(ok ? src : asafe);
            aok[j] = ok;
        }
#pragma unroll
        for (int j = 0; j < BLT; ++j) {
            const bool ok = bon[j] && k0 + 8 * bgi[j] < Kd;
            const uint16_t *src = DGRAD ? a.w + (bt[j] * cin + n0 + bn[j]) * a.cout + bc[j]
                                        : a.wt + (n0 + bn[j]) * Kd + k0 + 8 * bgi[j];
            rb[j] = *reinterpret_cast<const uint4 *>(ok ? src : (DGRAD ? a.w : a.wt));
            bok[j] = ok;
        }
    };
    auto advance = [&]() {
#pragma unroll
        for (int j = 0; j < GPT; ++j) {
            gc[j] += BK;
            while (gc[j] >= kc) {
                gc[j] -= kc;
                ++gt[j];
            }
        }
        if (DGRAD) {
#pragma unroll
            for (int j = 0; j < BLT; ++j) {
                bc[j] += BK;
                while (bc[j] >= kc) {
                    bc[j] -= kc;
                    ++bt[j];
                }
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int j = 0; j < GPT; ++j)
            *reinterpret_cast<uint4 *>(&As[buf][ar * LDK + 8 * (ag0 + j)]) = aok[j] ? ra[j] : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < BLT; ++j)
            if (tid + 256 * j < BLD)
                *reinterpret_cast<uint4 *>(&Bs[buf][bn[j] * LDK + 8 * bgi[j]]) = bok[j] ? rb[j] : make_uint4(0, 0, 0, 0);
    };

    v16f acc[MB][NB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

    const int nst = s1 - s0;
    load(s0 * BK);
    store(0);
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
        const int cur = st & 1;
        if (st + 1 < nst) {
            advance();
            load((s0 + st + 1) * BK);
        }
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            v8bf fa[MB], fb[NB];
#pragma unroll
            for (int i = 0; i < MB; ++i)
                fa[i] = *reinterpret_cast<const v8bf *>(&As[cur][(wm + 32 * i + (l & 31)) * LDK + kk + 8 * (l >> 5)]);
#pragma unroll
            for (int j = 0; j < NB; ++j)
                fb[j] = *reinterpret_cast<const v8bf *>(&Bs[cur][(wn + 32 * j + (l & 31)) * LDK + kk + 8 * (l >> 5)]);
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        }
        if (st + 1 < nst) store(cur ^ 1);
        __syncthreads();
    }

    // D element e of lane l: row 8 (e / 4) + 4 (l / 32) + e % 4, column l % 32
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int col = n0 + wn + 32 * j + (l & 31);
            if (col >= N) continue;
            const float bias = (!DGRAD && a.b) ? a.b[col] : 0.0f;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = m0 + wm + 32 * i + 8 * (e >> 2) + 4 * (l >> 5) + (e & 3);
                if (row >= P) continue;
                if (split) {
                    atomicAdd((DGRAD ? dx + row * cin : acc_out + row * a.cout) + col, acc[i][j][e]);
                } else if (DGRAD) {
                    dx[row * cin + col] = acc[i][j][e];
                } else {
                    float v = acc[i][j][e] + bias;
                    if (a.relu) v = fmaxf(v, 0.0f);
                    if (a.y) a.y[row * a.cout + col] = f2bf(v);
                    if (a.yf) a.yf[row * a.cout + col] = v;
                }
            }
        }
}

// Forward convolution of a brick of ZB x 8 x 8 positions (M = 64 ZB rows)
// against up to 32 WN output channels, for volumes made of whole bricks:
// ZB = 4, WN = 1 for layers of up to 32 output channels, ZB = 2, WN = 2 for
// up to 64.  Per chunk of 32 input channels the brick's (ZB + 2) x 10 x 10
// input halo is staged in LDS once, the weights nine taps at a time; every
// tap's A operand is then the halo read at the tap's offset, so each input
// element leaves L2 a few times instead of 27.  Each wavefront owns 64 rows
// (two 32-row MFMA blocks) of one 32-column block.  Summation order: chunk,
// tap, channel.
constexpr int BRY = 8, BRX = 8, HLY = BRY + 2, HLX = BRX + 2;
constexpr int BR_TG = 9;  // taps per weight stage (one dz plane of taps)

template <int ZB, int WN>
struct Brick {
    static constexpr int BN = 32 * WN;
    static constexpr int NHALO = (ZB + 2) * HLY * HLX;
    static constexpr int HL = (NHALO * 4 + 255) / 256;          // halo loads per thread
    static constexpr int WE = BR_TG * BN * 4;                   // 16-byte weight elements per stage
    static constexpr int WL = (WE + 255) / 256;                 // weight loads per thread
    static_assert(64 * ZB * WN == 256, "four wavefronts of 64 rows x 32 columns");
};

// per-component select (a select between two uint4 values is lowered to a
// load through a selected address with the zero kept in scratch)
__device__ __forceinline__ uint4 keep4(bool ok, uint4 v) {
    return make_uint4(ok ? v.x : 0u, ok ? v.y : 0u, ok ? v.z : 0u, ok ? v.w : 0u);
}

// loads of a brick's input halo for channels c0 .. c0 + 31 into registers;
// an invalid element loads a safe address and becomes zero
template <int ZB, int WN, bool DG>
__device__ __forceinline__ void brick_fetch_halo(const ConvArgs &a, const uint16_t *g, int tid, int x0, int y0,
                                                 int z0, int c0, uint4 (&hv)[Brick<ZB, WN>::HL]) {
    using B = Brick<ZB, WN>;
    const int cin = DG ? a.cout : a.c1 + a.c2;  // channels of the staged input
    const int H2 = a.H >> 1, W2 = a.W >> 1;
#pragma unroll
    for (int j = 0; j < B::HL; ++j) {
        const int e = tid + 256 * j;
        const int hp = e >> 2, gi = e & 3;
        const int hz = hp / (HLY * HLX), hy = (hp / HLX) % HLY, hx = hp % HLX;
        const int z = z0 + hz - 1, y = y0 + hy - 1, x = x0 + hx - 1;
        const int c = c0 + 8 * gi;
        const bool ok = e < B::NHALO * 4 && z >= 0 && z < a.D && y >= 0 && y < a.H && x >= 0 && x < a.W && c < cin;
        const uint16_t *src = DG ? g : a.x1;
        if (ok && DG) {
            src = g + int64_t(z * a.H + y) * a.W * a.cout + int64_t(x) * a.cout + c;
        } else if (ok) {
            if (c < a.c1)
                src = a.up1 ? a.x1 + (int64_t((z >> 1) * H2 + (y >> 1)) * W2 + (x >> 1)) * a.c1 + c
                            : a.x1 + (int64_t(z * a.H + y) * a.W + x) * a.c1 + c;
            else
                src = a.x2 + (int64_t(z * a.H + y) * a.W + x) * a.c2 + (c - a.c1);
        }
        hv[j] = keep4(ok, *reinterpret_cast<const uint4 *>(src));
    }
}

// loads of the weights of taps t0 .. t0 + 8 for channels c0 .. c0 + 31
// forward: B[n = output channel][k = input channel] = wt[n][t][c]
// input gradient: B[n = input channel][k = output channel] = w[t][n][k]
template <int ZB, int WN, bool DG>
__device__ __forceinline__ void brick_fetch_w(const ConvArgs &a, int tid, int c0, int t0,
                                              uint4 (&wr)[Brick<ZB, WN>::WL]) {
    using B = Brick<ZB, WN>;
    const int cin = a.c1 + a.c2, Kd = 27 * cin;
    const int kc = DG ? a.cout : cin, nn = DG ? cin : a.cout;
#pragma unroll
    for (int j = 0; j < B::WL; ++j) {
        const int e = tid + 256 * j;
        const int t = t0 + e / (B::BN * 4), n = (e >> 2) % B::BN, gi = e & 3;
        const int c = c0 + 8 * gi;
        const bool ok = e < B::WE && n < nn && c < kc;
        const uint16_t *src = DG ? a.w + (int64_t(t) * cin + n) * a.cout + c : a.wt + int64_t(n) * Kd + t * cin + c;
        wr[j] = keep4(ok, *reinterpret_cast<const uint4 *>(ok ? src : (DG ? a.w : a.wt)));
    }
}

// DG: the input gradient dx[q][c] = sum_{t, o} g[q - o_t][o] w[t][c][o], the
// same computation over g with the taps mirrored, dx stored in FP32
template <int ZB, int WN, bool DG>
__global__ void __launch_bounds__(256, 2) conv_brick_kernel(ConvArgs a, const uint16_t *g, float *dx) {
    using B = Brick<ZB, WN>;
    __shared__ __attribute__((aligned(16))) uint16_t Hs[B::NHALO * LDK];
    __shared__ __attribute__((aligned(16))) uint16_t Ws[BR_TG * B::BN * LDK];
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
    const int cin = DG ? a.cout : a.c1 + a.c2;  // channels summed over (k)
    const int ncol = DG ? a.c1 + a.c2 : a.cout;  // columns of the result
    const int nbx = a.W / BRX, nby = a.H / BRY;
    const int b = blockIdx.x;
    const int x0 = (b % nbx) * BRX, y0 = ((b / nbx) % nby) * BRY, z0 = (b / (nbx * nby)) * ZB;
    const int wm = (wv / WN) * 64, wn = (wv % WN) * 32;
    v16f acc[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[i][e] = 0.0f;
    // halo rows read by this lane's two A blocks (tap offset added per tap)
    int hrow[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int m = wm + 32 * i + (l & 31);
        hrow[i] = ((m >> 6) * HLY + ((m >> 3) & 7)) * HLX + (m & 7);
    }
    // Staging: each thread issues all of a stage's loads into registers and
    // stores them after the barrier that ends the previous stage; the next
    // stage's loads are issued before this stage's MFMAs.
    uint4 hv[B::HL], wr[B::WL];
    brick_fetch_halo<ZB, WN, DG>(a, g, tid, x0, y0, z0, 0, hv);
    brick_fetch_w<ZB, WN, DG>(a, tid, 0, 0, wr);
    for (int c0 = 0; c0 < cin; c0 += BK) {
#pragma unroll
        for (int j = 0; j < B::HL; ++j) {
            const int e = tid + 256 * j;
            if (e < B::NHALO * 4) *reinterpret_cast<uint4 *>(&Hs[(e >> 2) * LDK + 8 * (e & 3)]) = hv[j];
        }
        const int kn = min(BK, cin - c0);
        for (int t0 = 0; t0 < 27; t0 += BR_TG) {
#pragma unroll
            for (int j = 0; j < B::WL; ++j) {
                const int e = tid + 256 * j;
                if (e < B::WE) *reinterpret_cast<uint4 *>(&Ws[(e >> 2) * LDK + 8 * (e & 3)]) = wr[j];
            }
            __syncthreads();
            if (t0 + BR_TG < 27) {
                brick_fetch_w<ZB, WN, DG>(a, tid, c0, t0 + BR_TG, wr);
            } else if (c0 + BK < cin) {
                brick_fetch_halo<ZB, WN, DG>(a, g, tid, x0, y0, z0, c0 + BK, hv);
                brick_fetch_w<ZB, WN, DG>(a, tid, c0 + BK, 0, wr);
            }
            // the stage's nine taps share dz = t0 / 9; unrolled so that the
            // LDS reads of the next taps go out ahead of the MFMAs.  The input
            // gradient reads the halo at the mirrored offset -o_t.
            const int zoff = (DG ? 2 - t0 / BR_TG : t0 / BR_TG) * HLY * HLX;
#pragma unroll
            for (int tt = 0; tt < BR_TG; ++tt) {
                const int toff = DG ? zoff + (2 - tt / 3) * HLX + (2 - tt % 3) : zoff + (tt / 3) * HLX + tt % 3;
#pragma unroll
                for (int kq = 0; kq < 2; ++kq) {
                    if (16 * kq < kn) {  // uniform: the chunk's last channels may end at 8 or 24
                        const int ko = 16 * kq + 8 * (l >> 5);
                        const v8bf fb =
                            *reinterpret_cast<const v8bf *>(&Ws[(tt * B::BN + wn + (l & 31)) * LDK + ko]);
                        const v8bf fa0 = *reinterpret_cast<const v8bf *>(&Hs[(hrow[0] + toff) * LDK + ko]);
                        const v8bf fa1 = *reinterpret_cast<const v8bf *>(&Hs[(hrow[1] + toff) * LDK + ko]);
                        acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa0, fb, acc[0], 0, 0, 0);
                        acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa1, fb, acc[1], 0, 0, 0);
                    }
                }
            }
            __syncthreads();  // the next stage overwrites the weights (and the halo)
        }
    }
    // D element e of lane l: row 8 (e / 4) + 4 (l / 32) + e % 4, column l % 32
    const int col = wn + (l & 31);
    if (col >= ncol) return;
    const float bias = (!DG && a.b) ? a.b[col] : 0.0f;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int m = wm + 32 * i + 8 * (e >> 2) + 4 * (l >> 5) + (e & 3);
            const int64_t p = (int64_t(z0 + (m >> 6)) * a.H + (y0 + ((m >> 3) & 7))) * a.W + (x0 + (m & 7));
            if (DG) {
                dx[p * ncol + col] = acc[i][e];
                continue;
            }
            float v = acc[i][e] + bias;
            if (a.relu) v = fmaxf(v, 0.0f);
            if (a.y) a.y[p * a.cout + col] = f2bf(v);
            if (a.yf) a.yf[p * a.cout + col] = v;
        }
}

// packed forward weights: wt[o][t][c] = w[t][c][o]
__global__ void pack_weights_kernel(const uint16_t *w, int cin, int cout, uint16_t *wt) {
    const int n = 27 * cin * cout;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int o = e / (27 * cin), k = e % (27 * cin);
        wt[e] = w[k * cout + o];
    }
}

// g = BF16(dy (y > 0)) (or BF16(dy) without the ReLU)
__global__ void relu_grad_kernel(const float *dy, const uint16_t *y, int64_t n, int relu, uint16_t *g) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const float v = (relu && !(bf2f(y[i]) > 0.0f)) ? 0.0f : dy[i];
        g[i] = f2bf(v);
    }
}


// Weight gradient as one GEMM over all taps: C[(t, c)][o] = sum_p x[p + o_t][c]
// g[p][o], M = 27 cin rows in dw's own (tap-major) order, N = cout, K = the
// positions of one chunk; chunks add their partial sums with FP32 atomics.
// Operands are staged K-contiguous ([row][position]): each thread loads 8
// channels of one position (16 bytes) and scatters them down a column.  A
// g tile serves every tap of the row tile.
template <int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(256) conv_wgrad_kernel(ConvArgs a, const uint16_t *g, float *dw, int chunk) {
    constexpr int MB = BM / WM / 32, NB = BN / WN / 32;
    static_assert(WM * WN == 4 && MB * WM * 32 == BM && NB * WN * 32 == BN, "tile shape");
    constexpr int XL = BM / 64, GL = BN / 64;  // loads per thread (0: the first 4 BM or 4 BN threads)
    constexpr int XLT = XL > 0 ? XL : 1, GLT = GL > 0 ? GL : 1;
    __shared__ __attribute__((aligned(16))) uint16_t Xs[2][BM * LDK];
    __shared__ __attribute__((aligned(16))) uint16_t Gs[2][BN * LDK];
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
    const int P = a.D * a.H * a.W, HW = a.H * a.W;
    const int cin = a.c1 + a.c2;
    const int M = 27 * cin;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.z * BN;
    const int wm = (wv / WN) * MB * 32, wn = (wv % WN) * NB * 32;
    const int pbeg = blockIdx.x * chunk, pend = min(P, pbeg + chunk);
    const int pl = tid & 31;
    const int H2 = a.H >> 1, W2 = a.W >> 1;

    // x loads: rows m0 + 8 rg .. + 7 (tap t, channels c .. c + 7), position pl
    int xc[XLT], xr[XLT], xdz[XLT], xdy[XLT], xdx[XLT];
    bool xon[XLT];
#pragma unroll
    for (int j = 0; j < XLT; ++j) {
        const int rg = (tid >> 5) + 8 * j;
        xr[j] = 8 * rg;
        const int r = m0 + xr[j];
        xon[j] = (XL > 0 || tid < 4 * BM) && r < M;
        const int t = xon[j] ? r / cin : 13;
        xc[j] = r % cin;
        xdz[j] = t / 9 - 1;
        xdy[j] = (t / 3) % 3 - 1;
        xdx[j] = t % 3 - 1;
    }
    int go[GLT];
    bool gon[GLT];
#pragma unroll
    for (int j = 0; j < GLT; ++j) {
        go[j] = 8 * ((tid >> 5) + 8 * j);
        gon[j] = (GL > 0 || tid < 4 * BN) && n0 + go[j] < a.cout;
    }
    // this thread's position, advanced by BK per stage
    int cp = pbeg + pl, cw = cp % a.W, chh = (cp / a.W) % a.H, cd = cp / HW;

    uint4 rx[XLT], rg[GLT];
    bool xok[XLT], gok[GLT];
    auto load = [&]() {
        const bool valid = cp < pend;
#pragma unroll
        for (int j = 0; j < XLT; ++j) {
            const int qd = cd + xdz[j], qh = chh + xdy[j], qw = cw + xdx[j];
            const bool ok = valid && xon[j] && unsigned(qd) < unsigned(a.D) && unsigned(qh) < unsigned(a.H) &&
                            unsigned(qw) < unsigned(a.W);
            const int c = xc[j];
            const uint16_t *src;
            if (c < a.c1)
                src = a.up1 ? a.x1 + (((qd >> 1) * H2 + (qh >> 1)) * W2 + (qw >> 1)) * a.c1 + c
                            : a.x1 + ((qd * a.H + qh) * a.W + qw) * a.c1 + c;
            else
                src = a.x2 + ((qd * a.H + qh) * a.W + qw) * a.c2 + (c - a.c1);
            rx[j] = *reinterpret_cast<const uint4 *>(ok ? src : a.x1);
            xok[j] = ok;
        }
#pragma unroll
        for (int j = 0; j < GLT; ++j) {
            const bool ok = valid && gon[j];
            rg[j] = *reinterpret_cast<const uint4 *>(ok ? g + cp * a.cout + n0 + go[j] : g);
            gok[j] = ok;
        }
    };
    auto advance = [&]() {
        cp += BK;
        cw += BK;
        while (cw >= a.W) {
            cw -= a.W;
            if (++chh >= a.H) {
                chh = 0;
                ++cd;
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int j = 0; j < XLT; ++j) {
            if (!(XL > 0 || tid < 4 * BM)) continue;
            const uint4 w = xok[j] ? rx[j] : make_uint4(0, 0, 0, 0);
            const uint16_t *v = reinterpret_cast<const uint16_t *>(&w);
#pragma unroll
            for (int e = 0; e < 8; ++e) Xs[buf][(xr[j] + e) * LDK + pl] = v[e];
        }
#pragma unroll
        for (int j = 0; j < GLT; ++j) {
            if (!(GL > 0 || tid < 4 * BN)) continue;
            const uint4 w = gok[j] ? rg[j] : make_uint4(0, 0, 0, 0);
            const uint16_t *v = reinterpret_cast<const uint16_t *>(&w);
#pragma unroll
            for (int e = 0; e < 8; ++e) Gs[buf][(go[j] + e) * LDK + pl] = v[e];
        }
    };

    v16f acc[MB][NB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

    const int nst = (pend - pbeg + BK - 1) / BK;
    load();
    store(0);
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
        const int cur = st & 1;
        if (st + 1 < nst) {
            advance();
            load();
        }
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            v8bf fa[MB], fb[NB];
#pragma unroll
            for (int i = 0; i < MB; ++i)
                fa[i] = *reinterpret_cast<const v8bf *>(&Xs[cur][(wm + 32 * i + (l & 31)) * LDK + kk + 8 * (l >> 5)]);
#pragma unroll
            for (int j = 0; j < NB; ++j)
                fb[j] = *reinterpret_cast<const v8bf *>(&Gs[cur][(wn + 32 * j + (l & 31)) * LDK + kk + 8 * (l >> 5)]);
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        }
        if (st + 1 < nst) store(cur ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int col = n0 + wn + 32 * j + (l & 31);
            if (col >= a.cout) continue;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = m0 + wm + 32 * i + 8 * (e >> 2) + 4 * (l >> 5) + (e & 3);
                if (row < M) atomicAdd(dw + int64_t(row) * a.cout + col, acc[i][j][e]);
            }
        }
}

// bias gradient: db[o] += sum_p g[p, o] over a chunk of positions.  Each
// thread reads 8 channels (16 bytes) of one position per iteration, 256 /
// (channel groups) positions side by side; the sums are combined in LDS and
// added with one FP32 atomic per channel and chunk (one thread per channel).
__global__ void conv_bgrad_kernel(int P, int cout, int chunk, const uint16_t *g, float *db) {
    __shared__ float part[256][9];
    const int ng = cout >> 3;  // groups of 8 channels (cout is a multiple of 8)
    const int pbeg = blockIdx.x * chunk, pend = min(P, pbeg + chunk);
    const int t = threadIdx.x;
    for (int g0 = 0; g0 < ng; g0 += 256) {
        const int gw = min(ng - g0, 256), rows = 256 / gw;
        const int gi = g0 + t % gw, r = t / gw;
        float acc[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        if (r < rows)
#pragma unroll 8
            for (int p = pbeg + r; p < pend; p += rows) {
                const uint4 v = *reinterpret_cast<const uint4 *>(g + int64_t(p) * cout + 8 * gi);
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    acc[2 * q] += __uint_as_float(w[q] << 16);
                    acc[2 * q + 1] += __uint_as_float(w[q] & 0xFFFF0000u);
                }
            }
#pragma unroll
        for (int q = 0; q < 8; ++q) part[t][q] = acc[q];
        __syncthreads();
        // one channel per thread, so one atomic instruction covers the block's channels
        if (t < 8 * gw) {
            const int gt = t >> 3, q = t & 7;
            float tot = 0.0f;
            for (int rr = 0; rr < rows; ++rr) tot += part[rr * gw + gt][q];
            atomicAdd(db + 8 * g0 + t, tot);
        }
        __syncthreads();
    }
}

// split-K forward epilogue: y = ReLU(acc + b) in BF16 and/or FP32
__global__ void conv_finalize_kernel(ConvArgs a, const float *acc) {
    const int64_t n = int64_t(a.D) * a.H * a.W * a.cout;
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
        float v = acc[e] + (a.b ? a.b[e % a.cout] : 0.0f);
        if (a.relu) v = fmaxf(v, 0.0f);
        if (a.y) a.y[e] = f2bf(v);
        if (a.yf) a.yf[e] = v;
    }
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

// network input: y[:, c] = BF16((x[:, c] - shift[c]) * gain[c]) on [P][8] cells
__global__ void normalize_kernel(const float *x, int64_t P, ChanScale shift, ChanScale gain, uint16_t *y) {
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < P * 8; e += int64_t(gridDim.x) * blockDim.x) {
        const int c = int(e & 7);
        y[e] = f2bf((x[e] - shift.s[c]) * gain.s[c]);
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
// (Shan-Chen force F of the fused step, velocity shift of the collision).  The stored state is the
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

// Largest lifted speed: half the lattice's |u| > 0.3 stability flag.  A
// predicted canvas can hold negative densities or such speeds, which the
// method's own states never do; the lift maps each prolonged node back: rho_k
// clamped at 0, u scaled down to this speed with its direction kept.
constexpr double kLiftSpeedMax = 0.15;

__device__ inline void make_admissible(double a[5]) {
    a[0] = fmax(a[0], 0.0);
    a[1] = fmax(a[1], 0.0);
    const double sp = sqrt(a[2] * a[2] + a[3] * a[3] + a[4] * a[4]);
    if (sp > kLiftSpeedMax) {
        const double sc = kLiftSpeedMax / sp;
        for (int d = 2; d < 5; ++d) a[d] *= sc;
    }
}

// The lift keeps each component's mass: after the admissible map, rho_k on
// the fluid nodes is scaled by s_k = (canvas total of rho_k x fluid nodes of
// each cell) / (lifted total), when both totals are positive.  First the
// lifted totals, per block in a fixed order (grid-stride nodes per thread,
// then a tree over the block) ...
__global__ void __launch_bounds__(256) lift_mass_kernel(const float *coarse, int H, int W, SurLattice L, double *part) {
    __shared__ double red[2][256];
    const int64_t n_all = int64_t(L.nx) * L.ny * L.nz;
    double t[2] = {0.0, 0.0};
    for (int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; n < n_all; n += int64_t(gridDim.x) * blockDim.x) {
        if ((L.mat[n] & MAT_ID_MASK) != MAT_FLUID) continue;
        const int x = int(n % L.nx), y = int((n / L.nx) % L.ny), z = int(n / (int64_t(L.nx) * L.ny));
        double a[5];
        prolong_at(coarse, H, W, L.nz / 2, L.ny / 2, L.nx / 2, x, y, z, a);
        make_admissible(a);
        t[0] += a[0];
        t[1] += a[1];
    }
    red[0][threadIdx.x] = t[0];
    red[1][threadIdx.x] = t[1];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x < 2) part[2 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// ... then, in one work-group, the canvas totals over the cells inside the
// lattice, the blocks' totals in block order, and the two factors
__global__ void __launch_bounds__(256) lift_scale_kernel(const float *coarse, int H, int W, SurLattice L,
                                                         const double *part, int nb, double *scale) {
    __shared__ double red[4][256];
    const int ncz = L.nz / 2, ncy = L.ny / 2, ncx = L.nx / 2;
    const int64_t ncell = int64_t(ncz) * ncy * ncx;
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t c = threadIdx.x; c < ncell; c += blockDim.x) {
        const int cx = int(c % ncx), cy = int((c / ncx) % ncy), cz = int(c / (int64_t(ncx) * ncy));
        const float *cc = coarse + ((int64_t(cz) * H + cy) * W + cx) * 8;
        const double nf = 8.0 * double(cc[7]);
        t[0] += double(cc[0]) * nf;
        t[1] += double(cc[1]) * nf;
    }
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        t[2] += part[2 * b];
        t[3] += part[2 * b + 1];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = t[q];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 2) {
        const double want = red[threadIdx.x][0], have = red[2 + threadIdx.x][0];
        scale[threadIdx.x] = (want > 0.0 && have > 0.0) ? want / have : 1.0;
    }
}

// psi_k of the lifted state: prolonged rho_k on fluid nodes, the material's value elsewhere
__global__ void psi_lift_kernel(const float *coarse, int H, int W, SurLattice L, const double *scale) {
    const int64_t n_all = int64_t(L.nx) * L.ny * L.nz;
    for (int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; n < n_all; n += int64_t(gridDim.x) * blockDim.x) {
        const uint8_t m = L.mat[n];
        double v[2];
        if ((m & MAT_ID_MASK) == MAT_FLUID) {
            const int x = int(n % L.nx), y = int((n / L.nx) % L.ny), z = int(n / (int64_t(L.nx) * L.ny));
            double a[5];
            prolong_at(coarse, H, W, L.nz / 2, L.ny / 2, L.nx / 2, x, y, z, a);
            make_admissible(a);
            v[0] = a[0] * scale[0];
            v[1] = a[1] * scale[1];
        } else {
            v[0] = psi_solid(L, m, 0);
            v[1] = psi_solid(L, m, 1);
        }
        L.psi[n] = v[0];
        L.psi[n_all + n] = v[1];
    }
}

template <class S>
__global__ void lift_kernel(const float *coarse, int H, int W, SurLattice L, const double *scale, S *f) {
    const int64_t n_all = int64_t(L.nx) * L.ny * L.nz;
    for (int64_t n = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; n < n_all; n += int64_t(gridDim.x) * blockDim.x) {
        if ((L.mat[n] & MAT_ID_MASK) != MAT_FLUID) continue;
        const int x = int(n % L.nx), y = int((n / L.nx) % L.ny), z = int(n / (int64_t(L.nx) * L.ny));
        double a[5];
        prolong_at(coarse, H, W, L.nz / 2, L.ny / 2, L.nx / 2, x, y, z, a);
        make_admissible(a);
        const double rho[2] = {a[0] * scale[0], a[1] * scale[1]};
        double F[2][3];
        force_at(L, x, y, z, rho, F);
        const double tot = rho[0] + rho[1];
        const double ih = tot > 1e-12 ? 0.5 / tot : 0.0;  // no shift where the density vanishes
        double up[3];
        for (int d = 0; d < 3; ++d) up[d] = a[2 + d] - (F[0][d] + F[1][d]) * ih;
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

template <bool DGRAD>
static hipError_t launch_gemm(const ConvArgs &a, const uint16_t *g, float *dx, float *acc, hipStream_t s) {
    const int P = a.D * a.H * a.W;
    const int N = DGRAD ? a.c1 + a.c2 : a.cout;
    const int kc = DGRAD ? a.cout : a.c1 + a.c2;
    const int nst = (27 * kc + BK - 1) / BK;
    // 256-row tiles while they give at least ~2 work-groups per CU, else 128;
    // layers with fewer tiles than that split K over up to 512 work-groups
    // (at least 8 stages each) when there is somewhere to add the partials
    const int bn = N <= 32 ? 32 : (N <= 64 ? 64 : 128);
    const unsigned ny = unsigned((N + bn - 1) / bn);
    const bool big = int64_t((P + 255) / 256) * ny >= 512;
    const unsigned gx = unsigned(big ? (P + 255) / 256 : (P + 127) / 128);
    unsigned gz = 1;
    if ((DGRAD || acc) && gx * ny < 256) gz = unsigned(std::max(1, std::min(nst / 8, int(512 / (gx * ny)))));
    if (gz > 1) {
        float *dst = DGRAD ? dx : acc;
        const int64_t n = int64_t(P) * N;
        hipLaunchKernelGGL(fill_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, dst, n, 0.0f);
    }
    const dim3 grid(gx, ny, gz);
    if (N <= 32) {
        if (big)
            hipLaunchKernelGGL((conv_gemm_kernel<256, 32, 4, 1, DGRAD>), grid, dim3(256), 0, s, a, g, dx, acc);
        else
            hipLaunchKernelGGL((conv_gemm_kernel<128, 32, 4, 1, DGRAD>), grid, dim3(256), 0, s, a, g, dx, acc);
    } else if (N <= 64) {
        if (big)
            hipLaunchKernelGGL((conv_gemm_kernel<256, 64, 4, 1, DGRAD>), grid, dim3(256), 0, s, a, g, dx, acc);
        else
            hipLaunchKernelGGL((conv_gemm_kernel<128, 64, 2, 2, DGRAD>), grid, dim3(256), 0, s, a, g, dx, acc);
    } else {
        if (big)
            hipLaunchKernelGGL((conv_gemm_kernel<256, 128, 2, 2, DGRAD>), grid, dim3(256), 0, s, a, g, dx, acc);
        else
            hipLaunchKernelGGL((conv_gemm_kernel<128, 128, 2, 2, DGRAD>), grid, dim3(256), 0, s, a, g, dx, acc);
    }
    if (!DGRAD && gz > 1)
        hipLaunchKernelGGL(conv_finalize_kernel, dim3(grid_for(int64_t(P) * N)), dim3(256), 0, s, a, acc);
    return hipGetLastError();
}

hipError_t launch_conv_fwd(const ConvArgs &a, float *acc, hipStream_t s) {
    // volumes of whole bricks: the halo-staged kernel (4 x 8 x 8 bricks for up
    // to 32 output channels, 2 x 8 x 8 for up to 64)
    if (a.H % BRY == 0 && a.W % BRX == 0) {
        const int nxy = (a.H / BRY) * (a.W / BRX);
        if (a.cout <= 32 && a.D % 4 == 0) {
            hipLaunchKernelGGL((conv_brick_kernel<4, 1, false>), dim3(unsigned(nxy * (a.D / 4))), dim3(256), 0, s, a,
                               nullptr, nullptr);
            return hipGetLastError();
        }
        if (a.cout <= 64 && a.D % 2 == 0) {
            hipLaunchKernelGGL((conv_brick_kernel<2, 2, false>), dim3(unsigned(nxy * (a.D / 2))), dim3(256), 0, s, a,
                               nullptr, nullptr);
            return hipGetLastError();
        }
    }
    return launch_gemm<false>(a, nullptr, nullptr, acc, s);
}

hipError_t launch_conv_dgrad(const ConvArgs &a, const uint16_t *g, float *dx, hipStream_t s) {
    // volumes of whole bricks: the halo-staged kernel over g with mirrored taps
    const int cin = a.c1 + a.c2;
    if (a.H % BRY == 0 && a.W % BRX == 0) {
        const int nxy = (a.H / BRY) * (a.W / BRX);
        if (cin <= 32 && a.D % 4 == 0) {
            hipLaunchKernelGGL((conv_brick_kernel<4, 1, true>), dim3(unsigned(nxy * (a.D / 4))), dim3(256), 0, s, a, g,
                               dx);
            return hipGetLastError();
        }
        if (cin <= 64 && a.D % 2 == 0) {
            hipLaunchKernelGGL((conv_brick_kernel<2, 2, true>), dim3(unsigned(nxy * (a.D / 2))), dim3(256), 0, s, a, g,
                               dx);
            return hipGetLastError();
        }
    }
    return launch_gemm<true>(a, g, dx, nullptr, s);
}

hipError_t launch_conv_wgrad(const ConvArgs &a, const uint16_t *g, float *dw, float *db, hipStream_t s) {
    const int P = a.D * a.H * a.W;
    const int M = 27 * (a.c1 + a.c2);
    // position chunks: the longest (256 to 16384 positions) that still give
    // about 1024 work-groups for the 256-row tiles (the full-resolution
    // layers need the occupancy) and about 256 for the others (there the
    // FP32 atomics of each work-group's tile into dw weigh more)
    auto launch = [&](auto kern, int BM, int BN) {
        const unsigned tm = unsigned((M + BM - 1) / BM), tn = unsigned((a.cout + BN - 1) / BN);
        const int64_t target = BM == 256 ? 1024 : 256;
        int chunk = 16384;
        while (chunk > 256 && int64_t((P + chunk - 1) / chunk) * tm * tn < target) chunk /= 2;
        hipLaunchKernelGGL(kern, dim3(unsigned((P + chunk - 1) / chunk), tm, tn), dim3(256), 0, s, a, g, dw, chunk);
    };
    if (a.cout <= 32)
        launch(conv_wgrad_kernel<256, 32, 4, 1>, 256, 32);
    else if (a.cout <= 64)
        launch(conv_wgrad_kernel<128, 64, 2, 2>, 128, 64);
    else
        launch(conv_wgrad_kernel<128, 128, 2, 2>, 128, 128);
    if (db) {
        // about 512 chunks (at least 128 positions each)
        const int chunk = std::max(128, (P + 511) / 512);
        hipLaunchKernelGGL(conv_bgrad_kernel, dim3(unsigned((P + chunk - 1) / chunk)), dim3(256), 0, s, P, a.cout, chunk,
                           g, db);
    }
    return hipGetLastError();
}

hipError_t launch_pack_weights(const uint16_t *w, int cin, int cout, uint16_t *wt, hipStream_t s) {
    hipLaunchKernelGGL(pack_weights_kernel, dim3(grid_for(int64_t(27) * cin * cout)), dim3(256), 0, s, w, cin, cout, wt);
    return hipGetLastError();
}

hipError_t launch_relu_grad(const float *dy, const uint16_t *y, int64_t n, int relu, uint16_t *g, hipStream_t s) {
    hipLaunchKernelGGL(relu_grad_kernel, dim3(grid_for(n)), dim3(256), 0, s, dy, y, n, relu, g);
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

hipError_t launch_normalize(const float *x, int64_t P, const ChanScale &shift, const ChanScale &gain, uint16_t *y,
                            hipStream_t s) {
    hipLaunchKernelGGL(normalize_kernel, dim3(grid_for(P * 8)), dim3(256), 0, s, x, P, shift, gain, y);
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
    const int64_t n_all = int64_t(L.nx) * L.ny * L.nz;
    const int gn = grid_for(n_all);
    // the block totals and the two factors follow psi in the scratch buffer
    // (the other population buffer: 2 Q fs elements of at least 2 bytes,
    // against 8 (2 n_all + 2 gn + 2) bytes here)
    double *part = L.psi + 2 * n_all;
    double *scale = part + 2 * gn;
    if ((2 * n_all + 2 * int64_t(gn) + 2) * 8 > 2 * int64_t(Q) * L.fs * 2) return hipErrorInvalidValue;
    return by_prec(prec, [&](auto *tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        hipLaunchKernelGGL(lift_mass_kernel, dim3(gn), dim3(256), 0, s, coarse, H, W, L, part);
        hipLaunchKernelGGL(lift_scale_kernel, dim3(1), dim3(256), 0, s, coarse, H, W, L, part, gn, scale);
        hipLaunchKernelGGL(psi_lift_kernel, dim3(gn), dim3(256), 0, s, coarse, H, W, L, scale);
        hipLaunchKernelGGL(lift_kernel<S>, dim3(gn), dim3(256), 0, s, coarse, H, W, L, scale, static_cast<S *>(f));
        return hipGetLastError();
    });
}

}  // namespace lbm
