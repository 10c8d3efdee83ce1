// Warm-start network on the GPU: a multilayer perceptron (3 inputs, hidden layers of width
// 128 with tanh, 3 outputs) trained with Adam on steady fields the solver produced.
//
// The 128 x 128 hidden-to-hidden products run on the matrix cores (bf16 operands, fp32
// accumulation, v_mfma_f32_32x32x16_bf16); the thin input and output layers (3 wide), the
// bias additions, tanh and its derivative, the loss and Adam run in fp32.
//
// Inference: a block of four waves per 64 samples.  Training step (three launches, then Adam):
//   mlp_train_kernel   forward and backward of 32 samples per block of four waves; wave w owns
//                      features 32 w .. 32 w + 31 of every layer, and each lane keeps its 16
//                      activations per layer in registers from the forward to the backward
//                      (the product that maps dE/dz_l back to layer l - 1 leaves its results in
//                      the same lanes as the forward product of layer l - 1 did); writes the
//                      bf16 transposes of h_l and dE/dz_l, in blocks of 16 samples
//                      ([layer][sample / 16][feature][16]: a wave's operand of one 16-sample
//                      step of the weight gradient is 1 KB of contiguous memory), and the
//                      block's gradient of every parameter that is not a hidden-to-hidden weight;
//   mlp_wgrad_kernel   dE/dW_l = sum_s dz_l[s]^T h_{l-1}[s] of the hidden layers over slices of
//                      256 samples on the matrix cores (eight waves per slice and layer);
//   mlp_reduce_kernel  slices and blocks summed in a fixed order (the gradient is
//                      reproducible to the bit), and the loss; in a training loop it also
//                      applies Adam, which writes the bf16 weight copies of the next step
//                      (mlp_adam_kernel: the same update on its own).
//
// MFMA 32x32x16 lane layout (lane l, 8 bf16 per operand register, 16 fp32 results):
//   A[i][k]: i = l % 32, k = 8 (l / 32) + t;   B[k][j]: j = l % 32, k = 8 (l / 32) + t;
//   D[i][j]: result r has i = 8 (r / 4) + 4 (l / 32) + r % 4, j = l % 32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "fdlb_internal.h"

namespace fdlb {

namespace {

constexpr int MW = MLP_WIDTH;        // 128
constexpr int TS = MLP_TILE;         // samples per inference block
constexpr int TT = MLP_TRAIN_TILE;   // samples per training block
constexpr int SL = MLP_SLICE;        // samples per weight-gradient block
constexpr int RS = MW + 8;           // bf16 row stride of [sample][feature] LDS tiles
constexpr int HS = MW + 1;           // fp32 row stride of [sample][feature] LDS tiles
static_assert(TT == 32 && SL % TT == 0, "the training tile is one 32-row MFMA tile");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// fp32 -> bf16 bits, round to nearest even (inputs are finite).
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {  // 16-byte aligned
    return __builtin_bit_cast(bf16x8, *(const u16x8*)p);
}

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// tanh in fp32 without branches: below |x| = 0.25 the odd Taylor polynomial to x^9 (the first
// omitted term, 1382 x^11 / 155925, is under 1e-8 of tanh x there); above it
// (1 - e^{-2|x|}) / (1 + e^{-2|x|}) with the hardware exp2 and reciprocal (1 - e^{-2|x|} >= 0.39
// there, so the quotient keeps a few ulp), and the sign of x.  Both are formed (the polynomial
// on x clamped to [-0.25, 0.25], so it stays finite) and blended with an exact 0/1 weight: a
// select here is compiled into two divergent branches per call.
__device__ __forceinline__ float tanh_fast(float x) {
    const float t = fabsf(x);
    const float e = __builtin_amdgcn_exp2f(-2.88539008177792681f * t);  // 2 log2(e) |x|
    const float big = copysignf((1.f - e) * __builtin_amdgcn_rcpf(1.f + e), x);
    const float xs = fminf(fmaxf(x, -0.25f), 0.25f);
    const float x2 = xs * xs;
    const float small =
        xs * (1.f + x2 * (-1.f / 3.f + x2 * (2.f / 15.f + x2 * (-17.f / 315.f + x2 * (62.f / 2835.f)))));
    const float m = t < 0.25f ? 1.f : 0.f;
    return m * small + (1.f - m) * big;
}

// Encoded input of cell (ix, iy) of an nx x ny grid on the unit square.
__device__ __forceinline__ void cell_features(float kn_feat, int64_t cell, int nx, int ny, float* a) {
    const int ix = (int)(cell % nx), iy = (int)(cell / nx);
    a[0] = kn_feat;
    a[1] = (float)(2.0 * (ix + 0.5) / nx - 1.0);
    a[2] = (float)(2.0 * (iy + 0.5) / ny - 1.0);
}

__device__ __forceinline__ const float* row_ptr(const float* base, const int32_t* rows, int64_t g) {
    return base + 3 * (rows ? (int64_t)rows[g] : g);
}

// Load the encoded inputs of the block's NS samples into a_s (zeros past n).
template <int NS>
__device__ __forceinline__ void load_inputs(const MlpArgs& A, int64_t s0, float (*a_s)[3]) {
    const int t = threadIdx.x;
    if (t < NS) {
        const int64_t g = s0 + t;
        float a[3] = {0.f, 0.f, 0.f};
        if (g < A.n) {
            if (A.cells_nx > 0) {
                cell_features(A.kn_feat, g, A.cells_nx, A.cells_ny, a);
            } else {
                const float* p = row_ptr(A.in, A.rows, g);
                a[0] = p[0];
                a[1] = p[1];
                a[2] = p[2];
            }
        }
        a_s[t][0] = a[0];
        a_s[t][1] = a[1];
        a_s[t][2] = a[2];
    }
}

// One 64 x 128 product tile set of the block: wave w computes rows 32 (w & 1) .. +31 and
// columns 64 (w >> 1) .. +63 of  D[s][n] = sum_k X[s][k] Y[n][k],  X from LDS ([s][k], stride
// RS), Y from global bf16 ([n][k], stride MW).  K = 128.
__device__ __forceinline__ void tile_64x128(const uint16_t* X, const uint16_t* __restrict__ Y, f32x16& acc0,
                                            f32x16& acc1) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rb = wave & 1, cb = (wave >> 1) * 2;
    const int i = lane & 31, kq = 8 * (lane >> 5);
    acc0 = f32x16{};
    acc1 = f32x16{};
    const uint16_t* xr = X + (rb * 32 + i) * RS + kq;
    const uint16_t* y0 = Y + (int64_t)(cb * 32 + i) * MW + kq;
    const uint16_t* y1 = y0 + 32 * MW;
#pragma unroll
    for (int kk = 0; kk < MW; kk += 16) {
        const bf16x8 a = ld8(xr + kk);
        acc0 = mfma(a, ld8(y0 + kk), acc0);
        acc1 = mfma(a, ld8(y1 + kk), acc1);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Inference: outputs of 64 samples per block.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) mlp_forward_kernel(const MlpArgs A) {
    __shared__ float a_s[TS][3];
    __shared__ float wl_s[3][MW];  // W_L: the output layer reads it for every sample
    __shared__ float h32[TS][MW];
    __shared__ __attribute__((aligned(16))) uint16_t hb[TS * RS];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t s0 = (int64_t)blockIdx.x * TS;
    const float* P = A.params;
    load_inputs<TS>(A, s0, a_s);
    for (int e = t; e < 3 * MW; e += 256) wl_s[e / MW][e % MW] = P[A.off_w[A.hidden] + e];
    __syncthreads();

    // Input layer (3 -> 128), fp32.
    {
        const int o = t & (MW - 1), half = t >> 7;
        const float* W0 = P + A.off_w[0];
        const float w0 = W0[3 * o], w1 = W0[3 * o + 1], w2 = W0[3 * o + 2], b = P[A.off_b[0] + o];
        for (int s = half * 32; s < half * 32 + 32; ++s) {
            const float h = tanh_fast(b + w0 * a_s[s][0] + w1 * a_s[s][1] + w2 * a_s[s][2]);
            h32[s][o] = h;
            hb[s * RS + o] = to_bf16(h);
        }
    }

    // Hidden layers (128 -> 128) on the matrix cores.
    for (int l = 1; l < A.hidden; ++l) {
        __syncthreads();
        f32x16 acc0, acc1;
        tile_64x128(hb, A.wbf + (int64_t)(l - 1) * MW * MW, acc0, acc1);
        __syncthreads();  // every wave has read hb
        const int rb = wave & 1, cb = (wave >> 1) * 2;
        const float* b = P + A.off_b[l];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int s = rb * 32 + 8 * (r / 4) + 4 * (lane >> 5) + (r & 3);
            const int n0 = cb * 32 + (lane & 31), n1 = n0 + 32;
            const float h0 = tanh_fast(acc0[r] + b[n0]), h1 = tanh_fast(acc1[r] + b[n1]);
            h32[s][n0] = h0;
            h32[s][n1] = h1;
            hb[s * RS + n0] = to_bf16(h0);
            hb[s * RS + n1] = to_bf16(h1);
        }
    }
    __syncthreads();

    // Output layer (128 -> 3), fp32.
    if (t < TS * 3) {
        const int s = t / 3, o = t % 3;
        const int64_t g = s0 + s;
        float y = P[A.off_b[A.hidden] + o];
        for (int i = 0; i < MW; ++i) y += wl_s[o][i] * h32[s][i];
        if (g < A.n) {
            if (A.f_rho) {
                float* dst = o == 0 ? A.f_rho : o == 1 ? A.f_ux : A.f_uy;
                dst[g] = (o == 0 ? 1.0f : 0.0f) + A.u_w * y;
            } else {
                A.out[3 * g + o] = y;
            }
        }
    }
}

namespace {

// Sample row (within a 32-row tile) of result register r of this lane in the MFMA layout.
__device__ __forceinline__ int d_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// The B operands of a 32 x 32 x 128 product for this lane: rows 32 w + lane % 32 of a bf16
// [n][k] matrix (stride 128) in global memory, issued before the block meets at a barrier.
__device__ __forceinline__ void load_b(const uint16_t* __restrict__ Y, bf16x8 (&b)[MW / 16]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint16_t* yr = Y + (int64_t)(wave * 32 + (lane & 31)) * MW + 8 * (lane >> 5);
#pragma unroll
    for (int q = 0; q < MW / 16; ++q) b[q] = ld8(yr + 16 * q);
}

// D[s][32 w + j] = sum_k X[s][k] Y[32 w + j][k] for the 32 rows of X (LDS, [s][k], stride RS).
__device__ __forceinline__ f32x16 mma_32x32(const uint16_t* X, const bf16x8 (&b)[MW / 16]) {
    const int lane = threadIdx.x & 63;
    const uint16_t* xr = X + (lane & 31) * RS + 8 * (lane >> 5);
    f32x16 acc = f32x16{};
#pragma unroll
    for (int q = 0; q < MW / 16; ++q) acc = mfma(ld8(xr + 16 * q), b[q], acc);
    return acc;
}

// This lane's 16 values of feature n (rows d_row(r) of the tile of samples s0 .. s0 + 31) as bf16
// into one layer of a [sample / 16][feature][16] array: four 8-byte stores.
__device__ __forceinline__ void store_column(uint16_t* __restrict__ layer, int n, int64_t s0, const float (&v)[16]) {
    const int lane = threadIdx.x & 63;
    uint16_t* col = layer + ((s0 / 16) * MW + n) * 16 + 4 * (lane >> 5);
#pragma unroll
    for (int q = 0; q < 4; ++q) {  // samples s0 + 8 q + 4 (lane / 32) + 0..3
        uint2 w;
        w.x = (uint32_t)to_bf16(v[4 * q]) | ((uint32_t)to_bf16(v[4 * q + 1]) << 16);
        w.y = (uint32_t)to_bf16(v[4 * q + 2]) | ((uint32_t)to_bf16(v[4 * q + 3]) << 16);
        *(uint2*)(col + (q >> 1) * MW * 16 + 8 * (q & 1)) = w;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Training: forward and backward of 32 samples per block (H hidden layers).
// ---------------------------------------------------------------------------
template <int H>
__global__ void __launch_bounds__(256) mlp_train_kernel(const MlpArgs A) {
    __shared__ float a_s[TT][3];
    __shared__ float dy[TT][3];
    __shared__ float h32[TT][HS];                                      // h_{H-1}, fp32
    __shared__ float wl_s[3][MW];                                      // W_L
    __shared__ float bl_s[3];                                          // b_L
    __shared__ float t_s[TT][3];                                       // targets
    __shared__ __attribute__((aligned(16))) uint16_t hb[2][TT * RS];   // h_l, bf16, [s][i]
    __shared__ __attribute__((aligned(16))) uint16_t zb[2][TT * RS];   // dE/dz_l, bf16, [s][o]
    __shared__ double red[128];
    constexpr int TB = 4 * MW, TWL = 4 * MW + (H - 1) * MW;  // thin numbers of b_1 and W_L
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int n = wave * 32 + (lane & 31);  // this lane's feature in every layer
    const int64_t s0 = (int64_t)blockIdx.x * TT, ld = A.n_cap;
    const int nvalid = A.n - s0 < TT ? (int)(A.n - s0) : TT;
    const float* P = A.params;
    float* TP = A.part_thin + blockIdx.x;  // thin parameter k of this block at TP[k nb_cap]
    const int64_t tst = A.nb_cap;
    float hreg[H][16];
    // Everything small the block reads, requested at once: the samples' inputs and targets and
    // W_L, b_L (LDS), this lane's row of W_0 and its biases (registers), and the first weights
    // of the matrix cores (each product's weights are then requested one layer ahead).
    if (t < TT) {
        const int64_t g = s0 + t;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, y0 = 0.f, y1 = 0.f, y2 = 0.f;
        if (g < A.n) {
            const float* in = row_ptr(A.in, A.rows, g);
            const float* tg = row_ptr(A.target, A.rows, g);
            a0 = in[0], a1 = in[1], a2 = in[2];
            y0 = tg[0], y1 = tg[1], y2 = tg[2];
        }
        a_s[t][0] = a0, a_s[t][1] = a1, a_s[t][2] = a2;
        t_s[t][0] = y0, t_s[t][1] = y1, t_s[t][2] = y2;
    }
    for (int e = t; e < 3 * MW; e += 256) wl_s[e / MW][e % MW] = P[A.off_w[H] + e];
    if (t < 3) bl_s[t] = P[A.off_b[H] + t];
    const float* W0 = P + A.off_w[0];
    const float w0 = W0[3 * n], w1 = W0[3 * n + 1], w2 = W0[3 * n + 2];
    float bias[H];
#pragma unroll
    for (int l = 0; l < H; ++l) bias[l] = P[A.off_b[l] + n];
    bf16x8 wb[2][MW / 16];  // weights of the product in flight and of the next one
    if constexpr (H > 1) load_b(A.wbf, wb[1]);  // layer l multiplies by wb[l & 1]
    __syncthreads();

    // Input layer (3 -> 128), fp32.
    {
        const float b = bias[0];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int s = d_row(r, lane);
            const float h = tanh_fast(b + w0 * a_s[s][0] + w1 * a_s[s][1] + w2 * a_s[s][2]);
            hreg[0][r] = h;
            if (H > 1) hb[0][s * RS + n] = to_bf16(h);
            else h32[s][n] = h;
        }
        if (H > 1) store_column(A.hT, n, s0, hreg[0]);
    }

    // Hidden layers (128 -> 128) on the matrix cores; h_l alternates between the two buffers.
#pragma unroll
    for (int l = 1; l < H; ++l) {
        __syncthreads();  // h_{l-1} complete (and every read of the buffer written below done)
        const f32x16 acc = mma_32x32(hb[(l - 1) & 1], wb[l & 1]);
        // next product: layer l + 1, or the first of the backward pass (W_{H-1} transposed)
        if (l < H - 1) load_b(A.wbf + (int64_t)l * MW * MW, wb[(l + 1) & 1]);
        else load_b(A.wbfT + (int64_t)(H - 2) * MW * MW, wb[(l + 1) & 1]);
        const float b = bias[l];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int s = d_row(r, lane);
            const float h = tanh_fast(acc[r] + b);
            hreg[l][r] = h;
            if (l < H - 1) hb[l & 1][s * RS + n] = to_bf16(h);
            else h32[s][n] = h;
        }
        if (l < H - 1) store_column(A.hT + (int64_t)l * MW * ld, n, s0, hreg[l]);
    }
    __syncthreads();

    // Output layer (128 -> 3), fp32; dE/dy = 2 (y - t) / (3 n) and the squared errors.
    double e2 = 0.0;
    if (t < TT * 3) {
        const int s = t / 3, o = t % 3;
        float y = bl_s[o];
        for (int i = 0; i < MW; ++i) y += wl_s[o][i] * h32[s][i];
        float d = 0.f;
        if (s < nvalid) {
            const float e = y - t_s[s][o];
            e2 = (double)e * e;
            d = 2.0f * e * A.inv_3n;
        }
        dy[s][o] = d;
    }
    if (t < 128) red[t] = e2;
    __syncthreads();
    if (wave == 0) {
        double e = red[lane] + red[lane + 64];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
        if (lane == 0) A.loss_part[blockIdx.x] = e;
    }

    // Output layer: dE/dW_L = dy^T h_{H-1} (e < 384), dE/db_L = sum dy (e = 384 + o); rows past
    // the samples have dy = 0, so every sum runs over the whole tile, unrolled.
    for (int e = t; e < 3 * MW + 3; e += 256) {
        float acc = 0.f;
        if (e < 3 * MW) {
            const int o = e / MW, i = e % MW;
#pragma unroll
            for (int s = 0; s < TT; ++s) acc += dy[s][o] * h32[s][i];
        } else {
#pragma unroll
            for (int s = 0; s < TT; ++s) acc += dy[s][e - 3 * MW];
        }
        TP[(TWL + e) * tst] = acc;
    }

    // dE/dz of the last hidden layer: (W_L^T dy) (1 - h^2), in this lane's registers.
    float dz[16];
    {
        const float w0 = wl_s[0][n], w1 = wl_s[1][n], w2 = wl_s[2][n];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int s = d_row(r, lane);
            const float h = hreg[H - 1][r];
            dz[r] = (w0 * dy[s][0] + w1 * dy[s][1] + w2 * dy[s][2]) * (1.f - h * h);
        }
    }

    // Hidden-to-hidden layers, last to first: dE/db_l, the bf16 transpose of dE/dz_l for the
    // weight gradient, and dE/dh_{l-1} = dz_l W_l (W_l^T rows from the transposed copy).
#pragma unroll
    for (int l = H - 1; l >= 1; --l) {
        float sb = 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r) sb += dz[r];
        sb += __shfl_xor(sb, 32);  // the lane holding the other 16 samples of feature n
        if (lane < 32) TP[(TB + (l - 1) * MW + n) * tst] = sb;
        store_column(A.dzT + (int64_t)(l - 1) * MW * ld, n, s0, dz);
        uint16_t* zl = zb[l & 1];
#pragma unroll
        for (int r = 0; r < 16; ++r) zl[d_row(r, lane) * RS + n] = to_bf16(dz[r]);
        __syncthreads();  // dz_l complete (and every read of the buffer written above done)
        // W_l transposed was requested a product earlier, into wb[(l + 1) & 1] (the last forward
        // layer, H - 1, put W_{H-1} there as wb[H & 1])
        const f32x16 acc = mma_32x32(zl, wb[(l + 1) & 1]);
        if (l > 1) load_b(A.wbfT + (int64_t)(l - 2) * MW * MW, wb[l & 1]);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float h = hreg[l - 1][r];
            dz[r] = acc[r] * (1.f - h * h);
        }
    }

    // Input layer: dE/dW_0 = dz^T a, dE/db_0 = sum dz.
    {
        float g0 = 0.f, g1 = 0.f, g2 = 0.f, gb = 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int s = d_row(r, lane);
            g0 += dz[r] * a_s[s][0];
            g1 += dz[r] * a_s[s][1];
            g2 += dz[r] * a_s[s][2];
            gb += dz[r];
        }
        g0 += __shfl_xor(g0, 32);
        g1 += __shfl_xor(g1, 32);
        g2 += __shfl_xor(g2, 32);
        gb += __shfl_xor(gb, 32);
        if (lane < 32) {
            TP[(3 * n) * tst] = g0;
            TP[(3 * n + 1) * tst] = g1;
            TP[(3 * n + 2) * tst] = g2;
            TP[(3 * MW + n) * tst] = gb;
        }
    }
}

// dE/dW_l[o][i] = sum over the slice's samples of dz_l[s][o] h_{l-1}[s][i]; block (slice j,
// layer l) of eight waves, wave w owns rows o in 32 (w % 4) .. + 31 and columns i in
// 64 (w / 4) .. + 63.  A full slice is unrolled so that all its loads are in flight at once.
__global__ void __launch_bounds__(512) mlp_wgrad_kernel(const MlpArgs A) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rb = wave & 3, cb = wave >> 2;
    const int j = blockIdx.x, l = blockIdx.y + 1;
    const int64_t ld = A.n_cap;
    const int64_t n32 = (A.n + TT - 1) / TT * TT;  // samples written by the training kernel
    const int64_t k0 = (int64_t)j * SL, k1 = k0 + SL < n32 ? k0 + SL : n32;
    const int i32 = lane & 31, kq = 8 * (lane >> 5);
    // element (sample s, feature f) of a layer at ((s / 16) 128 + f) 16 + s % 16; k-step q of the
    // slice is 16 q samples, i.e. 2048 elements, further on
    const int64_t lay = (int64_t)(l - 1) * MW * ld, blk0 = k0 / 16 * MW;
    const uint16_t* za = A.dzT + lay + (blk0 + rb * 32 + i32) * 16 + kq;
    const uint16_t* h0 = A.hT + lay + (blk0 + cb * 64 + i32) * 16 + kq;
    const uint16_t* h1 = h0 + 32 * 16;
    constexpr int KST = MW * 16;
    f32x16 acc0 = f32x16{}, acc1 = f32x16{};
    const int nk = (int)((k1 - k0) / 16);
    if (nk == SL / 16) {
        // two halves: the loads of the second are in flight while the first is multiplied
        constexpr int NQ = SL / 32;
        bf16x8 a[2][NQ], b0[2][NQ], b1[2][NQ];
#pragma unroll
        for (int hf = 0; hf < 2; ++hf)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int k = KST * (hf * NQ + q);
                a[hf][q] = ld8(za + k);
                b0[hf][q] = ld8(h0 + k);
                b1[hf][q] = ld8(h1 + k);
            }
        __builtin_amdgcn_sched_barrier(0);  // keep every load of the slice ahead of the products
#pragma unroll
        for (int hf = 0; hf < 2; ++hf)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                acc0 = mfma(a[hf][q], b0[hf][q], acc0);
                acc1 = mfma(a[hf][q], b1[hf][q], acc1);
            }
    } else {
        for (int q = 0; q < nk; ++q) {
            const bf16x8 a = ld8(za + KST * q);
            acc0 = mfma(a, ld8(h0 + KST * q), acc0);
            acc1 = mfma(a, ld8(h1 + KST * q), acc1);
        }
    }
    float* pw = A.part_w + ((int64_t)j * (A.hidden - 1) + (l - 1)) * MW * MW;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        float* row = pw + (rb * 32 + d_row(r, lane)) * MW + cb * 64 + i32;
        row[0] = acc0[r];
        row[32] = acc1[r];
    }
}

namespace {
// Parameter index of thin parameter number k (numbering of mlp_thin_count).
__device__ __forceinline__ int thin_param(const MlpArgs& A, int k) {
    const int H = A.hidden;
    if (k < 4 * MW) return k;  // W_0 then b_0, contiguous from 0
    if (k < 4 * MW + (H - 1) * MW) {
        const int l = 1 + (k - 4 * MW) / MW;
        return A.off_b[l] + (k - 4 * MW) % MW;
    }
    return A.off_w[H] + (k - 4 * MW - (H - 1) * MW);  // W_L then b_L, contiguous
}
}  // namespace

// Adam (bias-corrected first and second moments), fp32, of parameter k with gradient gk; an
// updated hidden-to-hidden weight also goes to its bf16 copies ([o][i] and [i][o]) that the next
// training step multiplies by.  One function for the stand-alone update and the one fused into
// the gradient reduction, so both give the same bits.
__device__ __forceinline__ void adam_update(const MlpArgs& A, const AdamArgs& D, int k, float gk) {
    const float mk = D.b1 * D.m[k] + (1.f - D.b1) * gk;
    const float vk = D.b2 * D.v[k] + (1.f - D.b2) * gk * gk;
    D.m[k] = mk;
    D.v[k] = vk;
    const float pk = D.p[k] - D.lr * (mk * D.c1) / (sqrtf(vk * D.c2) + D.eps);
    D.p[k] = pk;
    for (int l = 1; l < A.hidden; ++l) {
        const int e = k - A.off_w[l];
        if (e >= 0 && e < MW * MW) {
            const uint16_t bb = to_bf16(pk);
            D.wbf[(int64_t)(l - 1) * MW * MW + e] = bb;
            D.wbfT[(int64_t)(l - 1) * MW * MW + (e % MW) * MW + e / MW] = bb;
        }
    }
}

// Gradient = the sum of the slice partials (hidden weights, a thread each, four running sums
// combined pairwise) and of the block partials (the other parameters, a wave each, lanes
// striding over the blocks and a butterfly across the wave), in a fixed order; loss = sum of
// squared errors / (3 n) (the last wave).  ADAM: the update follows, parameter by parameter.
template <bool ADAM>
__global__ void __launch_bounds__(256) mlp_reduce_kernel(const MlpArgs A, int nslices, int nblocks,
                                                         float* __restrict__ grad, double inv_3n,
                                                         double* __restrict__ loss, const AdamArgs D) {
    const int HW = (A.hidden - 1) * MW * MW;
    const int nA = HW / 256;
    if ((int)blockIdx.x < nA) {
        const int k = blockIdx.x * 256 + threadIdx.x;
        const float* p = A.part_w + k;
        // slice b goes to running sum b % 4, in increasing b; sixteen loads in flight
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
        int b = 0;
        for (; b + 16 <= nslices; b += 16) {
            float v[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = p[(int64_t)(b + q) * HW];
#pragma unroll
            for (int q = 0; q < 16; q += 4) {
                a0 += v[q];
                a1 += v[q + 1];
                a2 += v[q + 2];
                a3 += v[q + 3];
            }
        }
        for (; b + 4 <= nslices; b += 4) {
            a0 += p[(int64_t)b * HW];
            a1 += p[(int64_t)(b + 1) * HW];
            a2 += p[(int64_t)(b + 2) * HW];
            a3 += p[(int64_t)(b + 3) * HW];
        }
        if (b < nslices) a0 += p[(int64_t)b * HW];
        if (b + 1 < nslices) a1 += p[(int64_t)(b + 1) * HW];
        if (b + 2 < nslices) a2 += p[(int64_t)(b + 2) * HW];
        const int l = 1 + k / (MW * MW);
        const int kp = A.off_w[l] + k % (MW * MW);
        const float g = (a0 + a1) + (a2 + a3);
        grad[kp] = g;
        if (ADAM) adam_update(A, D, kp, g);
        return;
    }
    const int lane = threadIdx.x & 63;
    const int k = ((int)blockIdx.x - nA) * 4 + (threadIdx.x >> 6);
    const int T = mlp_thin_count(A.hidden);
    if (k < T) {
        const float* p = A.part_thin + (int64_t)k * A.nb_cap;
        float s = 0.f;
        for (int b = lane; b < nblocks; b += 64) s += p[b];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) {
            const int kp = thin_param(A, k);
            grad[kp] = s;
            if (ADAM) adam_update(A, D, kp, s);
        }
    } else if (k == T) {
        double e = 0.0;
        for (int b = lane; b < nblocks; b += 64) e += A.loss_part[b];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
        if (lane == 0) *loss = e * inv_3n;
    }
}

// Stand-alone Adam step of every parameter from the gradient buffer.
__global__ void __launch_bounds__(256) mlp_adam_kernel(const MlpArgs A, const float* __restrict__ g,
                                                       const AdamArgs D) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < A.P) adam_update(A, D, k, g[k]);
}

// bf16 copies of the hidden-to-hidden weights, as stored ([o][i]) and transposed ([i][o]).
__global__ void __launch_bounds__(256) mlp_weights_bf16_kernel(const MlpArgs A, uint16_t* __restrict__ wbf,
                                                               uint16_t* __restrict__ wbfT) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)(A.hidden - 1) * MW * MW;
    if (e >= total) return;
    const int l = (int)(e / (MW * MW)) + 1;
    const int o = (int)((e / MW) % MW), i = (int)(e % MW);
    const uint16_t b = to_bf16(A.params[A.off_w[l] + o * MW + i]);
    wbf[e] = b;
    wbfT[(int64_t)(l - 1) * MW * MW + i * MW + o] = b;
}

// Training samples from a solved state: encoded inputs of every cell and the fields scaled
// by the wall speed, ((rho - 1) / u_w, u_x / u_w, u_y / u_w).  post = [rho | ux | uy | ...].
__global__ void __launch_bounds__(256) field_samples_kernel(const double* __restrict__ post, int nx, int ny,
                                                            float kn_feat, double inv_uw, float* __restrict__ in,
                                                            float* __restrict__ target) {
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)nx * ny;
    if (cell >= n) return;
    float a[3];
    cell_features(kn_feat, cell, nx, ny, a);
    in[3 * cell] = a[0];
    in[3 * cell + 1] = a[1];
    in[3 * cell + 2] = a[2];
    target[3 * cell] = (float)((post[cell] - 1.0) * inv_uw);
    target[3 * cell + 1] = (float)(post[n + cell] * inv_uw);
    target[3 * cell + 2] = (float)(post[2 * n + cell] * inv_uw);
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
static unsigned grid_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

void launch_mlp_weights_bf16(const MlpArgs& a, uint16_t* wbf, uint16_t* wbfT, hipStream_t s) {
    const int64_t total = (int64_t)(a.hidden - 1) * MW * MW;
    if (total <= 0) return;
    hipLaunchKernelGGL(mlp_weights_bf16_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, a, wbf, wbfT);
    FDLB_HIP(hipGetLastError());
}

void launch_mlp_forward(const MlpArgs& a, hipStream_t s) {
    if (a.n <= 0) return;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(grid_for(a.n, TS)), dim3(256), 0, s, a);
    FDLB_HIP(hipGetLastError());
}

void launch_mlp_train(const MlpArgs& a, hipStream_t s) {
    if (a.n <= 0) return;
    const dim3 grid(grid_for(a.n, TT)), block(256);
    switch (a.hidden) {
#define FDLB_MLP_H(h) \
    case h: hipLaunchKernelGGL(mlp_train_kernel<h>, grid, block, 0, s, a); break;
        FDLB_MLP_H(1) FDLB_MLP_H(2) FDLB_MLP_H(3) FDLB_MLP_H(4) FDLB_MLP_H(5) FDLB_MLP_H(6) FDLB_MLP_H(7)
        FDLB_MLP_H(8)
#undef FDLB_MLP_H
        default: throw Error(FDLB_EINVAL, "hidden layers must be 1..8");
    }
    static_assert(MLP_MAX_HIDDEN == 8, "one instantiation per hidden-layer count");
    FDLB_HIP(hipGetLastError());
}

void launch_mlp_wgrad(const MlpArgs& a, hipStream_t s) {
    if (a.n <= 0 || a.hidden < 2) return;
    const int64_t n32 = (a.n + TT - 1) / TT * TT;
    hipLaunchKernelGGL(mlp_wgrad_kernel, dim3(grid_for(n32, SL), a.hidden - 1), dim3(512), 0, s, a);
    FDLB_HIP(hipGetLastError());
}

void launch_mlp_reduce(const MlpArgs& a, float* grad, double inv_3n, double* loss, const AdamArgs* adam,
                       hipStream_t s) {
    const int64_t n32 = (a.n + TT - 1) / TT * TT;
    const int nslices = (int)grid_for(n32, SL), nblocks = (int)grid_for(a.n, TT);
    const int nA = (a.hidden - 1) * MW * MW / 256, waves = mlp_thin_count(a.hidden) + 1;
    const dim3 grid(nA + grid_for(waves, 4)), block(256);
    if (adam)
        hipLaunchKernelGGL(mlp_reduce_kernel<true>, grid, block, 0, s, a, nslices, nblocks, grad, inv_3n, loss,
                           *adam);
    else
        hipLaunchKernelGGL(mlp_reduce_kernel<false>, grid, block, 0, s, a, nslices, nblocks, grad, inv_3n, loss,
                           AdamArgs{});
    FDLB_HIP(hipGetLastError());
}

void launch_mlp_adam(const MlpArgs& a, const float* g, const AdamArgs& adam, hipStream_t s) {
    hipLaunchKernelGGL(mlp_adam_kernel, dim3(grid_for(a.P, 256)), dim3(256), 0, s, a, g, adam);
    FDLB_HIP(hipGetLastError());
}

void launch_field_samples(const double* post, int nx, int ny, float kn_feat, double inv_uw, float* in, float* target,
                          hipStream_t s) {
    const int64_t n = (int64_t)nx * ny;
    hipLaunchKernelGGL(field_samples_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, post, nx, ny, kn_feat, inv_uw,
                       in, target);
    FDLB_HIP(hipGetLastError());
}

}  // namespace fdlb
