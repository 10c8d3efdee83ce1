// Warm-start network on the GPU: a multilayer perceptron (3 inputs, hidden layers of width
// 128 with tanh, 3 outputs) trained with Adam on steady fields the solver produced.
//
// The 128 x 128 hidden-to-hidden products run on the matrix cores (bf16 operands, fp32
// accumulation, v_mfma_f32_32x32x16_bf16); the thin input and output layers (3 wide), the
// bias additions, tanh and its derivative, the loss and Adam run in fp32.  One block of four
// waves owns a tile of 64 samples and keeps its activations in LDS.
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

constexpr int MW = MLP_WIDTH;   // 128
constexpr int TS = MLP_TILE;    // samples per block
constexpr int RS = MW + 8;      // bf16 row stride of [sample][feature] LDS tiles
constexpr int TSP = TS + 8;     // bf16 row stride of [feature][sample] LDS tiles

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

// Load the encoded inputs of the block's samples into a_s (zeros past n).
__device__ __forceinline__ void load_inputs(const MlpArgs& A, int64_t s0, float (*a_s)[3]) {
    const int t = threadIdx.x;
    if (t < TS) {
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
// Forward: inference (TRAIN = false) or the forward half of a training step, which also
// keeps every hidden activation (fp32) for the backward kernel.
// ---------------------------------------------------------------------------
template <bool TRAIN>
__global__ void __launch_bounds__(256) mlp_forward_kernel(const MlpArgs A) {
    __shared__ float a_s[TS][3];
    __shared__ float h32[TS][MW];
    __shared__ __attribute__((aligned(16))) uint16_t hb[TS * RS];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t s0 = (int64_t)blockIdx.x * TS;
    const float* P = A.params;
    load_inputs(A, s0, a_s);
    __syncthreads();

    // Input layer (3 -> 128), fp32.
    {
        const int o = t & (MW - 1), half = t >> 7;
        const float* W0 = P + A.off_w[0];
        const float w0 = W0[3 * o], w1 = W0[3 * o + 1], w2 = W0[3 * o + 2], b = P[A.off_b[0] + o];
        for (int s = half * 32; s < half * 32 + 32; ++s) {
            const float h = tanhf(b + w0 * a_s[s][0] + w1 * a_s[s][1] + w2 * a_s[s][2]);
            h32[s][o] = h;
            hb[s * RS + o] = to_bf16(h);
            if (TRAIN && s0 + s < A.n) A.act[(s0 + s) * MW + o] = h;  // layer 0 of act
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
            const float h0 = tanhf(acc0[r] + b[n0]), h1 = tanhf(acc1[r] + b[n1]);
            h32[s][n0] = h0;
            h32[s][n1] = h1;
            hb[s * RS + n0] = to_bf16(h0);
            hb[s * RS + n1] = to_bf16(h1);
            if (TRAIN && s0 + s < A.n) {
                float* act = A.act + ((int64_t)l * A.n_cap + s0 + s) * MW;
                act[n0] = h0;
                act[n1] = h1;
            }
        }
    }
    __syncthreads();

    // Output layer (128 -> 3), fp32.
    if (t < TS * 3) {
        const int s = t / 3, o = t % 3;
        const int64_t g = s0 + s;
        const float* WL = P + A.off_w[A.hidden] + o * MW;
        float y = P[A.off_b[A.hidden] + o];
        for (int i = 0; i < MW; ++i) y += WL[i] * h32[s][i];
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

// ---------------------------------------------------------------------------
// Backward: loss and the gradient of one tile of samples, written as this block's partial
// (every parameter once); mlp_reduce_kernel sums the partials in block order.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) mlp_backward_kernel(const MlpArgs A) {
    __shared__ float a_s[TS][3];
    __shared__ float dy[TS][3];
    __shared__ float d32[TS][MW];                                   // dE/dz of the current layer
    __shared__ __attribute__((aligned(16))) uint16_t dzb[TS * RS];  // same, bf16, [s][o]
    __shared__ __attribute__((aligned(16))) uint16_t dzT[MW * TSP]; // same, bf16, [o][s]
    __shared__ __attribute__((aligned(16))) uint16_t hT[MW * TSP];  // h of the layer below, bf16, [i][s]
    __shared__ double red[256];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t s0 = (int64_t)blockIdx.x * TS;
    const int H = A.hidden;
    const float* P = A.params;
    float* G = A.partial + (int64_t)blockIdx.x * A.P;
    auto act_row = [&](int l, int s) { return A.act + ((int64_t)l * A.n_cap + s0 + s) * MW; };
    const int nvalid = A.n - s0 < TS ? (int)(A.n - s0) : TS;
    load_inputs(A, s0, a_s);

    // dE/dy = 2 (y - t) / (3 n) and the block's share of the squared error.
    double e2 = 0.0;
    if (t < TS * 3) {
        const int s = t / 3, o = t % 3;
        float d = 0.f;
        if (s < nvalid) {
            const int64_t g = s0 + s;
            const float e = A.out[3 * g + o] - row_ptr(A.target, A.rows, g)[o];
            e2 = (double)e * e;
            d = 2.0f * e * A.inv_3n;
        }
        dy[s][o] = d;
    }
    red[t] = e2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) A.loss_part[blockIdx.x] = red[0];

    // Output layer: dE/dW_L = dy^T h_{L-1}, dE/db_L = sum dy.
    for (int e = t; e < 3 * MW; e += 256) {
        const int o = e / MW, i = e % MW;
        float acc = 0.f;
        for (int s = 0; s < nvalid; ++s) acc += dy[s][o] * act_row(H - 1, s)[i];
        G[A.off_w[H] + e] = acc;
    }
    if (t < 3) {
        float acc = 0.f;
        for (int s = 0; s < nvalid; ++s) acc += dy[s][t];
        G[A.off_b[H] + t] = acc;
    }
    // dE/dz of the last hidden layer: (W_L^T dy) (1 - h^2).
    {
        const int o = t & (MW - 1), half = t >> 7;
        const float* WL = P + A.off_w[H];
        const float w0 = WL[o], w1 = WL[MW + o], w2 = WL[2 * MW + o];
        for (int s = half * 32; s < half * 32 + 32; ++s) {
            float dz = 0.f;
            if (s < nvalid) {
                const float h = act_row(H - 1, s)[o];
                dz = (w0 * dy[s][0] + w1 * dy[s][1] + w2 * dy[s][2]) * (1.f - h * h);
            }
            d32[s][o] = dz;
            const uint16_t bz = to_bf16(dz);
            dzb[s * RS + o] = bz;
            dzT[o * TSP + s] = bz;
        }
    }

    // Hidden-to-hidden layers, last to first.
    for (int l = H - 1; l >= 1; --l) {
        {   // h_{l-1}, transposed, bf16
            const int i = t & (MW - 1), half = t >> 7;
            for (int s = half * 32; s < half * 32 + 32; ++s)
                hT[i * TSP + s] = to_bf16(s < nvalid ? act_row(l - 1, s)[i] : 0.f);
        }
        __syncthreads();
        if (t < MW) {
            float acc = 0.f;
            for (int s = 0; s < nvalid; ++s) acc += d32[s][t];
            G[A.off_b[l] + t] = acc;
        }
        {   // dE/dW_l[o][i] = sum_s dz[s][o] h[s][i]: wave w owns rows o in 32 w .. 32 w + 31.
            const int i32 = lane & 31, kq = 8 * (lane >> 5);
            f32x16 acc[4] = {f32x16{}, f32x16{}, f32x16{}, f32x16{}};
            const uint16_t* xa = dzT + (wave * 32 + i32) * TSP + kq;
#pragma unroll
            for (int kk = 0; kk < TS; kk += 16) {
                const bf16x8 a = ld8(xa + kk);
#pragma unroll
                for (int ib = 0; ib < 4; ++ib) acc[ib] = mfma(a, ld8(hT + (ib * 32 + i32) * TSP + kq + kk), acc[ib]);
            }
            float* gw = G + A.off_w[l];
#pragma unroll
            for (int ib = 0; ib < 4; ++ib)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int o = wave * 32 + 8 * (r / 4) + 4 * (lane >> 5) + (r & 3);
                    gw[o * MW + ib * 32 + i32] = acc[ib][r];
                }
        }
        // dE/dh_{l-1}[s][i] = sum_o dz[s][o] W_l[o][i]  (W_l^T rows from the transposed copy).
        f32x16 acc0, acc1;
        tile_64x128(dzb, A.wbfT + (int64_t)(l - 1) * MW * MW, acc0, acc1);
        __syncthreads();  // every wave is done with dzb, dzT, d32 and hT
        const int rb = wave & 1, cb = (wave >> 1) * 2;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int s = rb * 32 + 8 * (r / 4) + 4 * (lane >> 5) + (r & 3);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int i = (cb + c) * 32 + (lane & 31);
                float dz = 0.f;
                if (s < nvalid) {
                    const float h = act_row(l - 1, s)[i];
                    dz = (c == 0 ? acc0[r] : acc1[r]) * (1.f - h * h);
                }
                d32[s][i] = dz;
                const uint16_t bz = to_bf16(dz);
                dzb[s * RS + i] = bz;
                dzT[i * TSP + s] = bz;
            }
        }
        __syncthreads();
    }

    // Input layer: dE/dW_0 = dz^T a, dE/db_0 = sum dz.
    __syncthreads();
    if (t < MW) {
        float g0 = 0.f, g1 = 0.f, g2 = 0.f, gb = 0.f;
        for (int s = 0; s < nvalid; ++s) {
            const float d = d32[s][t];
            g0 += d * a_s[s][0];
            g1 += d * a_s[s][1];
            g2 += d * a_s[s][2];
            gb += d;
        }
        G[A.off_w[0] + 3 * t] = g0;
        G[A.off_w[0] + 3 * t + 1] = g1;
        G[A.off_w[0] + 3 * t + 2] = g2;
        G[A.off_b[0] + t] = gb;
    }
}

// Gradient = sum of the block partials (in block order); loss = sum of squared errors / (3 n).
__global__ void __launch_bounds__(256) mlp_reduce_kernel(const float* __restrict__ partial, int nblocks, int P,
                                                         float* __restrict__ grad, const double* __restrict__ loss_part,
                                                         double inv_3n, double* __restrict__ loss) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < P) {
        // four independent running sums (blocks b = 4i + j go to sum j), combined pairwise: a
        // fixed order, with four loads in flight instead of one dependent chain
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
        int b = 0;
        for (; b + 4 <= nblocks; b += 4) {
            a0 += partial[(int64_t)b * P + k];
            a1 += partial[(int64_t)(b + 1) * P + k];
            a2 += partial[(int64_t)(b + 2) * P + k];
            a3 += partial[(int64_t)(b + 3) * P + k];
        }
        if (b < nblocks) a0 += partial[(int64_t)b * P + k];
        if (b + 1 < nblocks) a1 += partial[(int64_t)(b + 1) * P + k];
        if (b + 2 < nblocks) a2 += partial[(int64_t)(b + 2) * P + k];
        grad[k] = (a0 + a1) + (a2 + a3);
    }
    if (k == 0) {
        double e = 0.0;
        for (int b = 0; b < nblocks; ++b) e += loss_part[b];
        *loss = e * inv_3n;
    }
}

// Adam (bias-corrected first and second moments), fp32.
__global__ void __launch_bounds__(256) mlp_adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                       float* __restrict__ m, float* __restrict__ v, int P, float lr,
                                                       float b1, float b2, float eps, float c1, float c2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk * c1) / (sqrtf(vk * c2) + eps);
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

void launch_mlp_forward(const MlpArgs& a, bool train, hipStream_t s) {
    if (a.n <= 0) return;
    if (train)
        hipLaunchKernelGGL(mlp_forward_kernel<true>, dim3(grid_for(a.n, TS)), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(mlp_forward_kernel<false>, dim3(grid_for(a.n, TS)), dim3(256), 0, s, a);
    FDLB_HIP(hipGetLastError());
}

void launch_mlp_backward(const MlpArgs& a, hipStream_t s) {
    if (a.n <= 0) return;
    hipLaunchKernelGGL(mlp_backward_kernel, dim3(grid_for(a.n, TS)), dim3(256), 0, s, a);
    FDLB_HIP(hipGetLastError());
}

void launch_mlp_reduce(const float* partial, int nblocks, int P, float* grad, const double* loss_part, double inv_3n,
                       double* loss, hipStream_t s) {
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3(grid_for(P, 256)), dim3(256), 0, s, partial, nblocks, P, grad,
                       loss_part, inv_3n, loss);
    FDLB_HIP(hipGetLastError());
}

void launch_mlp_adam(float* p, const float* g, float* m, float* v, int P, float lr, float b1, float b2, float eps,
                     float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(mlp_adam_kernel, dim3(grid_for(P, 256)), dim3(256), 0, s, p, g, m, v, P, lr, b1, b2, eps,
                       c1, c2);
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
