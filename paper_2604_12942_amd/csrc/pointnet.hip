// Per-voxel point network of the model branch of the cascaded initialisation (Sec. III-B,
// Eq. 3): a shared MLP 3 -> 64 -> 64 -> 64 (ReLU) over each voxel's 32 input rows, max-pool, the
// 12 voxel-PCA features appended, 76 -> 64 (ReLU) -> 8 = (log-scales, quaternion, opacity logit).
//
// One 256-lane workgroup takes 8 voxels = 256 point rows.  The two 64 x 64 layers run on the
// matrix cores (v_mfma_f32_32x32x16_bf16, BF16 inputs, FP32 accumulate): each wave owns two
// 32-row tiles (two voxels) x both 32-column tiles.  The 3-wide first layer, the per-voxel
// 76- and 64-wide layers and the weight gradients run on the VALU.  BF16 rounding points
// (round to nearest even): weights and every GEMM input; bias, ReLU and accumulation in FP32.
//
// The backward (one training step's gradient) is persistent: each workgroup loops over voxel
// tiles, recomputes the forward in LDS, forms the loss gradient per voxel
// (KL(N(0, Sigma_pred) || N(0, Sigma_tgt)) + 0.1 |sigmoid(omega) - o_tgt|, mean over voxels with
// a target), back-propagates (max-pool to the argmax row, lowest row on ties) and keeps its
// weight-gradient partial sums in registers; a fixed-order reduction over workgroups follows.
#include "gsr_internal.h"

namespace gsr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kRows = 32, kWidth = 64, kFeat = 12, kOut = 8, kVox = 8;  // 8 voxels per workgroup
constexpr int kLd = 72;                                                   // padded LDS row (bf16)
// flat weight layout (floats): W1[3][64] b1 W2[64][64] b2 W3[64][64] b3 W4[76][64] b4 W5[64][8] b5
constexpr int oW1 = 0, oB1 = 192, oW2 = 256, oB2 = 4352, oW3 = 4416, oB3 = 8512, oW4 = 8576, oB4 = 13440,
              oW5 = 13504, oB5 = 14016, kNW = 14024;

__device__ __forceinline__ __bf16 tobf(float x) { return (__bf16)x; }
__device__ __forceinline__ float fbf(__bf16 x) { return (float)x; }

struct PnShared {
    __attribute__((aligned(16))) __bf16 w2t[kWidth][kLd];  // W2 transposed: [out][in]
    __attribute__((aligned(16))) __bf16 w3t[kWidth][kLd];
    __attribute__((aligned(16))) __bf16 h1[kVox * kRows][kLd];
    __attribute__((aligned(16))) __bf16 h2[kVox * kRows][kLd];
    __bf16 w4[kWidth + kFeat][kWidth];
    __bf16 w5[kWidth][kOut];
    __bf16 w1[3][kWidth];
    float b[kWidth * 4 + kOut];  // b1 b2 b3 b4 b5
    __attribute__((aligned(8))) __bf16 x[kVox * kRows][4];
    float g[kVox][kWidth];           // max-pooled layer-3 activations
    uint8_t arg[kVox][kWidth];       // argmax row
    __bf16 z[kVox][kWidth + kFeat];  // layer-4 input
    float a4[kVox][kWidth];
    __bf16 h4[kVox][kWidth];
    float y[kVox][kOut];
};

__device__ void load_weights(const float *__restrict__ W, PnShared &S) {
    const int t = threadIdx.x;
    for (int q = t; q < kWidth * kWidth; q += 256) {
        const int k = q / kWidth, n = q % kWidth;
        S.w2t[n][k] = tobf(W[oW2 + q]);
        S.w3t[n][k] = tobf(W[oW3 + q]);
    }
    for (int q = t; q < (kWidth + kFeat) * kWidth; q += 256) S.w4[q / kWidth][q % kWidth] = tobf(W[oW4 + q]);
    for (int q = t; q < kWidth * kOut; q += 256) S.w5[q / kOut][q % kOut] = tobf(W[oW5 + q]);
    if (t < 3 * kWidth) S.w1[t / kWidth][t % kWidth] = tobf(W[oW1 + t]);
    S.b[t] = t < 64 ? W[oB1 + t] : (t < 128 ? W[oB2 + t - 64] : (t < 192 ? W[oB3 + t - 128] : W[oB4 + t - 192]));
    if (t < kOut) S.b[256 + t] = W[oB5 + t];
}

// Input rows of the tile: voxel v0 + (t / 32), row t % 32 = fitting point (t % 32) mod n_sel.
__device__ void load_inputs(const float *__restrict__ pts, int64_t n, const gsr_voxels &V, uint32_t v0, uint32_t nv,
                            PnShared &S) {
    const int t = threadIdx.x;
    const uint32_t v = v0 + (t >> 5);
    float x[3] = {0.f, 0.f, 0.f};
    if (v < nv) {
        const uint32_t cnt = V.count[v];
        const uint32_t m = cnt < (uint32_t)kRows ? cnt : (uint32_t)kRows;
        const uint32_t p = V.point_order[V.start[v] + (uint32_t)(t & 31) % m];
        for (int c = 0; c < 3; c++) x[c] = (pts[c * n + p] - V.mu[c * n + v]) / 0.5f;
    }
    for (int c = 0; c < 3; c++) S.x[t][c] = tobf(x[c]);
    S.x[t][3] = tobf(0.f);
}

// layer 1 (3 -> 64, VALU): thread t computes row t
__device__ void layer1(PnShared &S) {
    const int t = threadIdx.x;
    const float x0 = fbf(S.x[t][0]), x1 = fbf(S.x[t][1]), x2 = fbf(S.x[t][2]);
    for (int j = 0; j < kWidth; j++) {
        float a = S.b[j];
        a = __builtin_fmaf(x0, fbf(S.w1[0][j]), a);
        a = __builtin_fmaf(x1, fbf(S.w1[1][j]), a);
        a = __builtin_fmaf(x2, fbf(S.w1[2][j]), a);
        S.h1[t][j] = tobf(fmaxf(a, 0.f));
    }
}

// [256 x 64] x [64 x 64] on the matrix cores: A rows from LDS (row-major, stride kLd), B given
// transposed ([out][in], stride kLd).  Wave w produces row tiles 2w, 2w+1 and both column tiles:
// acc[2 * rt + ct] holds rows 32 (2w + rt) + 8 (r / 4) + 4 (lane / 32) + r % 4, column
// 32 ct + lane % 32 for r = 0..15.
__device__ __forceinline__ void gemm64(const __bf16 (*A)[kLd], const __bf16 (*Bt)[kLd], f32x16 acc[4]) {
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    for (int q = 0; q < 4; q++) acc[q] = f32x16{};
    for (int kb = 0; kb < 4; kb++) {
        const int k0 = 16 * kb + 8 * half;
        bf16x8 a[2], b[2];
        for (int rt = 0; rt < 2; rt++) a[rt] = *reinterpret_cast<const bf16x8 *>(&A[32 * (2 * w + rt) + l32][k0]);
        for (int ct = 0; ct < 2; ct++) b[ct] = *reinterpret_cast<const bf16x8 *>(&Bt[32 * ct + l32][k0]);
        for (int rt = 0; rt < 2; rt++)
            for (int ct = 0; ct < 2; ct++)
                acc[2 * rt + ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[rt], b[ct], acc[2 * rt + ct], 0, 0, 0);
    }
}

__device__ __forceinline__ int acc_row(int rt, int r) {
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    return 32 * (2 * w + rt) + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

// layer 2: h2 = bf16(relu(h1 W2 + b2))
__device__ void layer2(PnShared &S) {
    f32x16 acc[4];
    gemm64(S.h1, S.w2t, acc);
    const int lane = __lane_id();
    for (int rt = 0; rt < 2; rt++)
        for (int ct = 0; ct < 2; ct++) {
            const int col = 32 * ct + (lane & 31);
            const float bb = S.b[64 + col];
            for (int r = 0; r < 16; r++) S.h2[acc_row(rt, r)][col] = tobf(fmaxf(acc[2 * rt + ct][r] + bb, 0.f));
        }
}

// layer 3 and the max-pool over each voxel's 32 rows (first maximum = lowest row on ties)
__device__ void layer3_pool(PnShared &S) {
    f32x16 acc[4];
    gemm64(S.h2, S.w3t, acc);
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    for (int rt = 0; rt < 2; rt++)
        for (int ct = 0; ct < 2; ct++) {
            const int col = 32 * ct + (lane & 31);
            const float bb = S.b[128 + col];
            float best = -1.f;
            int brow = 0;
            for (int r = 0; r < 16; r++) {
                const float h = fmaxf(acc[2 * rt + ct][r] + bb, 0.f);
                const int row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);  // row within the voxel
                if (h > best || (h == best && row < brow)) {
                    best = h;
                    brow = row;
                }
            }
            const float ob = __shfl_xor(best, 32);
            const int orow = __shfl_xor(brow, 32);
            if (ob > best || (ob == best && orow < brow)) {
                best = ob;
                brow = orow;
            }
            if (lane < 32) {
                const int v = 2 * w + rt;
                S.g[v][col] = best;
                S.arg[v][col] = (uint8_t)brow;
            }
        }
}

// voxel features (12): log(max(lambda, floor) / 0.25) ascending, then v_min, v_mid, v_max
__device__ void head(const gsr_voxels &V, int64_t n, uint32_t v0, uint32_t nv, PnShared &S) {
    const int t = threadIdx.x;
    for (int q = t; q < kVox * (kWidth + kFeat); q += 256) {
        const int v = q / (kWidth + kFeat), k = q % (kWidth + kFeat);
        const uint32_t vg = v0 + v;
        float val = 0.f;
        if (k < kWidth) {
            val = S.g[v][k];
        } else if (vg < nv) {
            const int f = k - kWidth;
            if (f < 3) {
                val = logf(fmaxf(V.evals[f * n + vg], 0.005f * 0.005f) / 0.25f);
            } else {
                const int col = 2 - (f - 3) / 3, row = (f - 3) % 3;  // R_pca columns: v_max, v_mid, v_min
                val = V.R[(row * 3 + col) * n + vg];
            }
        }
        S.z[v][k] = tobf(val);
    }
    __syncthreads();
    for (int q = t; q < kVox * kWidth; q += 256) {
        const int v = q / kWidth, j = q % kWidth;
        float a = S.b[192 + j];
        for (int k = 0; k < kWidth + kFeat; k++) a = __builtin_fmaf(fbf(S.z[v][k]), fbf(S.w4[k][j]), a);
        S.a4[v][j] = a;
        S.h4[v][j] = tobf(fmaxf(a, 0.f));
    }
    __syncthreads();
    if (t < kVox * kOut) {
        const int v = t / kOut, j = t % kOut;
        float a = S.b[256 + j];
        for (int k = 0; k < kWidth; k++) a = __builtin_fmaf(fbf(S.h4[v][k]), fbf(S.w5[k][j]), a);
        S.y[v][j] = a;
    }
    __syncthreads();
}

__device__ void forward_tile(const float *pts, int64_t n, const gsr_voxels &V, uint32_t v0, uint32_t nv,
                             PnShared &S) {
    load_inputs(pts, n, V, v0, nv, S);
    __syncthreads();
    layer1(S);
    __syncthreads();
    layer2(S);
    __syncthreads();
    layer3_pool(S);
    __syncthreads();
    head(V, n, v0, nv, S);
}

// ---- forward (inference) ------------------------------------------------------------------------
// Persistent, wave-independent: each wave takes an equal contiguous range of voxels (its share of
// the whole batch, so that no wave runs a group more than another) in groups of 32.  Per voxel the
// wave runs the
// three shared layers on the matrix cores with the activations kept in registers:
//   layers 1 and 2 transposed, out^T = W^T h^T (M = 64 output features in two row tiles, N = the
//   voxel's 32 rows), so the accumulators hold, per lane, one row and 16 features of each tile;
//   those 32 values, bias + ReLU + BF16, are directly the next layer's K-operand once K is taken in
//   the order phi below (the weights are loaded in the same order; the contraction does not care);
//   layer 3 the other way round, out = h2 W3 (M = the 32 rows), so that each lane holds one output
//   column over 16 rows and the max-pool is 15 maxima and one cross-half exchange.
// Biases enter as the accumulators' initial value.  The pooled features of the group's 32 voxels
// and their 12 PCA features gather in the wave's LDS block; the head 76 -> 64 -> 8 then runs
// transposed on the matrix cores for all 32 voxels at once (N = 32 voxels, the output's 8 rows
// padded to 32).  Rounding points as everywhere: BF16 weights and layer inputs, FP32 bias, ReLU
// and accumulation.
//
// K order of a 64-wide chained operand: position (kb, half, j) of k-block kb (16 wide), lane half
// and element j (0..7) holds feature phi = 32 (kb / 2) + 16 (kb % 2) + 8 (j / 4) + 4 half + j % 4,
// which is where the 32 x 32 accumulator layout keeps it (register 8 (kb % 2) + j of tile kb / 2).
__device__ __forceinline__ int phi_k(int kb, int half, int j) {
    return 32 * (kb >> 1) + 16 * (kb & 1) + 8 * (j >> 2) + 4 * half + (j & 3);
}

constexpr int kGrp = 32;   // voxels per wave group (the head's N)
constexpr int kStage = 16; // voxels whose input rows are staged at once
constexpr int kZld = 80;   // LDS row of the head input (76 used), bf16

struct PnFwdShared {
    bf16x8 a4[2][5][64];  // layer-4 A fragments (W4^T, K padded to 80)
    bf16x8 a5[4][64];     // layer-5 A fragments (W5^T, M padded to 32, K in phi order)
    float b1[kWidth], b2[kWidth], b4[kWidth], b5[kOut];
    __attribute__((aligned(16))) __bf16 z[4][kGrp][kZld];            // per wave: head inputs
    __attribute__((aligned(8))) __bf16 xs[4][kStage][kRows][4];      // per wave: staged input rows
};

__device__ __forceinline__ f32x16 bias_tile(const float *b, int rt, int half) {
    // accumulator register r of row tile rt holds feature 32 rt + 8 (r / 4) + 4 half + r % 4
    f32x16 c;
    const float4 *p = reinterpret_cast<const float4 *>(b + 32 * rt + 4 * half);
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const float4 v = p[2 * q];
        c[4 * q] = v.x;
        c[4 * q + 1] = v.y;
        c[4 * q + 2] = v.z;
        c[4 * q + 3] = v.w;
    }
    return c;
}

// bias already in the accumulators: h = bf16(relu(acc)), as the four k-blocks of the next layer.
// The ReLU is taken after the rounding, on the BF16 bit patterns as signed 16-bit integers
// (negative values and -0 have the sign bit set): rounding keeps the sign, so this equals
// rounding the ReLU.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void relu_operands(const f32x16 d[2], bf16x8 h[4]) {
#pragma unroll
    for (int kb = 0; kb < 4; kb++) {
        u32x4 u;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int r = 8 * (kb & 1) + 2 * i;
            const f32x2 f = {d[kb >> 1][r], d[kb >> 1][r + 1]};
            const bf16x2 b = __builtin_convertvector(f, bf16x2);  // round to nearest even
            const i16x2 m = __builtin_elementwise_max(__builtin_bit_cast(i16x2, b), i16x2{});
            u[i] = __builtin_bit_cast(uint32_t, m);
        }
        h[kb] = __builtin_bit_cast(bf16x8, u);
    }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_pn_fwd(const float *__restrict__ pts, int64_t n, gsr_voxels V,
                                                const float *__restrict__ W, float *__restrict__ y) {
    __shared__ PnFwdShared S;
    const uint32_t nv = *V.n_voxels;
    const int t = threadIdx.x, lane = __lane_id(), w = t >> 6, half = lane >> 5, l32 = lane & 31;
    const uint32_t nwaves = gridDim.x * 4, gw = blockIdx.x * 4 + w;
    const uint32_t vbeg = (uint32_t)((uint64_t)gw * nv / nwaves), vend = (uint32_t)((uint64_t)(gw + 1) * nv / nwaves);
    // head fragments and biases
    for (int q = t; q < 2 * 5 * 64; q += 256) {
        const int rt = q / 320, kb = (q / 64) % 5, ln = q % 64, h = ln >> 5, o = 32 * rt + (ln & 31);
        bf16x8 f;
        for (int j = 0; j < 8; j++) {
            const int k = 16 * kb + 8 * h + j;
            f[j] = tobf(k < kWidth + kFeat ? W[oW4 + k * kWidth + o] : 0.f);
        }
        S.a4[rt][kb][ln] = f;
    }
    for (int q = t; q < 4 * 64; q += 256) {
        const int kb = q / 64, ln = q % 64, h = ln >> 5, o = ln & 31;
        bf16x8 f;
        for (int j = 0; j < 8; j++) f[j] = tobf(o < kOut ? W[oW5 + phi_k(kb, h, j) * kOut + o] : 0.f);
        S.a5[kb][ln] = f;
    }
    if (t < kWidth) {
        S.b1[t] = W[oB1 + t];
        S.b2[t] = W[oB2 + t];
        S.b4[t] = W[oB4 + t];
    }
    if (t < kOut) S.b5[t] = W[oB5 + t];
    for (int q = lane; q < kGrp * (kZld - kWidth - kFeat); q += 64)
        S.z[w][q / (kZld - kWidth - kFeat)][kWidth + kFeat + q % (kZld - kWidth - kFeat)] = tobf(0.f);
    // shared-layer fragments in registers: W1^T (K = 3 padded to 16), W2^T and W3 in phi order
    bf16x8 a1[2], a2[2][4], b3[2][4];
    for (int rt = 0; rt < 2; rt++) {
        for (int j = 0; j < 8; j++) a1[rt][j] = tobf(half == 0 && j < 3 ? W[oW1 + j * kWidth + 32 * rt + l32] : 0.f);
        for (int kb = 0; kb < 4; kb++)
            for (int j = 0; j < 8; j++) {
                const int k = phi_k(kb, half, j);
                a2[rt][kb][j] = tobf(W[oW2 + k * kWidth + 32 * rt + l32]);
                b3[rt][kb][j] = tobf(W[oW3 + k * kWidth + 32 * rt + l32]);
            }
    }
    const float bb3[2] = {W[oB3 + l32], W[oB3 + 32 + l32]};
    float *const y4 = y + 4 * n;  // outputs 4..7
    __syncthreads();
    __bf16(*Z)[kZld] = S.z[w];
    for (uint32_t vg = vbeg; vg < vend; vg += kGrp) {
        const int ng = (int)min((uint32_t)kGrp, vend - vg);  // voxels of this group
        for (int s0 = 0; s0 < ng; s0 += kStage) {
            // stage the input rows of kStage voxels: lane -> voxel lane / 4, rows 8 (lane % 4) ..
            {
                const int sv = lane >> 2, r0 = 8 * (lane & 3);
                const uint32_t v = vg + s0 + sv;
                float x[8][3];
                if (s0 + sv < ng) {
                    const uint32_t cnt = V.count[v], st = V.start[v];
                    const uint32_t m = cnt < (uint32_t)kRows ? cnt : (uint32_t)kRows;
                    const float m0 = V.mu[v], m1 = V.mu[n + v], m2 = V.mu[2 * n + v];
                    uint32_t p[8];
#pragma unroll
                    for (int i = 0; i < 8; i++) p[i] = V.point_order[st + (uint32_t)(r0 + i) % m];
#pragma unroll
                    for (int i = 0; i < 8; i++) {
                        x[i][0] = (pts[p[i]] - m0) / 0.5f;
                        x[i][1] = (pts[n + p[i]] - m1) / 0.5f;
                        x[i][2] = (pts[2 * n + p[i]] - m2) / 0.5f;
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < 8; i++) x[i][0] = x[i][1] = x[i][2] = 0.f;
                }
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    __bf16 *d = S.xs[w][sv][r0 + i];
                    d[0] = tobf(x[i][0]);
                    d[1] = tobf(x[i][1]);
                    d[2] = tobf(x[i][2]);
                    d[3] = tobf(0.f);
                }
            }
            __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
            __builtin_amdgcn_wave_barrier();
            const int s1 = min(s0 + kStage, ng);
            for (int s = s0; s < s1; s++) {
                // layer 1: B = the voxel's rows (K = 3 of 16, first half-wave)
                bf16x8 bx = bf16x8{};
                if (half == 0) {
                    // the staged row: three BF16 coordinates and a zero
                    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
                    const bf16x4 xr = *reinterpret_cast<const bf16x4 *>(S.xs[w][s - s0][l32]);
                    bx[0] = xr[0];
                    bx[1] = xr[1];
                    bx[2] = xr[2];
                }
                f32x16 d[2];
#pragma unroll
                for (int rt = 0; rt < 2; rt++)
                    d[rt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1[rt], bx, bias_tile(S.b1, rt, half), 0, 0, 0);
                bf16x8 h[4];
                relu_operands(d, h);
                // layer 2
#pragma unroll
                for (int rt = 0; rt < 2; rt++) {
                    f32x16 acc = bias_tile(S.b2, rt, half);
#pragma unroll
                    for (int kb = 0; kb < 4; kb++)
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2[rt][kb], h[kb], acc, 0, 0, 0);
                    d[rt] = acc;
                }
                relu_operands(d, h);
                // layer 3 (rows = the voxel's points) and the max-pool: relu(max_r acc + b) equals
                // max_r relu(acc + b), rounding included (both maps are monotone)
#pragma unroll
                for (int ct = 0; ct < 2; ct++) {
                    f32x16 acc = f32x16{};
#pragma unroll
                    for (int kb = 0; kb < 4; kb++)
                        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(h[kb], b3[ct][kb], acc, 0, 0, 0);
                    float best = acc[0];
#pragma unroll
                    for (int r = 1; r < 16; r++) best = fmaxf(best, acc[r]);
                    best = fmaxf(best, __shfl_xor(best, 32));
                    if (half == 0) Z[s][32 * ct + l32] = tobf(fmaxf(best + bb3[ct], 0.f));
                }
            }
            __builtin_amdgcn_wave_barrier();  // the next stage overwrites the rows just read
        }
        // the 12 voxel features: log(max(lambda, floor) / 0.25) ascending, then v_min, v_mid, v_max
        if (half == 0) {
            const uint32_t v = vg + l32;
            float f[kFeat];
            for (int q = 0; q < kFeat; q++) f[q] = 0.f;
            if (l32 < ng) {
                for (int q = 0; q < 3; q++) f[q] = logf(fmaxf(V.evals[q * n + v], 0.005f * 0.005f) / 0.25f);
                for (int q = 3; q < kFeat; q++) {
                    const int col = 2 - (q - 3) / 3, row = (q - 3) % 3;  // R_pca columns: v_max, v_mid, v_min
                    f[q] = V.R[(row * 3 + col) * n + v];
                }
            }
            for (int q = 0; q < kFeat; q++) Z[l32][kWidth + q] = tobf(f[q]);
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        // layer 4 (76 -> 64), transposed over the 32 voxels
        f32x16 d[2];
#pragma unroll
        for (int rt = 0; rt < 2; rt++) {
            f32x16 acc = bias_tile(S.b4, rt, half);
#pragma unroll
            for (int kb = 0; kb < 5; kb++) {
                const bf16x8 bz = *reinterpret_cast<const bf16x8 *>(&Z[l32][16 * kb + 8 * half]);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(S.a4[rt][kb][lane], bz, acc, 0, 0, 0);
            }
            d[rt] = acc;
        }
        bf16x8 h[4];
        relu_operands(d, h);
        // layer 5 (64 -> 8; rows 8..31 are padding): lane holds outputs 4 half .. 4 half + 3 of voxel l32
        f32x16 acc = f32x16{};
#pragma unroll
        for (int r = 0; r < 4; r++) acc[r] = S.b5[4 * half + r];
#pragma unroll
        for (int kb = 0; kb < 4; kb++) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(S.a5[kb][lane], h[kb], acc, 0, 0, 0);
        const uint32_t v = vg + l32;
        // (one store path per half-wave, each from a uniform base)
        if (l32 < ng && half == 0) {
#pragma unroll
            for (int r = 0; r < 4; r++) y[(int64_t)r * n + v] = acc[r];
        }
        if (l32 < ng && half == 1) {
#pragma unroll
            for (int r = 0; r < 4; r++) y4[(int64_t)r * n + v] = acc[r];
        }
        __builtin_amdgcn_wave_barrier();  // the next group overwrites the head inputs
    }
}

// ---- backward ----------------------------------------------------------------------------------

// B fragment of a backward GEMM straight from the float32 weights in their natural [in][out]
// layout (row n of the transposed operand = 8 consecutive floats of row n)
__device__ __forceinline__ bf16x8 wfrag(const float *__restrict__ Wn, int row, int k0) {
    const float4 a = *reinterpret_cast<const float4 *>(Wn + row * kWidth + k0);
    const float4 b = *reinterpret_cast<const float4 *>(Wn + row * kWidth + k0 + 4);
    bf16x8 r;
    r[0] = tobf(a.x), r[1] = tobf(a.y), r[2] = tobf(a.z), r[3] = tobf(a.w);
    r[4] = tobf(b.x), r[5] = tobf(b.y), r[6] = tobf(b.z), r[7] = tobf(b.w);
    return r;
}

// out[row][k] = sum_c dA[row][c] W[k][c]  (the data gradient through a 64 x 64 layer)
__device__ __forceinline__ void gemm64_bwd(const __bf16 (*A)[kLd], const float *__restrict__ Wn, f32x16 acc[4]) {
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    for (int q = 0; q < 4; q++) acc[q] = f32x16{};
    for (int kb = 0; kb < 4; kb++) {
        const int k0 = 16 * kb + 8 * half;
        bf16x8 a[2], b[2];
        for (int rt = 0; rt < 2; rt++) a[rt] = *reinterpret_cast<const bf16x8 *>(&A[32 * (2 * w + rt) + l32][k0]);
        for (int ct = 0; ct < 2; ct++) b[ct] = wfrag(Wn, 32 * ct + l32, k0);
        for (int rt = 0; rt < 2; rt++)
            for (int ct = 0; ct < 2; ct++)
                acc[2 * rt + ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[rt], b[ct], acc[2 * rt + ct], 0, 0, 0);
    }
}

// G[4 k][4 c] += sum over the 256 rows of H[row][k] dA[row][c]: thread t owns the 4 x 4 block
// (k = 4 (t / 16) .., c = 4 (t % 16) ..)
__device__ __forceinline__ void wgrad64(const __bf16 (*H)[kLd], const __bf16 (*dA)[kLd], float G[16]) {
    const int kb = 4 * (threadIdx.x >> 4), cb = 4 * (threadIdx.x & 15);
    for (int row = 0; row < kVox * kRows; row++) {
        float h[4], d[4];
        for (int i = 0; i < 4; i++) {
            h[i] = fbf(H[row][kb + i]);
            d[i] = fbf(dA[row][cb + i]);
        }
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) G[4 * i + j] = __builtin_fmaf(h[i], d[j], G[4 * i + j]);
    }
}

struct PnBwdShared {
    __attribute__((aligned(16))) __bf16 dA[kVox * kRows][kLd];
    float dy[kVox][kOut];
    float da4[kVox][kWidth];
    float dg[kVox][kWidth];
    float gb[kWidth * 4 + kOut];  // bias gradients (b1 b2 b3 b4 b5), kept across tiles
};

// dL/dy of one voxel: KL(N(0, Sp) || N(0, St)) + 0.1 |sigmoid(omega) - o_t|, scaled by inv_count
__device__ void loss_grad(const float y[8], const double St[6], double ot, double scale, float dy[8], double *lval) {
    double s[3] = {y[0], y[1], y[2]}, q[4] = {y[3], y[4], y[5], y[6]}, om = y[7];
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double w = q[0] / qn, x = q[1] / qn, yy = q[2] / qn, z = q[3] / qn;
    const double R[9] = {1 - 2 * (yy * yy + z * z), 2 * (x * yy - w * z), 2 * (x * z + w * yy),
                         2 * (x * yy + w * z), 1 - 2 * (x * x + z * z), 2 * (yy * z - w * x),
                         2 * (x * z - w * yy), 2 * (yy * z + w * x), 1 - 2 * (x * x + yy * yy)};
    // A = St^-1 (symmetric; St = [[a, b, c], [b, d, e], [c, e, f]])
    const double a = St[0], b = St[1], c = St[2], d = St[3], e = St[4], f = St[5];
    const double c00 = d * f - e * e, c01 = c * e - b * f, c02 = b * e - c * d;
    const double c11 = a * f - c * c, c12 = b * c - a * e, c22 = a * d - b * b;
    const double det = a * c00 + b * c01 + c * c02;
    const double A[9] = {c00 / det, c01 / det, c02 / det, c01 / det, c11 / det, c12 / det, c02 / det, c12 / det,
                         c22 / det};
    double AR[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) AR[i * 3 + j] = A[i * 3] * R[j] + A[i * 3 + 1] * R[3 + j] + A[i * 3 + 2] * R[6 + j];
    double ds[3], dR[9], tr = 0.0;
    for (int j = 0; j < 3; j++) {
        const double e2 = exp(2 * s[j]);
        const double rar = R[j] * AR[j] + R[3 + j] * AR[3 + j] + R[6 + j] * AR[6 + j];
        tr += e2 * rar;
        ds[j] = e2 * rar - 1.0;
        for (int i = 0; i < 3; i++) dR[i * 3 + j] = e2 * AR[i * 3 + j];
    }
    // d R / d (w, x, y, z) of the unit quaternion, contracted with dR
    const double dqh[4] = {
        dR[1] * (-2 * z) + dR[2] * (2 * yy) + dR[3] * (2 * z) + dR[5] * (-2 * x) + dR[6] * (-2 * yy) + dR[7] * (2 * x),
        dR[1] * (2 * yy) + dR[2] * (2 * z) + dR[3] * (2 * yy) + dR[4] * (-4 * x) + dR[5] * (-2 * w) + dR[6] * (2 * z) +
            dR[7] * (2 * w) + dR[8] * (-4 * x),
        dR[0] * (-4 * yy) + dR[1] * (2 * x) + dR[2] * (2 * w) + dR[3] * (2 * x) + dR[5] * (2 * z) + dR[6] * (-2 * w) +
            dR[7] * (2 * z) + dR[8] * (-4 * yy),
        dR[0] * (-4 * z) + dR[1] * (-2 * w) + dR[2] * (2 * x) + dR[3] * (2 * w) + dR[4] * (-4 * z) + dR[5] * (2 * yy) +
            dR[6] * (2 * x) + dR[7] * (2 * yy)};
    const double qh[4] = {w, x, yy, z};
    const double pr = qh[0] * dqh[0] + qh[1] * dqh[1] + qh[2] * dqh[2] + qh[3] * dqh[3];
    const double sg = 1.0 / (1.0 + exp(-om));
    const double sgn = (sg > ot) ? 1.0 : ((sg < ot) ? -1.0 : 0.0);
    for (int j = 0; j < 3; j++) dy[j] = (float)(scale * ds[j]);
    for (int k = 0; k < 4; k++) dy[3 + k] = (float)(scale * (dqh[k] - qh[k] * pr) / qn);
    dy[7] = (float)(scale * 0.1 * sgn * sg * (1 - sg));
    *lval = scale * (0.5 * (tr - 3.0 + log(det) - 2.0 * (s[0] + s[1] + s[2])) + 0.1 * fabs(sg - ot));
}

__global__ __launch_bounds__(256) void k_pn_bwd(const float *__restrict__ pts, int64_t n, gsr_voxels V,
                                                const float *__restrict__ W, const float *__restrict__ cov_t,
                                                const float *__restrict__ o_t, const uint8_t *__restrict__ tmask,
                                                float inv_count, float *__restrict__ part, double *__restrict__ loss) {
    __shared__ PnShared S;
    __shared__ PnBwdShared B;
    const uint32_t nv = *V.n_voxels;
    const int t = threadIdx.x, lane = __lane_id();
    load_weights(W, S);
    for (int q = t; q < kWidth * 4 + kOut; q += 256) B.gb[q] = 0.f;
    float gW2[16], gW3[16], gW4[19], gW5[2], gW1 = 0.f;
    for (int i = 0; i < 16; i++) gW2[i] = gW3[i] = 0.f;
    for (int i = 0; i < 19; i++) gW4[i] = 0.f;
    gW5[0] = gW5[1] = 0.f;
    __syncthreads();
    const uint32_t ntiles = (nv + kVox - 1) / kVox;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint32_t v0 = tile * kVox;
        forward_tile(pts, n, V, v0, nv, S);
        // loss gradient, one thread per voxel
        if (t < kVox) {
            const uint32_t v = v0 + t;
            float dy[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (v < nv && (!tmask || tmask[v])) {
                double St[6];
                for (int k = 0; k < 6; k++) St[k] = cov_t[k * n + v];
                double lv;
                loss_grad(S.y[t], St, o_t[v], inv_count, dy, &lv);
                atomicAdd(loss, lv);
            }
            for (int k = 0; k < 8; k++) B.dy[t][k] = dy[k];
        }
        __syncthreads();
        // head backward: layer 5 (64 -> 8) and layer 4 (76 -> 64)
        for (int m = 0; m < 2; m++) {
            const int q = t + 256 * m, k = q / kOut, j = q % kOut;
            for (int v = 0; v < kVox; v++) gW5[m] = __builtin_fmaf(fbf(S.h4[v][k]), fbf(tobf(B.dy[v][j])), gW5[m]);
        }
        if (t < kOut)
            for (int v = 0; v < kVox; v++) B.gb[256 + t] += B.dy[v][t];
        for (int q = t; q < kVox * kWidth; q += 256) {
            const int v = q / kWidth, k = q % kWidth;
            float dh = 0.f;
            for (int j = 0; j < kOut; j++) dh = __builtin_fmaf(fbf(tobf(B.dy[v][j])), fbf(S.w5[k][j]), dh);
            B.da4[v][k] = S.a4[v][k] > 0.f ? dh : 0.f;
        }
        __syncthreads();
        for (int m = 0; m < 19; m++) {
            const int q = t + 256 * m, k = q / kWidth, j = q % kWidth;
            for (int v = 0; v < kVox; v++) gW4[m] = __builtin_fmaf(fbf(S.z[v][k]), fbf(tobf(B.da4[v][j])), gW4[m]);
        }
        if (t < kWidth)
            for (int v = 0; v < kVox; v++) B.gb[192 + t] += B.da4[v][t];
        for (int q = t; q < kVox * kWidth; q += 256) {
            const int v = q / kWidth, c = q % kWidth;
            float dz = 0.f;
            for (int j = 0; j < kWidth; j++) dz = __builtin_fmaf(fbf(tobf(B.da4[v][j])), fbf(S.w4[c][j]), dz);
            B.dg[v][c] = S.g[v][c] > 0.f ? dz : 0.f;  // through the ReLU at the pooled maximum
        }
        __syncthreads();
        // max-pool backward: the gradient goes to the argmax row only
        for (int q = t; q < kVox * kRows * kWidth; q += 256) {
            const int row = q / kWidth, c = q % kWidth, v = row / kRows;
            B.dA[row][c] = tobf(S.arg[v][c] == (row % kRows) ? B.dg[v][c] : 0.f);
        }
        if (t < kWidth)
            for (int v = 0; v < kVox; v++) B.gb[128 + t] += B.dg[v][t];
        __syncthreads();
        wgrad64(S.h2, B.dA, gW3);
        __syncthreads();
        // layer 3 data gradient on the matrix cores, then through layer 2's ReLU
        {
            f32x16 acc[4];
            gemm64_bwd(B.dA, W + oW3, acc);
            for (int rt = 0; rt < 2; rt++)
                for (int ct = 0; ct < 2; ct++) {
                    const int col = 32 * ct + (lane & 31);
                    float bsum = 0.f;
                    for (int r = 0; r < 16; r++) {
                        const int row = acc_row(rt, r);
                        const float da = fbf(S.h2[row][col]) > 0.f ? acc[2 * rt + ct][r] : 0.f;
                        bsum += da;
                        B.dA[row][col] = tobf(da);
                    }
                    atomicAdd(&B.gb[64 + col], bsum);
                }
        }
        __syncthreads();
        wgrad64(S.h1, B.dA, gW2);
        __syncthreads();
        {
            f32x16 acc[4];
            gemm64_bwd(B.dA, W + oW2, acc);
            for (int rt = 0; rt < 2; rt++)
                for (int ct = 0; ct < 2; ct++) {
                    const int col = 32 * ct + (lane & 31);
                    float bsum = 0.f;
                    for (int r = 0; r < 16; r++) {
                        const int row = acc_row(rt, r);
                        const float da = fbf(S.h1[row][col]) > 0.f ? acc[2 * rt + ct][r] : 0.f;
                        bsum += da;
                        B.dA[row][col] = tobf(da);
                    }
                    atomicAdd(&B.gb[col], bsum);
                }
        }
        __syncthreads();
        if (t < 3 * kWidth) {
            const int k = t / kWidth, c = t % kWidth;
            for (int row = 0; row < kVox * kRows; row++) gW1 = __builtin_fmaf(fbf(S.x[row][k]), fbf(B.dA[row][c]), gW1);
        }
        __syncthreads();
    }
    // this workgroup's partial gradient, in the flat weight layout
    float *P = part + (int64_t)blockIdx.x * kNW;
    {
        const int kb = 4 * (t >> 4), cb = 4 * (t & 15);
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) {
                P[oW2 + (kb + i) * kWidth + cb + j] = gW2[4 * i + j];
                P[oW3 + (kb + i) * kWidth + cb + j] = gW3[4 * i + j];
            }
    }
    for (int m = 0; m < 19; m++) P[oW4 + t + 256 * m] = gW4[m];
    for (int m = 0; m < 2; m++) P[oW5 + t + 256 * m] = gW5[m];
    if (t < 3 * kWidth) P[oW1 + t] = gW1;
    P[t < 64 ? oB1 + t : (t < 128 ? oB2 + t - 64 : (t < 192 ? oB3 + t - 128 : oB4 + t - 192))] = B.gb[t];
    if (t < kOut) P[oB5 + t] = B.gb[256 + t];
}

// fixed-order sum of the workgroups' partial gradients
__global__ void k_pn_reduce(const float *__restrict__ part, int nb, float *__restrict__ grad) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < kNW; q += gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int b = 0; b < nb; b++) s += part[(int64_t)b * kNW + q];
        grad[q] = s;
    }
}

}  // namespace gsr

using namespace gsr;

extern "C" int gsr_pointnet_weight_count(void) { return kNW; }

extern "C" gsr_status gsr_pointnet_fwd_launch(const float *pts, int64_t n, const gsr_voxels *vox, const float *W,
                                              float *y, hipStream_t st) {
    if (n == 0) return GSR_OK;
    // persistent: three workgroups per compute unit (the LDS allows three), each wave loops over
    // groups of 32 voxels
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    const int64_t blocks = ceil_div(ceil_div(n, kGrp), 4);
    const int nb = (int)(blocks < 3 * cus ? blocks : 3 * cus);
    k_pn_fwd<<<nb, 256, 0, st>>>(pts, n, *vox, W, y);
    return last_launch();
}

extern "C" size_t gsr_pointnet_bwd_ws_bytes(int blocks) { return (size_t)blocks * kNW * sizeof(float) + 256; }

extern "C" gsr_status gsr_pointnet_bwd_launch(const float *pts, int64_t n, const gsr_voxels *vox, const float *W,
                                              const float *cov_t, const float *o_t, const uint8_t *tmask,
                                              float inv_count, int blocks, float *grad, double *loss, void *ws,
                                              hipStream_t st) {
    float *part = static_cast<float *>(ws);
    k_pn_bwd<<<blocks, 256, 0, st>>>(pts, n, *vox, W, cov_t, o_t, tmask, inv_count, part, loss);
    k_pn_reduce<<<(kNW + 255) / 256, 256, 0, st>>>(part, blocks, grad);
    return last_launch();
}

