// Learned warm start for the PageRank power iteration: degree features, a
// 3 -> 64 -> 64 -> 1 GELU network with BF16 weights and FP32 accumulation
// (forward, backward and Adam, all on the GPU), and the start vector
// r0 = softmax(y) (the network predicts log(V * r)). The plain iteration from
// this vector still decides convergence.
//
// Parameter vector (4481 values): W1[64][3], b1[64], W2[64][64] (row j =
// output j), b2[64], w3[64], b3.
#include <math.h>

#include "common.h"

namespace cagra {

cagra_status launch_gather(const cagra_segments *seg, int32_t op, int32_t value_type, const void *values,
                           void *partial, hipStream_t st);
cagra_status launch_merge(const cagra_segments *seg, int32_t op, const void *partial, void *out, hipStream_t st);
cagra_status launch_merge_sum_fixed24(const cagra_segments *seg, const float *partial, float *out, hipStream_t st);
cagra_status launch_softmax(const float *y, int32_t V, float *r0, double *scal, void *ws, hipStream_t st);

constexpr int kH = 64;
constexpr int kOffW1 = 0, kOffB1 = 192, kOffW2 = 256, kOffB2 = 4352, kOffW3 = 4416, kOffB3 = 4480;
constexpr int kNParam = CAGRA_MLP_PARAMS;
static_assert(kNParam == 4481, "parameter layout");

// erf(x) by Abramowitz & Stegun, Handbook of Mathematical Functions, formula
// 7.1.26 (|error| <= 1.5e-7): branch-free, one reciprocal and one exp2.
__device__ __forceinline__ float erf_as(float x) {
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
    float p = fmaf(1.061405429f, t, -1.453152027f);
    p = fmaf(p, t, 1.421413741f);
    p = fmaf(p, t, -0.284496736f);
    p = fmaf(p, t, 0.254829592f);
    p *= t;
    const float e = __builtin_amdgcn_exp2f(-ax * ax * 1.4426950408889634f);
    return copysignf(fmaf(-p, e, 1.0f), x);
}
// GELU(x) = x * Phi(x) (Hendrycks & Gimpel 2016) and its derivative Phi(x) + x * phi(x).
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erf_as(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
    return 0.5f * (1.0f + erf_as(x * 0.70710678118654752f)) +
           x * __builtin_amdgcn_exp2f(-0.5f * x * x * 1.4426950408889634f) * 0.39894228040143268f;
}

// ------------------------------------------------------------------ features

__global__ void k_log1p_outdeg(const int32_t *__restrict__ outdeg, int32_t V, float *__restrict__ vals) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < V) vals[v] = log1pf((float)outdeg[v]);
}

__global__ void k_features(const int32_t *__restrict__ off, const int32_t *__restrict__ outdeg,
                           const float *__restrict__ sumlog, int32_t V, float *__restrict__ feats) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const int32_t indeg = off[v + 1] - off[v];
    feats[v * 3 + 0] = log1pf((float)indeg);
    feats[v * 3 + 1] = log1pf((float)outdeg[v]);
    feats[v * 3 + 2] = indeg > 0 ? sumlog[v] / (float)indeg : 0.0f;
}

size_t features_ws_bytes(const cagra_segments *seg) {
    return align_up((size_t)seg->V * 4, 256) * 2 + align_up((size_t)(seg->Q > 0 ? seg->Q : 1) * 4, 256) + 256;
}

cagra_status launch_features(const cagra_graph *g, const cagra_segments *seg, float *feats, void *ws,
                             hipStream_t st) {
    char *p = (char *)ws;
    float *vals = (float *)p;
    float *sumlog = (float *)(p + align_up((size_t)seg->V * 4, 256));
    float *partial = (float *)(p + 2 * align_up((size_t)seg->V * 4, 256));
    const unsigned grid = (unsigned)ceil_div(g->V, 256);
    k_log1p_outdeg<<<grid, 256, 0, st>>>(g->out_degree, g->V, vals);
    CAGRA_LAUNCH_CHECK();
    cagra_status s;
    if ((s = launch_gather(seg, CAGRA_SUM_F32, CAGRA_F32, vals, partial, st)) != CAGRA_OK) return s;
    if ((s = launch_merge_sum_fixed24(seg, partial, sumlog, st)) != CAGRA_OK) return s;
    k_features<<<grid, 256, 0, st>>>(g->in_offsets, g->out_degree, sumlog, g->V, feats);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

// ------------------------------------------------------------------ network

// BF16 weights to FP32 in LDS, shared by all rows of the workgroup.
__device__ __forceinline__ void load_weights(const uint16_t *__restrict__ wb, float *w) {
    for (int i = threadIdx.x; i < kNParam; i += blockDim.x) w[i] = bf16_to_f32(wb[i]);
}

constexpr int kFwdThreads = 256;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __bf16 bits_to_bf16(uint16_t b) { return __builtin_bit_cast(__bf16, b); }

// Forward pass, 16 rows per wave step. The 64x64 hidden layer is a dense
// contraction and runs on the matrix cores (v_mfma_f32_16x16x32_bf16: BF16
// inputs, FP32 accumulation). Lane l computes the first-layer units
// u = 32s + 8(l/16) + t of row l%16 directly in the A-operand layout, holds the
// BF16 weights of W2 as B operands for the whole kernel, and receives
// z2[4(l/16) + r][16c + l%16] in the accumulators; the output layer is a
// 16-lane butterfly sum. The weights are BF16 by definition; the FP32
// activations are not, so each one enters the product as two BF16 operands,
// hi = bf16(h) and lo = bf16(h - hi) (|h - hi - lo| <= 2^-17 |h|), and both
// halves are accumulated: the hidden product keeps FP32-level accuracy for
// twice the (cheap) matrix instructions.
// With kRows, the i-th row processed is rows[i] (features read and output
// written at that row); the count is n_dev[0] when n_dev is given. Each
// row's arithmetic does not depend on the other rows of its tile, so a row's
// output is the same bits whichever rows share its tile.
template <bool kRows>
__global__ __launch_bounds__(kFwdThreads) void k_mlp_forward(const float *__restrict__ feats, int64_t n,
                                                             const uint16_t *__restrict__ wb,
                                                             const float *__restrict__ norm,
                                                             float *__restrict__ y,
                                                             const int32_t *__restrict__ rows,
                                                             const int32_t *__restrict__ n_dev) {
    if (n_dev) n = n_dev[0];
    const int lane = threadIdx.x & 63, kq = lane >> 4, jl = lane & 15;
    // first-layer weights of this lane's 16 units, second-layer operands, output weights
    float w1[16][3], b1[16];
    bf16x8 B[4][2];
    float b2[4], w3[4];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int u = 32 * s + 8 * kq + t;
            w1[8 * s + t][0] = bf16_to_f32(wb[kOffW1 + 3 * u + 0]);
            w1[8 * s + t][1] = bf16_to_f32(wb[kOffW1 + 3 * u + 1]);
            w1[8 * s + t][2] = bf16_to_f32(wb[kOffW1 + 3 * u + 2]);
            b1[8 * s + t] = bf16_to_f32(wb[kOffB1 + u]);
        }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int j = 16 * c + jl;
        b2[c] = bf16_to_f32(wb[kOffB2 + j]);
        w3[c] = bf16_to_f32(wb[kOffW3 + j]);
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int t = 0; t < 8; ++t) B[c][s][t] = bits_to_bf16(wb[kOffW2 + j * kH + 32 * s + 8 * kq + t]);
    }
    const float b3 = bf16_to_f32(wb[kOffB3]);
    const float m0 = norm[0], m1 = norm[1], m2 = norm[2], s0 = norm[3], s1 = norm[4], s2 = norm[5];
    const int64_t tiles = (n + 15) / 16;
    const int64_t wave = ((int64_t)blockIdx.x * kFwdThreads + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * kFwdThreads) >> 6;
    if (wave >= tiles) return;  // no workgroup-wide synchronization below
    // The features of the next tile and the row ids of the one after it are
    // loaded while a tile is computed. Loads past the last row read row n - 1
    // (their results are not used).
    // row ids stay 32-bit (and the loads unconditional) until used as addresses
    auto row_id = [&](int64_t t) -> int32_t {
        const int64_t ii = t * 16 + jl < n ? t * 16 + jl : n - 1;
        if constexpr (kRows) return rows[ii];
        else return (int32_t)ii;
    };
    int32_t r_cur = row_id(wave);
    float f0 = feats[(int64_t)r_cur * 3 + 0], f1 = feats[(int64_t)r_cur * 3 + 1], f2 = feats[(int64_t)r_cur * 3 + 2];
    int32_t r_nxt = row_id(wave + nwaves);
    for (int64_t tile = wave; tile < tiles; tile += nwaves) {
        const float *fn = feats + (int64_t)r_nxt * 3;
        const float g0 = fn[0], g1 = fn[1], g2 = fn[2];
        const int32_t r_nn = row_id(tile + 2 * nwaves);
        const bool live = tile * 16 + jl < n;
        const float x0 = live ? (f0 - m0) * s0 : 0.0f;
        const float x1 = live ? (f1 - m1) * s1 : 0.0f;
        const float x2 = live ? (f2 - m2) * s2 : 0.0f;
        bf16x8 A[2], Alo[2];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int q = 8 * s + t;
                const float h = gelu(fmaf(w1[q][2], x2, fmaf(w1[q][1], x1, fmaf(w1[q][0], x0, b1[q]))));
                const __bf16 hi = (__bf16)h;
                A[s][t] = hi;
                Alo[s][t] = (__bf16)(h - (float)hi);
            }
        float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Alo[0], B[c][0], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Alo[1], B[c][1], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[c][0], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], B[c][1], acc, 0, 0, 0);
#pragma unroll
            for (int q = 0; q < 4; ++q) part[q] = fmaf(w3[c], gelu(acc[q] + b2[c]), part[q]);
        }
        // sum over the 16 lanes (output units) that hold the same four rows
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 8; m >= 1; m >>= 1) part[q] += __shfl_xor(part[q], m, 16);
        // row id of output row 4 kq + q: held by the lane of this group with jl = 4 kq + q
        int32_t dest[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) dest[q] = __shfl(r_cur, 16 * kq + 4 * kq + q);
        if (jl == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t io = tile * 16 + 4 * kq + q;
                if (io < n) y[(int64_t)dest[q]] = part[q] + b3;
            }
        }
        f0 = g0;
        f1 = g1;
        f2 = g2;
        r_cur = r_nxt;
        r_nxt = r_nn;
    }
}

// Backward: persistent workgroups of 128 rows per pass; each thread owns a
// fixed set of parameters and accumulates their gradient over the rows the
// workgroup processes; workgroup partials are summed in a fixed order.
constexpr int kBwdThreads = 128;
constexpr int kBwdRows = 128;
constexpr int kPad = kH + 1;  // row pitch in LDS (avoids bank conflicts on row-private reads)
constexpr int kBwdGrid = 256;

__global__ __launch_bounds__(kBwdThreads) void k_mlp_backward(const float *__restrict__ feats,
                                                              const float *__restrict__ target, int64_t n,
                                                              const uint16_t *__restrict__ wb,
                                                              const float *__restrict__ norm,
                                                              float *__restrict__ part_grad,
                                                              double *__restrict__ part_loss) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    float *w = reinterpret_cast<float *>(smem);              // kNParam (+3 pad)
    float *xs = w + ((kNParam + 3 + 3) & ~3);                 // [rows][4]
    float *dys = xs + kBwdRows * 4;                           // [rows]
    float *h1s = dys + kBwdRows;                              // [rows][kPad]
    float *z2s = h1s + kBwdRows * kPad;                       // [rows][kPad]
    float *dz2s = z2s + kBwdRows * kPad;                      // [rows][kPad]
    float *dz1s = dz2s + kBwdRows * kPad;                     // [rows][kPad]
    load_weights(wb, w);
    __syncthreads();
    const int t = threadIdx.x;
    const float m0 = norm[0], m1 = norm[1], m2 = norm[2], s0 = norm[3], s1 = norm[4], s2 = norm[5];
    const float inv_n2 = 2.0f / (float)n;
    // owned parameters: W2[j][i0..i0+31], and for t < 64: w3[t], b2[t], W1[t][0..2], b1[t]; t == 0: b3
    const int jw = t >> 1, i0 = (t & 1) * 32;
    float gW2[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) gW2[q] = 0.0f;
    float gw3 = 0.0f, gb2 = 0.0f, gW1a = 0.0f, gW1b = 0.0f, gW1c = 0.0f, gb1 = 0.0f, gb3 = 0.0f;
    double loss = 0.0;

    for (int64_t base = (int64_t)blockIdx.x * kBwdRows; base < n; base += (int64_t)gridDim.x * kBwdRows) {
        const int64_t r = base + t;
        const bool live = r < n;
        // forward for this thread's row
        const float x0 = live ? (feats[r * 3 + 0] - m0) * s0 : 0.0f;
        const float x1 = live ? (feats[r * 3 + 1] - m1) * s1 : 0.0f;
        const float x2 = live ? (feats[r * 3 + 2] - m2) * s2 : 0.0f;
        float h1[kH];
#pragma unroll
        for (int i = 0; i < kH; ++i) {
            const float z1 = fmaf(w[kOffW1 + 3 * i + 2], x2,
                                  fmaf(w[kOffW1 + 3 * i + 1], x1, fmaf(w[kOffW1 + 3 * i], x0, w[kOffB1 + i])));
            h1[i] = gelu(z1);
            h1s[t * kPad + i] = h1[i];
        }
        float out = w[kOffB3];
        for (int j = 0; j < kH; ++j) {
            float z = w[kOffB2 + j];
#pragma unroll
            for (int i = 0; i < kH; ++i) z = fmaf(w[kOffW2 + j * kH + i], h1[i], z);
            z2s[t * kPad + j] = z;
            out = fmaf(w[kOffW3 + j], gelu(z), out);
        }
        const float res = live ? out - target[r] : 0.0f;
        loss += (double)res * (double)res;
        const float dy = res * inv_n2;
        dys[t] = dy;
        xs[t * 4 + 0] = x0;
        xs[t * 4 + 1] = x1;
        xs[t * 4 + 2] = x2;
        // dz2 = dy * w3 * gelu'(z2); dh1 = W2^T dz2; dz1 = dh1 * gelu'(z1)
        float dh1[kH];
#pragma unroll
        for (int i = 0; i < kH; ++i) dh1[i] = 0.0f;
        for (int j = 0; j < kH; ++j) {
            const float dz2 = dy * w[kOffW3 + j] * gelu_grad(z2s[t * kPad + j]);
            dz2s[t * kPad + j] = dz2;
#pragma unroll
            for (int i = 0; i < kH; ++i) dh1[i] = fmaf(w[kOffW2 + j * kH + i], dz2, dh1[i]);
        }
#pragma unroll
        for (int i = 0; i < kH; ++i) {
            const float z1 = fmaf(w[kOffW1 + 3 * i + 2], x2,
                                  fmaf(w[kOffW1 + 3 * i + 1], x1, fmaf(w[kOffW1 + 3 * i], x0, w[kOffB1 + i])));
            dz1s[t * kPad + i] = dh1[i] * gelu_grad(z1);
        }
        __syncthreads();
        // parameter-owner accumulation over the pass's rows, in row order
        for (int q = 0; q < kBwdRows; ++q) {
            const float dz2 = dz2s[q * kPad + jw];
#pragma unroll
            for (int c = 0; c < 32; ++c) gW2[c] = fmaf(dz2, h1s[q * kPad + i0 + c], gW2[c]);
        }
        if (t < kH) {
            for (int q = 0; q < kBwdRows; ++q) {
                const float dyq = dys[q];
                gw3 = fmaf(dyq, gelu(z2s[q * kPad + t]), gw3);
                gb2 += dz2s[q * kPad + t];
                const float dz1 = dz1s[q * kPad + t];
                gW1a = fmaf(dz1, xs[q * 4 + 0], gW1a);
                gW1b = fmaf(dz1, xs[q * 4 + 1], gW1b);
                gW1c = fmaf(dz1, xs[q * 4 + 2], gW1c);
                gb1 += dz1;
                if (t == 0) gb3 += dyq;
            }
        }
        __syncthreads();
    }
    float *pg = part_grad + (int64_t)blockIdx.x * kNParam;
#pragma unroll
    for (int c = 0; c < 32; ++c) pg[kOffW2 + jw * kH + i0 + c] = gW2[c];
    if (t < kH) {
        pg[kOffW3 + t] = gw3;
        pg[kOffB2 + t] = gb2;
        pg[kOffW1 + 3 * t + 0] = gW1a;
        pg[kOffW1 + 3 * t + 1] = gW1b;
        pg[kOffW1 + 3 * t + 2] = gW1c;
        pg[kOffB1 + t] = gb1;
    }
    if (t == 0) pg[kOffB3] = gb3;
    // loss: fixed-order sum over the workgroup's threads
    __shared__ double lred[kBwdThreads];
    lred[t] = loss;
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int q = 0; q < kBwdThreads; ++q) s += lred[q];
        part_loss[blockIdx.x] = s;
    }
}

__global__ void k_grad_reduce(const float *__restrict__ part_grad, const double *__restrict__ part_loss, int grid,
                              int64_t n, float *__restrict__ grad, double *__restrict__ loss_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kNParam) {
        double s = 0.0;
        for (int b = 0; b < grid; ++b) s += (double)part_grad[(int64_t)b * kNParam + i];
        grad[i] = (float)s;
    }
    if (i == 0) {
        double s = 0.0;
        for (int b = 0; b < grid; ++b) s += part_loss[b];
        loss_out[0] = s / (double)n;
    }
}

size_t mlp_grad_ws_bytes() { return align_up((size_t)kBwdGrid * kNParam * 4, 256) + (size_t)kBwdGrid * 8 + 256; }

static size_t bwd_lds_bytes() {
    return (size_t)(((kNParam + 3 + 3) & ~3) + kBwdRows * 4 + kBwdRows + 4 * kBwdRows * kPad) * sizeof(float);
}

static unsigned forward_grid(int64_t n) {
    int64_t g = ceil_div(ceil_div(n, 16), kFwdThreads / 64);
    return (unsigned)(g > 4096 ? 4096 : (g < 1 ? 1 : g));
}

cagra_status launch_mlp_forward(const float *feats, int64_t n, const uint16_t *wb, const float *norm, float *y,
                                hipStream_t st) {
    if (n == 0) return CAGRA_OK;
    k_mlp_forward<false><<<forward_grid(n), kFwdThreads, 0, st>>>(feats, n, wb, norm, y, nullptr, nullptr);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

cagra_status launch_mlp_grad(const float *feats, const float *target, int64_t n, const uint16_t *wb,
                             const float *norm, float *grad, double *loss, void *ws, hipStream_t st) {
    if (cagra_status a_ = ensure_dynamic_lds((const void *)k_mlp_backward)) return a_;
    float *pg = (float *)ws;
    double *pl = (double *)((char *)ws + align_up((size_t)kBwdGrid * kNParam * 4, 256));
    k_mlp_backward<<<kBwdGrid, kBwdThreads, bwd_lds_bytes(), st>>>(feats, target, n, wb, norm, pg, pl);
    CAGRA_LAUNCH_CHECK();
    k_grad_reduce<<<(unsigned)ceil_div(kNParam, 256), 256, 0, st>>>(pg, pl, kBwdGrid, n, grad, loss);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

// Adam (Kingma & Ba 2015) on the FP32 master weights, then round to BF16.
__global__ void k_adam(float *__restrict__ master, uint16_t *__restrict__ wb, float *__restrict__ m,
                       float *__restrict__ v, const float *__restrict__ g, int32_t step, float lr, float b1,
                       float b2, float eps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNParam) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.0f - powf(b1, (float)step));
    const float vh = vi / (1.0f - powf(b2, (float)step));
    const float p = master[i] - lr * mh / (sqrtf(vh) + eps);
    master[i] = p;
    wb[i] = f32_to_bf16(p);
}

cagra_status launch_adam(float *master, uint16_t *wb, float *m, float *v, const float *g, int32_t step, float lr,
                         float b1, float b2, float eps, hipStream_t st) {
    k_adam<<<(unsigned)ceil_div(kNParam, 256), 256, 0, st>>>(master, wb, m, v, g, step, lr, b1, b2, eps);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

// ------------------------------------------------------------------ start vector

// Spans of kSoftSpan outputs per workgroup, kSoftItems per thread with their
// loads issued together; the per-span partials are combined by one workgroup
// in a fixed order (so the start vector is the same bits on every run).
constexpr int kSoftThreads = 256;
constexpr int kSoftItems = 16;
constexpr int kSoftSpan = kSoftThreads * kSoftItems;

__global__ __launch_bounds__(kSoftThreads) void k_soft_max(const float *__restrict__ y, int32_t V,
                                                           double *__restrict__ blk) {
    __shared__ double red[2 * kSoftThreads / 64];
    const int64_t lo = (int64_t)blockIdx.x * kSoftSpan;
    float x[kSoftItems];
#pragma unroll
    for (int j = 0; j < kSoftItems; ++j) {
        const int64_t v = lo + j * kSoftThreads + threadIdx.x;
        x[j] = y[v < V ? v : lo];
    }
    double mx = -INFINITY, bad = 0.0;
#pragma unroll
    for (int j = 0; j < kSoftItems; ++j) {
        if (lo + j * kSoftThreads + threadIdx.x >= V) continue;
        if (!isfinite(x[j])) bad += 1.0;
        else mx = fmax(mx, (double)x[j]);
    }
    for (int d = 32; d >= 1; d >>= 1) {
        mx = fmax(mx, __shfl_down(mx, d, 64));
        bad += __shfl_down(bad, d, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[2 * w] = mx;
        red[2 * w + 1] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m2 = red[0], b2 = red[1];
        for (int i = 1; i < kSoftThreads / 64; ++i) {
            m2 = fmax(m2, red[2 * i]);
            b2 += red[2 * i + 1];
        }
        blk[blockIdx.x * 2 + 0] = m2;
        blk[blockIdx.x * 2 + 1] = b2;
    }
}

// scal[0] = max, scal[1] = count of non-finite outputs: one workgroup, thread t
// combining partials t, t + 256, ... in order, then a fixed reduction tree
__global__ __launch_bounds__(kSoftThreads) void k_soft_max_final(const double *__restrict__ blk, int32_t nblk,
                                                                 double *__restrict__ scal) {
    __shared__ double red[2 * kSoftThreads / 64];
    double mx = -INFINITY, bad = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kSoftThreads) {
        mx = fmax(mx, blk[b * 2]);
        bad += blk[b * 2 + 1];
    }
    for (int d = 32; d >= 1; d >>= 1) {
        mx = fmax(mx, __shfl_down(mx, d, 64));
        bad += __shfl_down(bad, d, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[2 * w] = mx;
        red[2 * w + 1] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m2 = red[0], b2 = red[1];
        for (int i = 1; i < kSoftThreads / 64; ++i) {
            m2 = fmax(m2, red[2 * i]);
            b2 += red[2 * i + 1];
        }
        scal[0] = m2;
        scal[1] = b2;
    }
}

__global__ __launch_bounds__(kSoftThreads) void k_soft_sum(const float *__restrict__ y, int32_t V,
                                                           const double *__restrict__ scal, double *__restrict__ blk) {
    __shared__ double red[kSoftThreads / 64];
    const int64_t lo = (int64_t)blockIdx.x * kSoftSpan;
    const double mx = scal[0];
    float x[kSoftItems];
#pragma unroll
    for (int j = 0; j < kSoftItems; ++j) {
        const int64_t v = lo + j * kSoftThreads + threadIdx.x;
        x[j] = y[v < V ? v : lo];
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kSoftItems; ++j)
        if (lo + j * kSoftThreads + threadIdx.x < V) s += exp((double)x[j] - mx);
    s = block_sum_f64<kSoftThreads>(s, red);
    if (threadIdx.x == 0) blk[blockIdx.x] = s;
}

// scal[2] = sum of exp(y - max) over all vertices (fixed order, as above)
__global__ __launch_bounds__(kSoftThreads) void k_soft_sum_final(const double *__restrict__ blk, int32_t nblk,
                                                                 double *__restrict__ scal) {
    __shared__ double red[kSoftThreads / 64];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kSoftThreads) s += blk[b];
    s = block_sum_f64<kSoftThreads>(s, red);
    if (threadIdx.x == 0) {
        scal[2] = s;
        scal[3] = 0.0;
    }
}

__global__ void k_soft_write(const float *__restrict__ y, int32_t V, const double *__restrict__ scal,
                             float *__restrict__ r0) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < V) r0[v] = (float)(exp((double)y[v] - scal[0]) / scal[2]);
}

size_t softmax_ws_bytes(int32_t V) { return (size_t)ceil_div(V, kSoftSpan) * 2 * sizeof(double) + 256; }

// ------------------------------------------------------------------ training inputs

// Regression target of one vertex: log(V * r) (the network predicts log-ranks
// relative to the uniform 1/V; ranks below 1e-30 are clamped there).
__global__ void k_targets(const float *__restrict__ rank, int32_t V, float *__restrict__ t) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < V) t[v] = (float)log((double)V * fmax((double)rank[v], 1e-30));
}

cagra_status launch_targets(const float *rank, int32_t V, float *t, hipStream_t st) {
    k_targets<<<(unsigned)ceil_div(V, 256), 256, 0, st>>>(rank, V, t);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

// Feature standardization: per column the mean and the sample standard
// deviation (n - 1 denominator), FP64, two passes, fixed order: per-block
// partial sums of kNormSpan rows, then one workgroup adds them in block order.
constexpr int kNormSpan = 65536;
int32_t norm_blocks(int64_t n) { return (int32_t)ceil_div(n, kNormSpan); }
size_t norm_ws_bytes(int64_t n) { return align_up((size_t)norm_blocks(n) * 3 * sizeof(double), 256) + 256; }

__global__ __launch_bounds__(256) void k_norm_pass(const float *__restrict__ f, int64_t n,
                                                   const double *__restrict__ mean, double *__restrict__ blk) {
    __shared__ double red[4 * 4];
    const int64_t lo = (int64_t)blockIdx.x * kNormSpan, hi = lo + kNormSpan < n ? lo + kNormSpan : n;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    const double m0 = mean ? mean[0] : 0.0, m1 = mean ? mean[1] : 0.0, m2 = mean ? mean[2] : 0.0;
    for (int64_t r = lo + threadIdx.x; r < hi; r += 256) {
        const double x0 = (double)f[r * 3 + 0] - m0, x1 = (double)f[r * 3 + 1] - m1, x2 = (double)f[r * 3 + 2] - m2;
        a[0] += mean ? x0 * x0 : x0;
        a[1] += mean ? x1 * x1 : x1;
        a[2] += mean ? x2 * x2 : x2;
    }
    block_sum4_f64<256>(a, red);
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) blk[(int64_t)blockIdx.x * 3 + c] = a[c];
}

// Adds the block partials in block order (one thread per column); pass 0
// writes the means into norm[0..2] and keeps them as FP64 in mean64, pass 1
// writes 1 / max(std, 1e-6) into norm[3..5].
__global__ void k_norm_final(const double *__restrict__ blk, int32_t nblk, int64_t n, int pass,
                             double *__restrict__ mean64, float *__restrict__ norm) {
    const int c = threadIdx.x;
    if (c >= 3) return;
    double s = 0.0;
    for (int32_t b = 0; b < nblk; ++b) s += blk[(int64_t)b * 3 + c];
    if (pass == 0) {
        mean64[c] = s / (double)n;
        norm[c] = (float)(s / (double)n);
    } else {
        const double sd = n > 1 ? sqrt(s / (double)(n - 1)) : 0.0;
        norm[3 + c] = (float)(1.0 / fmax(sd, 1e-6));
    }
}

cagra_status launch_feature_norm(const float *f, int64_t n, float *norm, void *ws, hipStream_t st) {
    const int32_t nblk = norm_blocks(n);
    double *blk = (double *)ws;
    double *mean64 = (double *)((char *)ws + align_up((size_t)nblk * 3 * sizeof(double), 256));
    k_norm_pass<<<nblk, 256, 0, st>>>(f, n, nullptr, blk);
    CAGRA_LAUNCH_CHECK();
    k_norm_final<<<1, 64, 0, st>>>(blk, nblk, n, 0, mean64, norm);
    CAGRA_LAUNCH_CHECK();
    k_norm_pass<<<nblk, 256, 0, st>>>(f, n, mean64, blk);
    CAGRA_LAUNCH_CHECK();
    k_norm_final<<<1, 64, 0, st>>>(blk, nblk, n, 1, mean64, norm);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

// SplitMix64 finalizer (Steele, Lea & Flood 2014).
__device__ __forceinline__ uint64_t splitmix64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Minibatch draw: row i of draw d is row floor(h * n / 2^64) of the data, with
// h the SplitMix64 output for counter d * batch + i under `seed` (Lemire's
// multiply-shift range reduction; bias below n / 2^64).
__global__ void k_sample_rows(const float *__restrict__ f, const float *__restrict__ t, int64_t n, uint64_t seed,
                              int64_t draw, int32_t batch, float *__restrict__ fo, float *__restrict__ to) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= batch) return;
    const uint64_t ctr = (uint64_t)draw * (uint64_t)batch + (uint64_t)i;
    const uint64_t h = splitmix64_mix(seed + (ctr + 1) * 0x9e3779b97f4a7c15ull);
    const int64_t r = (int64_t)__umul64hi(h, (uint64_t)n);
    fo[i * 3 + 0] = f[r * 3 + 0];
    fo[i * 3 + 1] = f[r * 3 + 1];
    fo[i * 3 + 2] = f[r * 3 + 2];
    to[i] = t[r];
}

cagra_status launch_sample_rows(const float *f, const float *t, int64_t n, uint64_t seed, int64_t draw, int32_t batch,
                                float *fo, float *to, hipStream_t st) {
    k_sample_rows<<<(unsigned)ceil_div(batch, 256), 256, 0, st>>>(f, t, n, seed, draw, batch, fo, to);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

// ------------------------------------------------------------------ learned start, fused

// A vertex without in-edges has features (0, log(1 + out-degree), 0): its
// network output depends on its out-degree alone. The fused start evaluates
// the network once per out-degree below kMemoDeg on exactly those features
// (the bits the feature kernel writes for such a vertex) and copies that
// output to every such vertex; all other rows go through the network
// individually. Since a row's output does not depend on the rows evaluated
// beside it, the result is bit-identical to evaluating every row.
constexpr int32_t kMemoDeg = 1024;

__global__ void k_memo_feats(float *__restrict__ f) {
    const int32_t od = blockIdx.x * blockDim.x + threadIdx.x;
    if (od >= kMemoDeg) return;
    f[od * 3 + 0] = log1pf((float)0);
    f[od * 3 + 1] = log1pf((float)od);
    f[od * 3 + 2] = 0.0f;
}

// The vertices are split in spans of kSplitSpan: a span's vertices without
// in-edges (and out-degree below kMemoDeg) take y from the memo, the others
// are listed in ascending order for the network (count, scan, list: no
// contended atomics, and the list is the same on every run).
constexpr int kSplitThreads = 256;
constexpr int kSplitItems = 16;
constexpr int kSplitSpan = kSplitThreads * kSplitItems;

// A vertex goes through the network unless it has no in-edges and an
// out-degree below kMemoDeg (then the memo holds its output).
__device__ __forceinline__ bool needs_network(int32_t off_v, int32_t off_next, int32_t outdeg_v) {
    return !(off_next == off_v && outdeg_v < kMemoDeg);
}

__global__ __launch_bounds__(kSplitThreads) void k_memo_split_count(const int32_t *__restrict__ off,
                                                                    const int32_t *__restrict__ outdeg, int32_t V,
                                                                    const float *__restrict__ ymemo,
                                                                    float *__restrict__ y,
                                                                    int32_t *__restrict__ span_count) {
    __shared__ int32_t wsum[kSplitThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kSplitSpan;
    // loads issued in one batch (vertices past the end read the span's first)
    int32_t o0[kSplitItems], o1[kSplitItems], od[kSplitItems];
#pragma unroll
    for (int j = 0; j < kSplitItems; ++j) {
        const int64_t v = base + j * kSplitThreads + threadIdx.x;
        const int64_t vv = v < V ? v : base;
        o0[j] = off[vv];
        o1[j] = off[vv + 1];
        od[j] = outdeg[vv];
    }
    float ym[kSplitItems];
#pragma unroll
    for (int j = 0; j < kSplitItems; ++j) ym[j] = ymemo[od[j] < kMemoDeg ? od[j] : 0];
    int32_t c = 0;
#pragma unroll
    for (int j = 0; j < kSplitItems; ++j) {
        const int64_t v = base + j * kSplitThreads + threadIdx.x;
        if (v < V) {
            if (needs_network(o0[j], o1[j], od[j])) ++c;
            else y[v] = ym[j];
        }
    }
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_down(c, d, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int i = 0; i < kSplitThreads / 64; ++i) t += wsum[i];
        span_count[blockIdx.x] = t;
    }
}

// Exclusive scan of n span counts in place (one workgroup); total[0] = the sum.
__global__ __launch_bounds__(1024) void k_scan_spans(int32_t *__restrict__ a, int32_t n, int32_t *__restrict__ total) {
    __shared__ int32_t wsum[16];
    const int per = (n + 1023) / 1024;
    const int lo = threadIdx.x * per;
    int32_t s = 0;
    for (int i = 0; i < per; ++i)
        if (lo + i < n) s += a[lo + i];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t incl = s;
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int32_t pre = incl - s;
    for (int i = 0; i < w; ++i) pre += wsum[i];
    for (int i = 0; i < per; ++i)
        if (lo + i < n) {
            const int32_t x = a[lo + i];
            a[lo + i] = pre;
            pre += x;
        }
    if (threadIdx.x == 1023) total[0] = pre;
}

__global__ __launch_bounds__(kSplitThreads) void k_memo_split_rows(const int32_t *__restrict__ off,
                                                                   const int32_t *__restrict__ outdeg, int32_t V,
                                                                   const int32_t *__restrict__ span_ofs,
                                                                   int32_t *__restrict__ rows) {
    __shared__ int32_t wc[kSplitThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kSplitSpan;
    int32_t run = span_ofs[blockIdx.x];
    // the span's loads in one batch, then the decisions, then the ordered listing
    int32_t o0[kSplitItems], o1[kSplitItems], od[kSplitItems];
#pragma unroll
    for (int j = 0; j < kSplitItems; ++j) {
        const int64_t v = base + j * kSplitThreads + threadIdx.x;
        const int64_t vv = v < V ? v : base;
        o0[j] = off[vv];
        o1[j] = off[vv + 1];
        od[j] = outdeg[vv];
    }
    bool needs[kSplitItems];
#pragma unroll
    for (int j = 0; j < kSplitItems; ++j)
        needs[j] = base + j * kSplitThreads + threadIdx.x < V && needs_network(o0[j], o1[j], od[j]);
#pragma unroll
    for (int j = 0; j < kSplitItems; ++j) {
        const int64_t v = base + j * kSplitThreads + threadIdx.x;
        const bool net = needs[j];
        const uint64_t m = __ballot(net);
        if (lane == 0) wc[w] = (int32_t)__popcll(m);
        __syncthreads();
        int32_t pos = run + (int32_t)__popcll(m & lanemask_lt());
        int32_t all = 0;
        for (int i = 0; i < kSplitThreads / 64; ++i) {
            if (i < w) pos += wc[i];
            all += wc[i];
        }
        if (net) rows[pos] = (int32_t)v;
        run += all;
        __syncthreads();  // wc is rewritten by the next step
    }
}

struct StartWs {
    float *feats, *y, *memo_f, *memo_y;
    int32_t *rows, *count, *spans;
    void *feat_ws, *soft_ws;
};

static size_t start_layout(const cagra_segments *seg, char *base, StartWs *w) {
    const int64_t V = seg->V;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes, 256);
        return base ? base + at : nullptr;
    };
    char *p;
    p = take((size_t)V * 3 * 4);
    if (w) w->feats = (float *)p;
    p = take((size_t)V * 4);
    if (w) w->y = (float *)p;
    p = take((size_t)kMemoDeg * 3 * 4);
    if (w) w->memo_f = (float *)p;
    p = take((size_t)kMemoDeg * 4);
    if (w) w->memo_y = (float *)p;
    p = take((size_t)V * 4);
    if (w) w->rows = (int32_t *)p;
    p = take(256);
    if (w) w->count = (int32_t *)p;
    p = take((size_t)ceil_div(V, kSplitSpan) * 4);
    if (w) w->spans = (int32_t *)p;
    p = take(features_ws_bytes(seg));
    if (w) w->feat_ws = p;
    p = take(softmax_ws_bytes(seg->V));
    if (w) w->soft_ws = p;
    return o + 256;
}

size_t learned_start_ws_bytes(const cagra_segments *seg) { return start_layout(seg, nullptr, nullptr); }

cagra_status launch_learned_start(const cagra_graph *g, const cagra_segments *seg, const uint16_t *wb,
                                  const float *norm, float *rank0, double *scal, void *ws, hipStream_t st) {
    StartWs w;
    start_layout(seg, (char *)ws, &w);
    const int32_t V = g->V;
    cagra_status s;
    if ((s = launch_features(g, seg, w.feats, w.feat_ws, st)) != CAGRA_OK) return s;
    k_memo_feats<<<(unsigned)ceil_div(kMemoDeg, 256), 256, 0, st>>>(w.memo_f);
    CAGRA_LAUNCH_CHECK();
    k_mlp_forward<false><<<forward_grid(kMemoDeg), kFwdThreads, 0, st>>>(w.memo_f, kMemoDeg, wb, norm, w.memo_y, nullptr,
                                                                 nullptr);
    CAGRA_LAUNCH_CHECK();
    const int32_t nspans = (int32_t)ceil_div(V, kSplitSpan);
    k_memo_split_count<<<nspans, kSplitThreads, 0, st>>>(g->in_offsets, g->out_degree, V, w.memo_y, w.y, w.spans);
    CAGRA_LAUNCH_CHECK();
    k_scan_spans<<<1, 1024, 0, st>>>(w.spans, nspans, w.count);
    CAGRA_LAUNCH_CHECK();
    k_memo_split_rows<<<nspans, kSplitThreads, 0, st>>>(g->in_offsets, g->out_degree, V, w.spans, w.rows);
    CAGRA_LAUNCH_CHECK();
    k_mlp_forward<true><<<forward_grid(V), kFwdThreads, 0, st>>>(w.feats, V, wb, norm, w.y, w.rows, w.count);
    CAGRA_LAUNCH_CHECK();
    if ((s = launch_softmax(w.y, V, rank0, scal, w.soft_ws, st)) != CAGRA_OK) return s;
    return CAGRA_OK;
}

cagra_status launch_softmax(const float *y, int32_t V, float *r0, double *scal, void *ws, hipStream_t st) {
    const int32_t nblk = (int32_t)ceil_div(V, kSoftSpan);
    double *blk = (double *)ws;
    k_soft_max<<<nblk, kSoftThreads, 0, st>>>(y, V, blk);
    CAGRA_LAUNCH_CHECK();
    k_soft_max_final<<<1, kSoftThreads, 0, st>>>(blk, nblk, scal);
    CAGRA_LAUNCH_CHECK();
    k_soft_sum<<<nblk, kSoftThreads, 0, st>>>(y, V, scal, blk);
    CAGRA_LAUNCH_CHECK();
    k_soft_sum_final<<<1, kSoftThreads, 0, st>>>(blk, nblk, scal);
    CAGRA_LAUNCH_CHECK();
    k_soft_write<<<(unsigned)ceil_div(V, 256), 256, 0, st>>>(y, V, scal, r0);
    CAGRA_LAUNCH_CHECK();
    return CAGRA_OK;
}

}  // namespace cagra
