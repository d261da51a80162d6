// rg_mlp.hip - the learned variant dispatcher: a 12 -> 64 -> 64 -> 6 ReLU
// network (fp32) that predicts the log2 cost of each count variant of one
// matched container pair. Hand-written kernels for its forward pass, its
// gradient (masked mean squared error, chain rule), the Adam update, the
// per-slot input features, and the dispatch table: the network evaluated once
// on a quantised feature grid, argmin over the applicable variants, so that
// per-pair dispatch is one table lookup inside the key-matching kernel.
//
// Parameter layout (flat fp32): W1[12][64], b1[64], W2[64][64], b2[64],
// W3[64][6], b3[6], row-major. Output v is the variant of bin v + BIN_GEN.
#include "rg_internal.h"

namespace rg {

constexpr int O_W1 = 0, O_B1 = O_W1 + MLP_IN * MLP_H, O_W2 = O_B1 + MLP_H, O_B2 = O_W2 + MLP_H * MLP_H,
              O_W3 = O_B2 + MLP_H, O_B3 = O_W3 + MLP_H * MLP_OUT;
static_assert(O_B3 + MLP_OUT == MLP_PARAMS, "parameter layout");

// Forward pass of one sample with the parameters in LDS; keeps z1, z2 for backward.
__device__ __forceinline__ void mlp_fwd(const float* P, const float* x, float* z1, float* z2, float* y) {
    for (int j = 0; j < MLP_H; ++j) {
        float s = P[O_B1 + j];
        for (int i = 0; i < MLP_IN; ++i) s = fmaf(x[i], P[O_W1 + i * MLP_H + j], s);
        z1[j] = s;
    }
    for (int j = 0; j < MLP_H; ++j) {
        float s = P[O_B2 + j];
        for (int i = 0; i < MLP_H; ++i) s = fmaf(fmaxf(z1[i], 0.f), P[O_W2 + i * MLP_H + j], s);
        z2[j] = s;
    }
    for (int v = 0; v < MLP_OUT; ++v) {
        float s = P[O_B3 + v];
        for (int i = 0; i < MLP_H; ++i) s = fmaf(fmaxf(z2[i], 0.f), P[O_W3 + i * MLP_OUT + v], s);
        y[v] = s;
    }
}

__device__ __forceinline__ void load_params(float* sP, const float* P) {
    for (int i = threadIdx.x; i < MLP_PARAMS; i += blockDim.x) sP[i] = P[i];
    __syncthreads();
}

// ---------------------------------------------------------------- inference
__global__ void __launch_bounds__(256) k_mlp_forward(const float* P, const float* X, uint64_t n, float* Y) {
    __shared__ float sP[MLP_PARAMS];
    load_params(sP, P);
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float x[MLP_IN], z1[MLP_H], z2[MLP_H], y[MLP_OUT];
    for (int k = 0; k < MLP_IN; ++k) x[k] = X[i * MLP_IN + k];
    mlp_fwd(sP, x, z1, z2, y);
    for (int v = 0; v < MLP_OUT; ++v) Y[i * MLP_OUT + v] = y[v];
}

// ---------------------------------------------------------------- gradient
// One workgroup per 256 samples: each thread back-propagates its sample and
// adds its parameter gradient into the workgroup's LDS accumulator; the
// workgroup writes its partial gradient and partial loss (fixed order, no
// global atomics); k_mlp_reduce sums the partials in workgroup order.
// inv_cnt = 1 / (number of unmasked targets of the whole batch).
__global__ void __launch_bounds__(256) k_mlp_grad(const float* P, const float* X, const float* T, const uint8_t* M,
                                                  uint64_t n, const float* d_inv_cnt, float* partial,
                                                  float* partial_loss) {
    const float inv_cnt = *d_inv_cnt;
    __shared__ float sP[MLP_PARAMS];
    __shared__ float sG[MLP_PARAMS];
    __shared__ float sL[256];
    for (int i = threadIdx.x; i < MLP_PARAMS; i += 256) sG[i] = 0.f;
    load_params(sP, P);
    const uint64_t s = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    float lsum = 0.f;
    if (s < n) {
        float x[MLP_IN], z1[MLP_H], z2[MLP_H], y[MLP_OUT], dy[MLP_OUT], d2[MLP_H];
        for (int k = 0; k < MLP_IN; ++k) x[k] = X[s * MLP_IN + k];
        mlp_fwd(sP, x, z1, z2, y);
        for (int v = 0; v < MLP_OUT; ++v) {
            const float m = M[s * MLP_OUT + v] ? 1.f : 0.f;
            const float e = y[v] - T[s * MLP_OUT + v];
            dy[v] = m * 2.f * e * inv_cnt;
            lsum += m * e * e;
        }
        // layer 3
        for (int v = 0; v < MLP_OUT; ++v) atomicAdd(&sG[O_B3 + v], dy[v]);
        for (int i = 0; i < MLP_H; ++i) {
            const float h = fmaxf(z2[i], 0.f);
            float g = 0.f;
            for (int v = 0; v < MLP_OUT; ++v) {
                if (h != 0.f) atomicAdd(&sG[O_W3 + i * MLP_OUT + v], h * dy[v]);
                g = fmaf(dy[v], sP[O_W3 + i * MLP_OUT + v], g);
            }
            d2[i] = z2[i] > 0.f ? g : 0.f;
        }
        // layer 2 (dh1 computed into z1's storage once its value is used)
        for (int j = 0; j < MLP_H; ++j)
            if (d2[j] != 0.f) atomicAdd(&sG[O_B2 + j], d2[j]);
        for (int i = 0; i < MLP_H; ++i) {
            const float h = fmaxf(z1[i], 0.f);
            float g = 0.f;
            for (int j = 0; j < MLP_H; ++j) {
                if (h != 0.f && d2[j] != 0.f) atomicAdd(&sG[O_W2 + i * MLP_H + j], h * d2[j]);
                g = fmaf(d2[j], sP[O_W2 + i * MLP_H + j], g);
            }
            z1[i] = z1[i] > 0.f ? g : 0.f;  // now dL/dz1
        }
        // layer 1
        for (int j = 0; j < MLP_H; ++j) {
            const float d1 = z1[j];
            if (d1 == 0.f) continue;
            atomicAdd(&sG[O_B1 + j], d1);
            for (int i = 0; i < MLP_IN; ++i)
                if (x[i] != 0.f) atomicAdd(&sG[O_W1 + i * MLP_H + j], x[i] * d1);
        }
    }
    sL[threadIdx.x] = lsum;
    __syncthreads();
    for (int i = threadIdx.x; i < MLP_PARAMS; i += 256) partial[(uint64_t)blockIdx.x * MLP_PARAMS + i] = sG[i];
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int i = 0; i < 256; ++i) t += sL[i];
        partial_loss[blockIdx.x] = t * inv_cnt;
    }
}

__global__ void k_mlp_reduce(const float* partial, const float* partial_loss, uint32_t nb, float* grad, float* loss) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < MLP_PARAMS) {
        float s = 0.f;
        for (uint32_t b = 0; b < nb; ++b) s += partial[(uint64_t)b * MLP_PARAMS + i];
        grad[i] = s;
    }
    if (i == 0 && loss) {
        float s = 0.f;
        for (uint32_t b = 0; b < nb; ++b) s += partial_loss[b];
        *loss = s;
    }
}

// ---------------------------------------------------------------- Adam
__global__ void k_mlp_adam(float* P, const float* G, float* m, float* v, float lr, float b1, float b2, float eps,
                           float c1, float c2) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MLP_PARAMS) return;
    const float g = G[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------- features
__device__ __forceinline__ void pair_features(uint8_t ta, uint8_t tb, uint32_t ca, uint32_t cb, uint32_t ra,
                                              uint32_t rb, float* f) {
    for (int k = 0; k < MLP_IN; ++k) f[k] = 0.f;
    f[ta - 1] = 1.f;
    f[3 + tb - 1] = 1.f;
    f[6] = log2f(1.f + (float)ca) * (1.f / 16);
    f[7] = log2f(1.f + (float)cb) * (1.f / 16);
    f[8] = log2f(1.f + (float)ra) * (1.f / 16);
    f[9] = log2f(1.f + (float)rb) * (1.f / 16);
    const uint32_t mx = ca > cb ? ca : cb, mn = ca < cb ? ca : cb;
    f[10] = log2f((float)mx / (float)(mn > 0 ? mn : 1)) * (1.f / 16);
    f[11] = 0.f;  // count-only dispatch: the kernels compute the intersection for every operation
}

// Training rows of the slots of one wave: features F[s][12] of matched slots
// (zeros otherwise), and column `col` of the targets: T[s][col] = log2 of the
// slot's measured cost, M[s][col] = 1 when the slot is a matched pair that ran
// with bin want_bin and has a cost.
__global__ void k_slot_features(const Task* tasks, uint64_t n, PoolView A, PoolView B, int want_bin, const float* cost,
                                int col, float* F, float* T, uint8_t* M) {
    const uint64_t s = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const Task t = tasks[s];
    float f[MLP_IN];
    uint8_t ok = 0;
    if (t.kind == KIND_MATCH) {
        const uint8_t ta = A.types[t.ia], tb = B.types[t.ib];
        const uint32_t ra = ta == RG_RUN ? A.size[t.ia] : 0u, rb = tb == RG_RUN ? B.size[t.ib] : 0u;
        pair_features(ta, tb, A.card[t.ia], B.card[t.ib], ra, rb, f);
        ok = t.bin == want_bin && cost[s] > 0.f;
    } else {
        for (int k = 0; k < MLP_IN; ++k) f[k] = 0.f;
    }
    for (int k = 0; k < MLP_IN; ++k) F[s * MLP_IN + k] = f[k];
    T[s * MLP_OUT + col] = ok ? log2f(cost[s]) : 0.f;
    M[s * MLP_OUT + col] = ok;
}

// ---------------------------------------------------------------- dispatch table
// Grid: type_a, type_b (3 x 3), log2 buckets of c_a and c_b (0..16), and of the
// run counts r_a, r_b (0..11, only for run containers; 0 otherwise). Each cell
// is evaluated at its bucket centre and stores the argmin over the applicable
// variants (ties to the lower index) as a bin number.
__global__ void __launch_bounds__(256) k_mlp_table(const float* P, uint8_t* table) {
    __shared__ float sP[MLP_PARAMS];
    load_params(sP, P);
    const uint32_t cell = blockIdx.x * 256 + threadIdx.x;
    if (cell >= MLP_TABLE) return;
    uint32_t r = cell;
    const uint32_t rb = r % 12; r /= 12;
    const uint32_t ra = r % 12; r /= 12;
    const uint32_t qb = r % 17; r /= 17;
    const uint32_t qa = r % 17; r /= 17;
    const uint8_t tb = (uint8_t)(r % 3 + 1); r /= 3;
    const uint8_t ta = (uint8_t)(r + 1);
    // bucket centres: log2(1 + c) = q + 0.5
    const float ca = exp2f(qa + 0.5f) - 1.f, cb = exp2f(qb + 0.5f) - 1.f;
    const float rra = ta == RG_RUN ? exp2f(ra + 0.5f) - 1.f : 0.f, rrb = tb == RG_RUN ? exp2f(rb + 0.5f) - 1.f : 0.f;
    float f[MLP_IN];
    for (int k = 0; k < MLP_IN; ++k) f[k] = 0.f;
    f[ta - 1] = 1.f;
    f[3 + tb - 1] = 1.f;
    f[6] = (qa + 0.5f) * (1.f / 16);
    f[7] = (qb + 0.5f) * (1.f / 16);
    f[8] = log2f(1.f + rra) * (1.f / 16);
    f[9] = log2f(1.f + rrb) * (1.f / 16);
    const float mx = fmaxf(ca, cb), mn = fmaxf(fminf(ca, cb), 1.f);
    f[10] = log2f(mx / mn) * (1.f / 16);
    float z1[MLP_H], z2[MLP_H], y[MLP_OUT];
    mlp_fwd(sP, f, z1, z2, y);
    int best = BIN_GEN;
    float bv = 3.4e38f;
    for (int v = 0; v < MLP_OUT; ++v) {
        const int bin = BIN_GEN + v;
        // a representative cardinality of the cell (its largest: 2^(q+1) - 2)
        if (!variant_applies(bin, ta, tb, (2u << qa) - 2u, (2u << qb) - 2u)) continue;
        if (y[v] < bv) {
            bv = y[v];
            best = bin;
        }
    }
    table[cell] = (uint8_t)best;
}

// ---------------------------------------------------------------- launchers
void launch_mlp_forward(const float* P, const float* X, uint64_t n, float* Y, hipStream_t st) {
    if (n) hipLaunchKernelGGL(k_mlp_forward, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, P, X, n, Y);
}
uint32_t mlp_grad_blocks(uint64_t n) { return (uint32_t)((n + 255) / 256); }
// 1 / (number of set mask bytes), 0 for an empty mask; one workgroup
__global__ void __launch_bounds__(256) k_mask_inv(const uint8_t* M, uint64_t n, float* inv) {
    __shared__ uint64_t tmp[4];
    uint64_t c = 0;
    for (uint64_t i = threadIdx.x; i < n; i += 256) c += M[i] ? 1u : 0u;
    c = block_sum_u64(c, tmp);
    if (threadIdx.x == 0) *inv = c ? 1.f / (float)c : 0.f;
}

void launch_mlp_grad(const float* P, const float* X, const float* T, const uint8_t* M, uint64_t n, float* d_inv,
                     float* partial, float* partial_loss, float* grad, float* loss, hipStream_t st) {
    const uint32_t nb = mlp_grad_blocks(n);
    hipLaunchKernelGGL(k_mask_inv, dim3(1), dim3(256), 0, st, M, n * MLP_OUT, d_inv);
    if (nb) hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(256), 0, st, P, X, T, M, n, (const float*)d_inv, partial,
                               partial_loss);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_PARAMS + 255) / 256), dim3(256), 0, st, partial, partial_loss, nb,
                       grad, loss);
}
void launch_mlp_adam(float* P, const float* G, float* m, float* v, float lr, float b1, float b2, float eps, float c1,
                     float c2, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_PARAMS + 255) / 256), dim3(256), 0, st, P, G, m, v, lr, b1, b2, eps, c1,
                       c2);
}
void launch_slot_features(const Task* tasks, uint64_t n, PoolView A, PoolView B, int want_bin, const float* cost,
                          int col, float* F, float* T, uint8_t* M, hipStream_t st) {
    if (n)
        hipLaunchKernelGGL(k_slot_features, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, tasks, n, A, B,
                           want_bin, cost, col, F, T, M);
}

// rows idx[b0 .. b0 + nb) of (X, T, M) into batch buffers
__global__ void k_gather_rows(const float* X, const float* T, const uint8_t* M, const uint32_t* idx, uint64_t b0,
                              uint32_t nb, float* Xb, float* Tb, uint8_t* Mb) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nb) return;
    const uint64_t src = idx[b0 + r];
    for (int k = 0; k < MLP_IN; ++k) Xb[(uint64_t)r * MLP_IN + k] = X[src * MLP_IN + k];
    for (int v = 0; v < MLP_OUT; ++v) {
        Tb[(uint64_t)r * MLP_OUT + v] = T[src * MLP_OUT + v];
        Mb[(uint64_t)r * MLP_OUT + v] = M[src * MLP_OUT + v];
    }
}

__global__ void k_accum_scaled(const float* x, float* acc, float scale) { *acc += *x * scale; }

void launch_gather_rows(const float* X, const float* T, const uint8_t* M, const uint32_t* idx, uint64_t b0,
                        uint32_t nb, float* Xb, float* Tb, uint8_t* Mb, hipStream_t st) {
    if (nb)
        hipLaunchKernelGGL(k_gather_rows, dim3((nb + 255) / 256), dim3(256), 0, st, X, T, M, idx, b0, nb, Xb, Tb,
                           Mb);
}
void launch_accum_scaled(const float* x, float* acc, float scale, hipStream_t st) {
    hipLaunchKernelGGL(k_accum_scaled, dim3(1), dim3(1), 0, st, x, acc, scale);
}
void launch_mlp_table(const float* P, uint8_t* table, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_table, dim3((MLP_TABLE + 255) / 256), dim3(256), 0, st, P, table);
}

}  // namespace rg
