// rg_dispatch.cpp - C ABI of the learned variant dispatcher: cost samples
// measured by the count kernels themselves, the network's forward pass,
// gradient and Adam step, a training loop, and installing a trained network
// as the dispatch table of a context.
#include <cmath>

#include "rg_host.h"

namespace {

uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// counter-based uniform in (0, 1]: SplitMix64 of (seed, stream, counter)
double unit(uint64_t seed, uint64_t stream, uint64_t ctr) {
    const uint64_t g = 0x9E3779B97F4A7C15ull;
    const uint64_t key = mix64(seed + (stream + 1) * g);
    return ((mix64(key + (ctr + 1) * g) >> 11) + 1) * 0x1.0p-53;
}

// He initialisation: weights N(0, 2 / fan_in) by Box-Muller, biases 0
std::vector<float> he_init(uint64_t seed) {
    std::vector<float> p(MLP_PARAMS, 0.f);
    const int fan[3] = {MLP_IN, MLP_H, MLP_H};
    const int rows[3] = {MLP_IN, MLP_H, MLP_H}, cols[3] = {MLP_H, MLP_H, MLP_OUT};
    size_t o = 0;
    uint64_t ctr = 0;
    for (int l = 0; l < 3; ++l) {
        const double sd = std::sqrt(2.0 / fan[l]);
        for (int i = 0; i < rows[l] * cols[l]; ++i) {
            const double u1 = unit(seed, 1, ctr++), u2 = unit(seed, 1, ctr++);
            p[o + i] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
        }
        o += (size_t)rows[l] * cols[l] + cols[l];
    }
    return p;
}

}  // namespace

extern "C" {

rg_status rg_mlp_forward(rg_ctx* c, const float* d_params, const float* d_x, uint64_t n, float* d_y, void* stream) {
    if (!c) return RG_EINVAL;
    if (!d_params || (n && (!d_x || !d_y))) return fail(c, RG_EINVAL, "rg_mlp_forward: null pointer");
    HIPCHK(c, hipSetDevice(c->device));
    launch_mlp_forward(d_params, d_x, n, d_y, (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return RG_OK;
}

rg_status rg_mlp_grad(rg_ctx* c, const float* d_params, const float* d_x, const float* d_t, const uint8_t* d_m,
                      uint64_t n, float* d_grad, float* d_loss, void* stream) {
    if (!c) return RG_EINVAL;
    if (!d_params || !d_grad || (n && (!d_x || !d_t || !d_m))) return fail(c, RG_EINVAL, "rg_mlp_grad: null pointer");
    HIPCHK(c, hipSetDevice(c->device));
    // the partial sums live in the workspace other calls use: order after them
    WorkspaceOrder order(c, (hipStream_t)stream);
    const size_t need = align256((size_t)mlp_grad_blocks(n) * MLP_PARAMS * 4 + 4) +
                        align256((size_t)mlp_grad_blocks(n) * 4 + 4) + 256;
    Scratch sc(c);
    void* base = nullptr;
    if (rg_status s = sc.take(WS_PAIRS, need, &base)) return s;
    Bump b{(uint8_t*)base};
    float* partial = b.take<float>((size_t)mlp_grad_blocks(n) * MLP_PARAMS + 1);
    float* partial_loss = b.take<float>(mlp_grad_blocks(n) + 1);
    float* inv = b.take<float>(1);
    launch_mlp_grad(d_params, d_x, d_t, d_m, n, inv, partial, partial_loss, d_grad, d_loss, (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return RG_OK;
}

rg_status rg_mlp_adam(rg_ctx* c, float* d_params, const float* d_grad, float* d_m, float* d_v, uint32_t step, float lr,
                      void* stream) {
    if (!c) return RG_EINVAL;
    if (!d_params || !d_grad || !d_m || !d_v || step < 1) return fail(c, RG_EINVAL, "rg_mlp_adam: bad argument");
    HIPCHK(c, hipSetDevice(c->device));
    const float b1 = 0.9f, b2 = 0.999f;
    launch_mlp_adam(d_params, d_grad, d_m, d_v, lr, b1, b2, 1e-8f, (float)(1.0 - std::pow(0.9, step)),
                    (float)(1.0 - std::pow(0.999, step)), (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return RG_OK;
}

rg_status rg_dispatch_sample(rg_ctx* c, const rg_pool* A, const rg_pool* B, const uint32_t* d_ia, const uint32_t* d_ib,
                             uint64_t n_pairs, int variant, float* d_x, float* d_t, uint8_t* d_m, uint64_t cap_slots,
                             uint64_t* n_slots, void* stream) {
    if (!c) return RG_EINVAL;
    if (variant < RG_V_GENERIC || variant > RG_V_THREAD)
        return fail(c, RG_EINVAL, "rg_dispatch_sample: variant must be RG_V_GENERIC..RG_V_THREAD");
    if (!n_slots || (cap_slots && (!d_x || !d_t || !d_m)))
        return fail(c, RG_EINVAL, "rg_dispatch_sample: null pointer");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    // count-only intersection with the variant forced, costs recorded per slot
    float* d_cost = nullptr;
    uint64_t* d_cards = nullptr;
    rg_status s = RG_OK;
    if (hipMalloc(&d_cost, 4 * std::max<uint64_t>(cap_slots, 1)) != hipSuccess ||
        hipMalloc(&d_cards, 8 * std::max<uint64_t>(n_pairs, 1)) != hipSuccess)
        s = fail(c, RG_EDEVICE, "rg_dispatch_sample: hipMalloc");
    const int mode0 = c->dispatch_mode, bin0 = c->fixed_bin;
    if (s == RG_OK) {
        c->dispatch_mode = RG_DISPATCH_FIXED;
        c->fixed_bin = variant;
        c->cost_out = d_cost;
        c->cost_cap = cap_slots;
        c->cost_slots = 0;
        s = run_batch(c, RG_AND, A, B, d_ia, d_ib, 0, 0, n_pairs, RG_FLAG_CARD, nullptr, d_cards, nullptr, st);
        c->dispatch_mode = mode0;
        c->fixed_bin = bin0;
        c->cost_out = nullptr;
    }
    if (s == RG_OK) {
        *n_slots = c->cost_slots;
        if (c->cost_slots > cap_slots) s = fail(c, RG_ECAPACITY, "rg_dispatch_sample: more slots than cap_slots");
    }
    if (s == RG_OK) {
        launch_slot_features(c->cost_tasks, c->cost_slots, view(*A), view(*B), variant, d_cost,
                             variant - RG_V_GENERIC, d_x, d_t, d_m, st);
        if (hipGetLastError() != hipSuccess) s = fail(c, RG_EDEVICE, "rg_dispatch_sample: launch failed");
    }
    (void)hipStreamSynchronize(st);
    if (d_cost) (void)hipFree(d_cost);
    if (d_cards) (void)hipFree(d_cards);
    return s;
}

rg_status rg_dispatch_train(rg_ctx* c, const float* d_x, const float* d_t, const uint8_t* d_m, uint64_t n,
                            uint32_t epochs, uint32_t batch, float lr, uint64_t seed, float* d_params,
                            float* d_epoch_loss, void* stream) {
    if (!c) return RG_EINVAL;
    if (!d_params || !d_epoch_loss || !n || !d_x || !d_t || !d_m || batch < 1 || n > 0xFFFFFFFFull)
        return fail(c, RG_EINVAL, "rg_dispatch_train: bad argument");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const uint32_t bsz = (uint32_t)std::min<uint64_t>(batch, n);
    const uint32_t nbk = mlp_grad_blocks(bsz);
    // own scratch: Adam state, gradient, batch rows, permutation, partials
    size_t bytes = 0;
    auto sz = [&](size_t b) { bytes += align256(b); };
    sz(4 * MLP_PARAMS);               // m
    sz(4 * MLP_PARAMS);               // v
    sz(4 * MLP_PARAMS);               // grad
    sz(4);                            // loss
    sz(4);                            // inv count
    sz((size_t)bsz * MLP_IN * 4);     // Xb
    sz((size_t)bsz * MLP_OUT * 4);    // Tb
    sz((size_t)bsz * MLP_OUT);        // Mb
    sz((size_t)n * 4);                // permutation
    sz((size_t)nbk * MLP_PARAMS * 4); // partials
    sz((size_t)nbk * 4);
    void* mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess) return fail(c, RG_EDEVICE, "rg_dispatch_train: hipMalloc");
    Bump b{(uint8_t*)mem};
    float* am = b.take<float>(MLP_PARAMS);
    float* av = b.take<float>(MLP_PARAMS);
    float* grad = b.take<float>(MLP_PARAMS);
    float* loss = b.take<float>(1);
    float* inv = b.take<float>(1);
    float* Xb = b.take<float>((size_t)bsz * MLP_IN);
    float* Tb = b.take<float>((size_t)bsz * MLP_OUT);
    uint8_t* Mb = b.take<uint8_t>((size_t)bsz * MLP_OUT);
    uint32_t* perm = b.take<uint32_t>(n);
    float* partial = b.take<float>((size_t)nbk * MLP_PARAMS);
    float* partial_loss = b.take<float>(nbk);
    auto done = [&](rg_status s) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(mem);
        return s;
    };
    if (seed) {
        std::vector<float> p0 = he_init(seed);
        if (hipMemcpyAsync(d_params, p0.data(), 4 * MLP_PARAMS, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return done(fail(c, RG_EDEVICE, "rg_dispatch_train: parameter upload"));
    }
    launch_fill_u32(reinterpret_cast<uint32_t*>(am), 0, MLP_PARAMS, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(av), 0, MLP_PARAMS, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(d_epoch_loss), 0, epochs, st);
    std::vector<uint32_t> h_perm(n);
    uint32_t step = 0;
    for (uint32_t e = 0; e < epochs; ++e) {
        // seeded Fisher-Yates shuffle of the sample order
        for (uint64_t i = 0; i < n; ++i) h_perm[i] = (uint32_t)i;
        for (uint64_t i = n - 1; i > 0; --i) {
            const uint64_t j = (uint64_t)(unit(seed ? seed : 1, 2 + e, i) * (double)(i + 1)) % (i + 1);
            std::swap(h_perm[i], h_perm[j]);
        }
        if (hipMemcpyAsync(perm, h_perm.data(), 4 * n, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return done(fail(c, RG_EDEVICE, "rg_dispatch_train: permutation upload"));
        const uint64_t nb = (n + bsz - 1) / bsz;
        for (uint64_t k = 0; k < nb; ++k) {
            const uint32_t rows = (uint32_t)std::min<uint64_t>(bsz, n - k * bsz);
            launch_gather_rows(d_x, d_t, d_m, perm, k * bsz, rows, Xb, Tb, Mb, st);
            launch_mlp_grad(d_params, Xb, Tb, Mb, rows, inv, partial, partial_loss, grad, loss, st);
            ++step;
            launch_mlp_adam(d_params, grad, am, av, lr, 0.9f, 0.999f, 1e-8f, (float)(1.0 - std::pow(0.9, step)),
                            (float)(1.0 - std::pow(0.999, step)), st);
            launch_accum_scaled(loss, d_epoch_loss + e, 1.0f / (float)nb, st);
        }
    }
    if (hipGetLastError() != hipSuccess) return done(fail(c, RG_EDEVICE, "rg_dispatch_train: launch failed"));
    return done(RG_OK);
}

rg_status rg_dispatch_set_mlp(rg_ctx* c, const float* d_params, void* stream) {
    if (!c) return RG_EINVAL;
    if (!d_params) return fail(c, RG_EINVAL, "rg_dispatch_set_mlp: null parameters");
    HIPCHK(c, hipSetDevice(c->device));
    if (!c->mlp_table) HIPCHK(c, hipMalloc(&c->mlp_table, MLP_TABLE));
    launch_mlp_table(d_params, c->mlp_table, (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
    c->dispatch_mode = RG_DISPATCH_MLP;
    return RG_OK;
}

rg_status rg_dispatch_table(rg_ctx* c, uint8_t* h_table, uint64_t cap) {
    if (!c) return RG_EINVAL;
    if (!c->mlp_table) return fail(c, RG_EINVAL, "rg_dispatch_table: no network installed");
    if (!h_table || cap < MLP_TABLE) return fail(c, RG_EINVAL, "rg_dispatch_table: buffer smaller than the table");
    HIPCHK(c, hipMemcpy(h_table, c->mlp_table, MLP_TABLE, hipMemcpyDeviceToHost));
    return RG_OK;
}

}  // extern "C"

static_assert(RG_MLP_PARAMS == MLP_PARAMS, "parameter count of the C ABI");
static_assert(RG_MLP_TABLE == MLP_TABLE, "table size of the C ABI");
