// synth_gpu.hip - device twin of the dense-bitset input generator in synth.c.
//
// Same definition as synth_dense_container(): SplitMix64 used as a
// counter-based generator; container (b, k) has threshold
// t = 13107 + rand(seed, b, k) % 39322 and bit 4i+j of word w is set iff
// 16-bit lane j of rand(seed, 2^40 + b*2^16 + k, 16w + i) is below t.
// It writes raw words, laid out [bitmap][key][1024]; it knows nothing of the
// container format that consumes them.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t stream_key(uint64_t seed, uint64_t stream) {
    return mix64(seed + (stream + 1) * GAMMA);
}

// one thread per 64-bit word; grid covers n_bitmaps * n_keys * 1024 words
__global__ void __launch_bounds__(256)
k_dense_words(uint64_t seed, uint32_t b0, uint32_t n_keys, uint64_t n_words, uint64_t* __restrict__ out) {
    uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n_words) return;
    uint64_t w = gid & 1023;
    uint64_t ck = gid >> 10;                 // container index within the launch
    uint64_t k = ck % n_keys;
    uint64_t b = b0 + ck / n_keys;
    uint32_t t = 13107u + (uint32_t)(mix64(stream_key(seed, b) + (k + 1) * GAMMA) % 39322u);
    uint64_t key = stream_key(seed, (1ULL << 40) + (b << 16) + k);
    uint64_t x = 0;
#pragma unroll 4
    for (uint64_t i = 0; i < 16; ++i) {
        uint64_t h = mix64(key + (w * 16 + i + 1) * GAMMA);
#pragma unroll
        for (uint64_t j = 0; j < 4; ++j) {
            uint32_t u = (uint32_t)(h >> (16 * j)) & 0xFFFFu;
            x |= (uint64_t)(u < t) << (4 * i + j);
        }
    }
    out[gid] = x;
}

extern "C" int synth_dense_bitsets_device(uint64_t seed, uint32_t b0, uint32_t n_bitmaps, uint32_t n_keys,
                                          uint64_t* d_words, void* stream) {
    uint64_t n_words = (uint64_t)n_bitmaps * n_keys * 1024;
    if (n_words == 0) return 0;
    uint64_t blocks = (n_words + 255) / 256;
    if (blocks > 0x7FFFFFFFull) return -1;
    hipLaunchKernelGGL(k_dense_words, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream, seed, b0,
                       n_keys, n_words, d_words);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
