// Synthetic frames on the device, the workload of Sec. VII-A (random
// codewords over BPSK-AWGN): uniform payload bits, the CRC appended inside
// K, polar encoding x = u F^{(x)n}, s = 1 - 2x, y = s + sigma n, LLR =
// 2y / sigma^2, quantised for the integer dtypes.  Random numbers come from
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011), normals from the Box-Muller transform.
// Frame f's bits and noise depend only on (seed, f), so a batch can be
// generated in any number of calls.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "pscl.h"

namespace {

#define GDEV __device__ __forceinline__

// One Philox4x32-10 block: counter c under key (k0, k1).
GDEV uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Counter domains: payload blocks and noise blocks of a frame.
constexpr uint32_t DOM_PAYLOAD = 1u, DOM_NOISE = 2u;

// (0, 1) from the top 23 bits, exact in float32: (m + 1/2) / 2^23.
GDEV float unit_open(uint32_t v) {
    return ((float)(v >> 9) + 0.5f) * (1.0f / 8388608.0f);
}

template <typename T>
GDEV T quantise(float l);
template <>
GDEV float quantise<float>(float l) {
    return l;
}
template <>
GDEV int16_t quantise<int16_t>(float l) {
    return (int16_t)fminf(fmaxf(rintf(64.0f * l), -32767.0f), 32767.0f);
}
template <>
GDEV int8_t quantise<int8_t>(float l) {
    return (int8_t)fminf(fmaxf(rintf(4.0f * l), -127.0f), 127.0f);
}

// One workgroup per frame at a time.  info positions ascending; crc_tab[j]
// = the CRC register contribution of payload bit j (MSB-first feeding).
template <typename T>
__global__ void __launch_bounds__(256)
    generate_kernel(int N, int K, int r, const uint16_t* __restrict__ info_pos,
                    const uint64_t* __restrict__ crc_tab, uint32_t k0, uint32_t k1, int64_t first,
                    int64_t F, float sigma, float scale, T* __restrict__ llr,
                    uint8_t* __restrict__ info_out) {
    extern __shared__ uint32_t xw[];  // the frame's bits, N / 32 words (at least one)
    __shared__ unsigned long long crc_acc;
    const int tid = threadIdx.x, NT = blockDim.x;
    const int W = (N + 31) >> 5;
    const int P = K - r;  // payload bits
    for (int64_t fi = blockIdx.x; fi < F; fi += gridDim.x) {
        const int64_t f = first + fi;
        const uint32_t f_lo = (uint32_t)f, f_hi = (uint32_t)(f >> 32);
        for (int w = tid; w < W; w += NT) xw[w] = 0u;
        if (tid == 0) crc_acc = 0ull;
        __syncthreads();
        // payload bit j: bit j % 32 of word (j / 32) % 4 of Philox block
        // j / 128; one 32-bit word per thread
        uint64_t acc = 0ull;
        for (int wd = tid; wd * 32 < P; wd += NT) {
            const uint4 rnd = philox4x32_10(make_uint4((uint32_t)(wd >> 2), f_lo, f_hi, DOM_PAYLOAD), k0, k1);
            const int q = wd & 3;
            const uint32_t word = q == 0 ? rnd.x : q == 1 ? rnd.y : q == 2 ? rnd.z : rnd.w;
            for (int b = 0; b < 32; ++b) {
                const int j = wd * 32 + b;
                if (j >= P) break;
                const uint32_t bit = (word >> b) & 1u;
                if (info_out) info_out[fi * K + j] = (uint8_t)bit;
                if (bit) {
                    acc ^= crc_tab[j];
                    const int pos = info_pos[j];
                    atomicOr(&xw[pos >> 5], 1u << (pos & 31));
                }
            }
        }
        if (r > 0 && acc) atomicXor(&crc_acc, (unsigned long long)acc);
        __syncthreads();
        // CRC: information position P + t carries register bit r - 1 - t
        for (int t = tid; t < r; t += NT) {
            const uint32_t bit = (uint32_t)(crc_acc >> (r - 1 - t)) & 1u;
            if (info_out) info_out[fi * K + P + t] = (uint8_t)bit;
            if (bit) {
                const int pos = info_pos[P + t];
                atomicOr(&xw[pos >> 5], 1u << (pos & 31));
            }
        }
        __syncthreads();
        // x = u F^{(x)n}: the butterfly within words, then across words
        for (int w = tid; w < W; w += NT) {
            uint32_t v = xw[w];
            v ^= (v >> 1) & 0x55555555u;
            v ^= (v >> 2) & 0x33333333u;
            v ^= (v >> 4) & 0x0f0f0f0fu;
            v ^= (v >> 8) & 0x00ff00ffu;
            v ^= (v >> 16) & 0x0000ffffu;
            xw[w] = v;
        }
        for (int sw = 1; sw < W; sw <<= 1) {
            __syncthreads();
            for (int w = tid; w < W; w += NT)
                if (!(w & sw)) xw[w] ^= xw[w + sw];
        }
        __syncthreads();
        // BPSK over AWGN: four values per Philox block (two Box-Muller pairs)
        T* out = llr + fi * N;
        for (int i4 = tid; i4 * 4 < N; i4 += NT) {
            const uint4 rnd = philox4x32_10(make_uint4((uint32_t)i4, f_lo, f_hi, DOM_NOISE), k0, k1);
            float nz[4];
            {
                const float rad0 = sqrtf(-2.0f * logf(unit_open(rnd.x)));
                const float rad1 = sqrtf(-2.0f * logf(unit_open(rnd.z)));
                float s0, c0, s1, c1;
                sincosf(6.283185307179586f * unit_open(rnd.y), &s0, &c0);
                sincosf(6.283185307179586f * unit_open(rnd.w), &s1, &c1);
                nz[0] = rad0 * c0;
                nz[1] = rad0 * s0;
                nz[2] = rad1 * c1;
                nz[3] = rad1 * s1;
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = i4 * 4 + e;
                if (i >= N) break;
                const float s = ((xw[i >> 5] >> (i & 31)) & 1u) ? -1.0f : 1.0f;
                out[i] = quantise<T>(scale * (s + sigma * nz[e]));
            }
        }
        __syncthreads();
    }
}

pscl_status hip_st(hipError_t e) {
    if (e == hipSuccess) return PSCL_OK;
    if (e == hipErrorOutOfMemory) return PSCL_E_NOMEM;
    return PSCL_E_HIP;
}

}  // namespace

struct pscl_generator {
    int N = 0, K = 0, r = 0, dtype = 0;
    int device = 0;  // the tables live on this device
    uint16_t* d_info = nullptr;
    uint64_t* d_crc = nullptr;
};

extern "C" {

void pscl_generator_destroy(pscl_generator* g) {
    if (!g) return;
    (void)hipDeviceSynchronize();
    (void)hipFree(g->d_info);
    (void)hipFree(g->d_crc);
    delete g;
}

pscl_status pscl_generator_create(int N, int K, const uint8_t* frozen_mask, uint64_t crc_poly,
                                  int crc_len, int dtype, pscl_generator** out) {
    if (!out || !frozen_mask || N < 2 || N > 4096 || (N & (N - 1))) return PSCL_E_INVALID;
    if (dtype < PSCL_F32 || dtype > PSCL_I8) return PSCL_E_INVALID;
    std::vector<uint16_t> info;
    for (int i = 0; i < N; ++i)
        if (!frozen_mask[i]) info.push_back((uint16_t)i);
    if ((int)info.size() != K || K < 1 || crc_len < 0 || crc_len > 64 || crc_len >= K)
        return PSCL_E_INVALID;
    // CRC register contribution of each payload bit: the last payload bit
    // contributes x^r mod g = poly, each earlier one x times more
    const int P = K - crc_len;
    std::vector<uint64_t> tab((size_t)P, 0ull);
    if (crc_len > 0) {
        const uint64_t mask = crc_len == 64 ? ~0ull : ((1ull << crc_len) - 1ull);
        const uint64_t top = 1ull << (crc_len - 1);
        uint64_t v = crc_poly & mask;
        for (int j = P - 1; j >= 0; --j) {
            tab[(size_t)j] = v;
            const bool carry = (v & top) != 0;
            v = (v << 1) & mask;
            if (carry) v ^= crc_poly & mask;
        }
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PSCL_E_NODEV;
    pscl_generator* g = new pscl_generator();
    g->device = dev;
    g->N = N;
    g->K = K;
    g->r = crc_len;
    g->dtype = dtype;
    pscl_status st = hip_st(hipMalloc((void**)&g->d_info, info.size() * 2));
    if (st == PSCL_OK)
        st = hip_st(hipMemcpy(g->d_info, info.data(), info.size() * 2, hipMemcpyHostToDevice));
    if (st == PSCL_OK) st = hip_st(hipMalloc((void**)&g->d_crc, std::max<size_t>(tab.size(), 1) * 8));
    if (st == PSCL_OK && !tab.empty())
        st = hip_st(hipMemcpy(g->d_crc, tab.data(), tab.size() * 8, hipMemcpyHostToDevice));
    if (st != PSCL_OK) {
        pscl_generator_destroy(g);
        return st;
    }
    *out = g;
    return PSCL_OK;
}

pscl_status pscl_generate(pscl_generator* g, uint64_t seed, int64_t first_frame, int64_t F,
                          double ebn0_db, void* llr, uint8_t* info, void* stream) {
    if (!g || F < 0 || first_frame < 0) return PSCL_E_INVALID;
    if (F == 0) return PSCL_OK;
    if (!llr) return PSCL_E_INVALID;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != g->device) return PSCL_E_INVALID;
    const double R = (double)(g->K - g->r) / g->N;
    const double sigma2 = 1.0 / (2.0 * R * std::pow(10.0, ebn0_db / 10.0));
    const float sigma = (float)std::sqrt(sigma2), scale = (float)(2.0 / sigma2);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const int grid = (int)std::min<int64_t>(F, 4096);
    const size_t lds = (size_t)((g->N + 31) >> 5) * 4;
    hipStream_t s = (hipStream_t)stream;
    switch (g->dtype) {
        case PSCL_F32:
            hipLaunchKernelGGL(generate_kernel<float>, dim3(grid), dim3(256), lds, s, g->N, g->K,
                               g->r, g->d_info, g->d_crc, k0, k1, first_frame, F, sigma, scale,
                               (float*)llr, info);
            break;
        case PSCL_I16:
            hipLaunchKernelGGL(generate_kernel<int16_t>, dim3(grid), dim3(256), lds, s, g->N,
                               g->K, g->r, g->d_info, g->d_crc, k0, k1, first_frame, F, sigma,
                               scale, (int16_t*)llr, info);
            break;
        default:
            hipLaunchKernelGGL(generate_kernel<int8_t>, dim3(grid), dim3(256), lds, s, g->N, g->K,
                               g->r, g->d_info, g->d_crc, k0, k1, first_frame, F, sigma, scale,
                               (int8_t*)llr, info);
            break;
    }
    return hipGetLastError() == hipSuccess ? PSCL_OK : PSCL_E_HIP;
}

}  // extern "C"
