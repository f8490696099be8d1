// Micro-benchmarks that measure the ceilings the renderer is compared with:
// random 4-byte gathers from a working set of a given size (global memory and
// LDS), FP64 atomic adds (device scope and workgroup scope, spread and
// hot-spot), VALU issue (FMA chains), and a plain streaming copy (for
// calibrating HBM byte counters).
// Exported through a separate C ABI (libmcrt_micro.so); none of this is on
// the rendering path.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    // integer hash (Wang-style avalanche) for addresses independent of data
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

__global__ void k_gather(const float* __restrict__ data, uint32_t n, uint32_t loads, float* sink) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    float acc = 0.f;
    uint32_t h = mix32(tid * 0x9E3779B9u + 1u);
#pragma unroll 8
    for (uint32_t j = 0; j < loads; ++j) {
        h = mix32(h + j);
        acc += data[h % n];
    }
    if (acc == 1234.5f) sink[tid] = acc;  // keeps the loads alive
}

__global__ void k_gather_lds(const float* __restrict__ data, uint32_t n, uint32_t loads, float* sink) {
    extern __shared__ float tile[];
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) tile[i] = data[i];
    __syncthreads();
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    float acc = 0.f;
    uint32_t h = mix32(tid * 0x9E3779B9u + 1u);
#pragma unroll 8
    for (uint32_t j = 0; j < loads; ++j) {
        h = mix32(h + j);
        acc += tile[h % n];
    }
    if (acc == 1234.5f) sink[tid] = acc;
}

// KIND: 0 f64 device scope, 1 f64 workgroup scope, 2 f32 device scope (no
// return), 3 f32 device scope with the old value used, 4 u64 device scope,
// 5 f64 LDS (n <= 8192), 6 f32 LDS (n <= 16384)
template <int KIND>
__global__ void k_atomic(void* data, uint32_t n, uint32_t ops) {
    __shared__ double lds[8192];
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (KIND == 5 || KIND == 6) {
        for (uint32_t i = threadIdx.x; i < 8192; i += blockDim.x) lds[i] = 0.0;
        __syncthreads();
    }
    // KIND 7 and 8: groups of 8 and 16 consecutive lanes add to consecutive
    // doubles of one hashed line (64 and 128 bytes)
    constexpr uint32_t G = KIND == 7 ? 8u : (KIND == 8 ? 16u : 1u);
    uint32_t h = mix32((G > 1 ? tid / G : tid) * 0x9E3779B9u + 7u);
    float keep = 0.f;
    for (uint32_t j = 0; j < ops; ++j) {
        h = mix32(h + j);
        const uint32_t i = G > 1 ? (h % (n / G)) * G + (tid % G) : h % n;
        if (KIND == 0 || KIND == 7 || KIND == 8) {
            unsafeAtomicAdd((double*)data + i, 1.0);
        } else if (KIND == 1) {
            __hip_atomic_fetch_add((double*)data + i, 1.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else if (KIND == 2) {
            unsafeAtomicAdd((float*)data + i, 1.0f);
        } else if (KIND == 3) {
            keep += atomicAdd((float*)data + i, 1.0f);
        } else if (KIND == 4) {
            atomicAdd((unsigned long long*)data + i, 1ull);
        } else if (KIND == 5) {
            atomicAdd(&lds[i & 8191u], 1.0);
        } else {
            atomicAdd(((float*)lds) + (i & 16383u), 1.0f);
        }
    }
    if (KIND == 5 || KIND == 6) {
        __syncthreads();
        if (threadIdx.x == 0 && lds[0] == -1.0) ((double*)data)[0] = lds[1];
    }
    if (KIND == 3 && keep == -1.f) ((float*)data)[0] = keep;
}

// Dependent gathers from a small working set (as in a voxel walk) with a
// side write every `period` iterations: KIND 0 none, 1 a 4-byte store, 2 an
// FP64 atomic add without return, 3 a 32-byte store, all to hashed
// addresses of `out` (n_out elements of 32 bytes).  Measures what writes
// in flight cost the loads that follow them.
template <int KIND>
__global__ void k_gather_write(const float* __restrict__ data, uint32_t n, uint32_t iters, uint32_t period,
                               float4* out, uint32_t n_out, float* sink) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t h = mix32(tid * 0x9E3779B9u + 3u);
    float acc = 0.f;
    for (uint32_t j = 0; j < iters; ++j) {
        const float v = data[h % n];
        acc += v;
        h = mix32(h + __float_as_uint(v));  // the next address depends on the load
        if (KIND != 0 && (j % period) == period - 1) {
            const uint32_t o = mix32(h ^ 0x5bd1e995u) % n_out;
            if (KIND == 1) {
                ((float*)out)[8 * (size_t)o] = acc;
            } else if (KIND == 2) {
                unsafeAtomicAdd((double*)out + 4 * (size_t)o, (double)acc);
            } else {
                out[2 * (size_t)o] = make_float4(acc, acc, acc, acc);
                out[2 * (size_t)o + 1] = make_float4(acc, acc, acc, acc);
            }
        }
    }
    if (acc == 1234.5f) sink[tid] = acc;
}

// A structured buffer load (element index times the descriptor's stride):
// an index at or past the record count returns zero with no memory access.
__device__ float buf_load_f32(__amdgpu_buffer_rsrc_t rsrc, int index, int offset, int soffset, int aux) __asm(
    "llvm.amdgcn.struct.ptr.buffer.load.f32");

// Replay of captured gather addresses (the walk's own address stream):
// wavefront w loads, lane by lane, the NS indices that captured wavefront w
// of the render loaded on NS consecutive walk steps (idx[(w NS + j) 64 +
// lane], clamped into data) and gathers data at them, `reps` times over, the
// way the render's walk loads them: through a buffer over the n_vox voxels,
// so that the indices past them (rays that have ended, empty runs) return
// zero without a memory access.  No walk arithmetic, and no load depends on
// another: the loads issue as fast as the vector-memory pipeline takes them,
// so the rate bounds what the walk can reach on the same addresses with the
// same wavefronts per CU.
template <int NS>
__global__ void __launch_bounds__(256, 4)
    k_gather_replay(const float* __restrict__ data, uint32_t n, uint32_t n_vox, const uint32_t* __restrict__ idx,
                    uint32_t reps, float* sink) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)data, (short)4, (int)n_vox, 0x00020000);
    const size_t w = (size_t)blockIdx.x * 4 + threadIdx.x / 64;
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t r[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) r[j] = min(idx[(w * NS + j) * 64 + lane], n - 1u);
    float acc = 0.f;
    for (uint32_t k = 0; k < reps; ++k) {
        // a zero offset that counts as changed on every pass, so that the
        // loads stay in the loop (an empty statement: no instruction)
        uint32_t z = 0u;
        asm volatile("" : "+s"(z));
        float v[NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) v[j] = buf_load_f32(rs, (int)(r[j] + z), 0, 0, 0);
#pragma unroll
        for (int j = 0; j < NS; ++j) acc += v[j];
    }
    if (acc == 1234.5f) sink[blockIdx.x * 256 + threadIdx.x] = acc;
}

// VALU issue: eight independent FMA chains per lane (wave64, no packed
// FP32), so that every wavefront has an instruction ready each cycle; the
// rate in wave instructions per CU cycle is the issue ceiling the counters of
// the other kernels are read against.
template <typename T>
__global__ void __launch_bounds__(256) k_valu(T* sink, uint32_t iters, T s) {
    T a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = (T)(threadIdx.x + k) * (T)1e-7;
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
#pragma unroll
            for (int k = 0; k < 8; ++k) a[k] = a[k] * s + (T)1;
    }
    T acc = (T)0;
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += a[k];
    if (acc == (T)1234.5) sink[blockIdx.x * 256 + threadIdx.x] = acc;
}

__global__ void k_copy(const float4* __restrict__ src, float4* __restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" {

// 64 FMAs per lane and iteration, `iters` iterations; grid = blocks x 256;
// fp64 selects double.  Returns a hipError_t value.
int mc_micro_valu(void* sink, uint32_t blocks, uint32_t iters, int fp64, void* stream) {
    if (!sink || blocks == 0) return (int)hipErrorInvalidValue;
    hipStream_t s = (hipStream_t)stream;
    if (fp64)
        hipLaunchKernelGGL(k_valu<double>, dim3(blocks), dim3(256), 0, s, (double*)sink, iters, 0.999999);
    else
        hipLaunchKernelGGL(k_valu<float>, dim3(blocks), dim3(256), 0, s, (float*)sink, iters, 0.999999f);
    return (int)hipGetLastError();
}

// loads per thread; grid = blocks x 256.  Returns a hipError_t value.
int mc_micro_gather(const float* data, uint32_t n, uint32_t blocks, uint32_t loads, int use_lds, float* sink,
                    void* stream) {
    if (!data || n == 0 || !sink) return (int)hipErrorInvalidValue;
    hipStream_t s = (hipStream_t)stream;
    if (use_lds) {
        if ((size_t)n * sizeof(float) > 64 * 1024) return (int)hipErrorInvalidValue;
        hipLaunchKernelGGL(k_gather_lds, dim3(blocks), dim3(256), n * sizeof(float), s, data, n, loads, sink);
    } else {
        hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(256), 0, s, data, n, loads, sink);
    }
    return (int)hipGetLastError();
}

// Atomic adds at hashed addresses in [0, n) of `data` (n elements of the
// kind's type; LDS kinds use min(n, LDS size) and data only as a sink).
int mc_micro_atomic(void* data, uint32_t n, uint32_t blocks, uint32_t ops, int kind, void* stream) {
    if (!data || n == 0 || kind < 0 || kind > 8) return (int)hipErrorInvalidValue;
    if ((kind == 7 && n < 8) || (kind == 8 && n < 16)) return (int)hipErrorInvalidValue;
    hipStream_t s = (hipStream_t)stream;
    switch (kind) {
        case 0: hipLaunchKernelGGL(k_atomic<0>, dim3(blocks), dim3(256), 0, s, data, n, ops); break;
        case 1: hipLaunchKernelGGL(k_atomic<1>, dim3(blocks), dim3(256), 0, s, data, n, ops); break;
        case 2: hipLaunchKernelGGL(k_atomic<2>, dim3(blocks), dim3(256), 0, s, data, n, ops); break;
        case 3: hipLaunchKernelGGL(k_atomic<3>, dim3(blocks), dim3(256), 0, s, data, n, ops); break;
        case 4: hipLaunchKernelGGL(k_atomic<4>, dim3(blocks), dim3(256), 0, s, data, n, ops); break;
        case 5: hipLaunchKernelGGL(k_atomic<5>, dim3(blocks), dim3(256), 0, s, data, n, ops); break;
        case 6: hipLaunchKernelGGL(k_atomic<6>, dim3(blocks), dim3(256), 0, s, data, n, ops); break;
        case 7: hipLaunchKernelGGL(k_atomic<7>, dim3(blocks), dim3(256), 0, s, data, n, ops); break;
        default: hipLaunchKernelGGL(k_atomic<8>, dim3(blocks), dim3(256), 0, s, data, n, ops); break;
    }
    return (int)hipGetLastError();
}

int mc_micro_gather_write(const float* data, uint32_t n, uint32_t blocks, uint32_t iters, uint32_t period, int kind,
                          void* out, uint32_t n_out, float* sink, void* stream) {
    if (!data || n == 0 || !sink || period == 0 || kind < 0 || kind > 3) return (int)hipErrorInvalidValue;
    if (kind != 0 && (!out || n_out == 0)) return (int)hipErrorInvalidValue;
    hipStream_t s = (hipStream_t)stream;
    float4* o = (float4*)out;
    switch (kind) {
        case 0: hipLaunchKernelGGL(k_gather_write<0>, dim3(blocks), dim3(256), 0, s, data, n, iters, period, o, n_out, sink); break;
        case 1: hipLaunchKernelGGL(k_gather_write<1>, dim3(blocks), dim3(256), 0, s, data, n, iters, period, o, n_out, sink); break;
        case 2: hipLaunchKernelGGL(k_gather_write<2>, dim3(blocks), dim3(256), 0, s, data, n, iters, period, o, n_out, sink); break;
        default: hipLaunchKernelGGL(k_gather_write<3>, dim3(blocks), dim3(256), 0, s, data, n, iters, period, o, n_out, sink); break;
    }
    return (int)hipGetLastError();
}

// Replay of n_waves captured wavefronts of n_steps (32 or 48) walk steps
// each: blocks of 4 wavefronts; indices are clamped into [0, n), and those
// at or past n_vox (<= n) read zero without an access.
int mc_micro_gather_replay(const float* data, uint32_t n, uint32_t n_vox, const uint32_t* idx, uint32_t n_waves,
                           uint32_t n_steps, uint32_t reps, float* sink, void* stream) {
    if (!data || n == 0 || n_vox > n || n_vox > 0x7fffffffu || !idx || !sink || n_waves < 4 || n_waves % 4 != 0)
        return (int)hipErrorInvalidValue;
    hipStream_t s = (hipStream_t)stream;
    if (n_steps == 32)
        hipLaunchKernelGGL(k_gather_replay<32>, dim3(n_waves / 4), dim3(256), 0, s, data, n, n_vox, idx, reps, sink);
    else if (n_steps == 48)
        hipLaunchKernelGGL(k_gather_replay<48>, dim3(n_waves / 4), dim3(256), 0, s, data, n, n_vox, idx, reps, sink);
    else
        return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}

// Streaming copy of n16 16-byte elements.
int mc_micro_copy(const void* src, void* dst, int64_t n16, uint32_t blocks, void* stream) {
    if (!src || !dst || n16 <= 0) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const float4*)src, (float4*)dst,
                       n16);
    return (int)hipGetLastError();
}

}  // extern "C"
