// Throughput probe of the LDS and global atomic paths on gfx950: the
// measurements that decide how the particle kernels accumulate the current
// and the field adjoints (FP64 LDS atomics against FP32 ones, LDS against
// global atomics).  A separate library (libpic355_micro.so) that the
// benchmark script loads; the PIC library does not use it.
//
// Every lane performs ITERS x 32 operations on index (base + 7 j + it) mod
// words of its workgroup's array, base = (thread * stride) mod words, so all
// accesses stay inside the array; stride spreads the lanes of a wave over
// the banks (stride 1: consecutive words).  words is a power of two and the
// modulo a mask, so that the index costs two VALU operations, not a division.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

enum Mode {
    LDS_ADD_F32 = 0,
    LDS_ADD_F64 = 1,
    LDS_ADD_U32 = 2,
    LDS_ADD_U64 = 3,
    LDS_READ_F32 = 4,
    LDS_READ_F64 = 5,
    LDS_WRITE_F32 = 6,
    LDS_WRITE_F64 = 7,
    GLOBAL_ADD_F32 = 8,
    GLOBAL_ADD_F64 = 9,
    NMODES = 10
};

constexpr int THREADS = 256;
constexpr int UNROLL = 32;

template <typename T, int OP>   // OP 0 atomic add, 1 read, 2 write
__global__ void __launch_bounds__(THREADS) k_lds(T *out, int iters, int stride, int words)
{
    extern __shared__ __align__(16) unsigned char raw[];
    T *s = reinterpret_cast<T *>(raw);
    for (int i = threadIdx.x; i < words; i += blockDim.x)
        s[i] = T(0);
    __syncthreads();
    T acc = T(0);
    const int mask = words - 1;
    const int base = (int)(threadIdx.x * stride) & mask;
    for (int it = 0; it < iters; ++it) {
#pragma unroll 8
        for (int j = 0; j < UNROLL; ++j) {
            const int a = (base + 7 * j + it) & mask;
            if (OP == 0)
                __hip_atomic_fetch_add(s + a, T(1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            else if (OP == 1)
                acc += s[a];
            else
                s[a] = (T)(it + j);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0)
        out[blockIdx.x] = s[0] + acc;
}

template <typename T>
__global__ void __launch_bounds__(THREADS) k_global(T *buf, int iters, int stride, int words)
{
    T *g = buf + (int64_t)blockIdx.x * words;   // this workgroup's array
    const int mask = words - 1;
    const int base = (int)(threadIdx.x * stride) & mask;
    for (int it = 0; it < iters; ++it) {
#pragma unroll 8
        for (int j = 0; j < UNROLL; ++j)
            unsafeAtomicAdd(g + ((base + 7 * j + it) & mask), T(1));
    }
}

template <typename T, int OP>
hipError_t launch_lds(void *out, int blocks, int iters, int stride, int words, hipStream_t st)
{
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_lds<T, OP>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_lds<T, OP>), dim3(blocks), dim3(THREADS), (size_t)words * sizeof(T), st,
                       static_cast<T *>(out), iters, stride, words);
    return hipGetLastError();
}

hipError_t launch(int mode, void *buf, int blocks, int iters, int stride, int words, hipStream_t st)
{
    switch (mode) {
    case LDS_ADD_F32: return launch_lds<float, 0>(buf, blocks, iters, stride, words, st);
    case LDS_ADD_F64: return launch_lds<double, 0>(buf, blocks, iters, stride, words, st);
    case LDS_ADD_U32: return launch_lds<uint32_t, 0>(buf, blocks, iters, stride, words, st);
    case LDS_ADD_U64: return launch_lds<unsigned long long, 0>(buf, blocks, iters, stride, words, st);
    case LDS_READ_F32: return launch_lds<float, 1>(buf, blocks, iters, stride, words, st);
    case LDS_READ_F64: return launch_lds<double, 1>(buf, blocks, iters, stride, words, st);
    case LDS_WRITE_F32: return launch_lds<float, 2>(buf, blocks, iters, stride, words, st);
    case LDS_WRITE_F64: return launch_lds<double, 2>(buf, blocks, iters, stride, words, st);
    case GLOBAL_ADD_F32:
        hipLaunchKernelGGL((k_global<float>), dim3(blocks), dim3(THREADS), 0, st, static_cast<float *>(buf), iters,
                           stride, words);
        return hipGetLastError();
    case GLOBAL_ADD_F64:
        hipLaunchKernelGGL((k_global<double>), dim3(blocks), dim3(THREADS), 0, st, static_cast<double *>(buf),
                           iters, stride, words);
        return hipGetLastError();
    default: return hipErrorInvalidValue;
    }
}

}   // namespace

extern "C" {

// Number of modes (0 .. n-1): LDS atomic add f32, f64, u32, u64; LDS read
// f32, f64; LDS write f32, f64; global atomic add f32, f64.
__attribute__((visibility("default"))) int picmb_num_modes(void)
{
    return NMODES;
}

// Time one launch of `blocks` workgroups of 256 threads (after one untimed
// launch) in mode `mode`; words: elements per workgroup array, a power of
// two (LDS modes: words * element size <= 160 KiB).  On success returns 0 and writes the
// launch time in ms and the lane-operations performed; else the HIP error
// code (or -1 for bad arguments).  Allocates and frees its own buffers.
__attribute__((visibility("default"))) int picmb_run(int mode, int blocks, int iters, int stride, int words,
                                                     double *ms, double *lane_ops)
{
    if (mode < 0 || mode >= NMODES || blocks <= 0 || iters <= 0 || stride <= 0 || words <= 0 ||
        (words & (words - 1)) != 0 || !ms || !lane_ops)
        return -1;
    const size_t esz = (mode == LDS_ADD_F32 || mode == LDS_ADD_U32 || mode == LDS_READ_F32 ||
                        mode == LDS_WRITE_F32 || mode == GLOBAL_ADD_F32)
                           ? 4
                           : 8;
    const bool global = mode >= GLOBAL_ADD_F32;
    if (!global && (size_t)words * esz > 160 * 1024)
        return -1;
    const size_t bytes = global ? (size_t)blocks * words * esz : (size_t)blocks * esz;
    void *buf = nullptr;
    hipError_t e = hipMalloc(&buf, bytes);
    if (e != hipSuccess)
        return (int)e;
    hipEvent_t a = nullptr, b = nullptr;
    float t = 0.f;
    if ((e = hipMemset(buf, 0, bytes)) == hipSuccess && (e = hipEventCreate(&a)) == hipSuccess &&
        (e = hipEventCreate(&b)) == hipSuccess && (e = launch(mode, buf, blocks, iters, stride, words, 0)) == hipSuccess &&
        (e = hipDeviceSynchronize()) == hipSuccess && (e = hipEventRecord(a, 0)) == hipSuccess &&
        (e = launch(mode, buf, blocks, iters, stride, words, 0)) == hipSuccess &&
        (e = hipEventRecord(b, 0)) == hipSuccess && (e = hipEventSynchronize(b)) == hipSuccess)
        e = hipEventElapsedTime(&t, a, b);
    if (a)
        hipEventDestroy(a);
    if (b)
        hipEventDestroy(b);
    hipFree(buf);
    if (e != hipSuccess)
        return (int)e;
    *ms = t;
    *lane_ops = (double)blocks * THREADS * iters * UNROLL;
    return 0;
}

}   // extern "C"
