// Internal helpers shared by the HIP kernels of the skew-symmetric eigensolver.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Accumulator vector type of the 16x16x4 MFMA for an element type.
template <typename T> struct acc4;
template <> struct acc4<double> { typedef d4 type; };
template <> struct acc4<float> { typedef f4 type; };

// D = A*B + C on a 16x16 tile with K = 4 (one wavefront).  Lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; it receives D[row][l%16] in its r-th
// result register (r = 0..3) with row = mfma_row<T>(l, r): l/16 + 4r for the
// FP64 instruction and 4(l/16) + r for the FP32 one (measured on gfx950).
template <typename T> __device__ __forceinline__ int mfma_row(int lane, int r);
template <> __device__ __forceinline__ int mfma_row<double>(int lane, int r) { return (lane >> 4) + 4 * r; }
template <> __device__ __forceinline__ int mfma_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }

__device__ __forceinline__ d4 mfma_16x16x4(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_16x16x4(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Bounded spin for device-side waits: a wait that exceeds it sets the error
// word and gives up, so every wave of a persistent kernel always exits.
#define SKEW_SPIN_LIMIT (1u << 22)

// Agent-scope acquire/release accessors for flags and counters.
__device__ __forceinline__ unsigned ld_acquire(const unsigned *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_relaxed(const unsigned *p)
{
    return __hip_atomic_load((const __attribute__((address_space(1))) unsigned *)p, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(unsigned *p, unsigned v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void add_release(unsigned *p, unsigned v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Coherent (agent-scope, relaxed) element accesses for data exchanged between
// workgroups inside one kernel: they bypass the per-XCD caches' stale lines
// without the whole-cache write-back/invalidate that agent-scope fences cost.
// (The pointers are cast to the global address space: a generic pointer
// would make these flat accesses, which also count against the LDS counter.)
typedef __attribute__((address_space(1))) double gbl_double;
typedef __attribute__((address_space(1))) unsigned gbl_unsigned;
__device__ __forceinline__ double ld_coh(const double *p)
{
    return __hip_atomic_load((const gbl_double *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh(double *p, double v)
{
    __hip_atomic_store((gbl_double *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(unsigned *p, unsigned v)
{
    __hip_atomic_store((gbl_unsigned *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait for this wave's outstanding vector memory operations (s_waitcnt
// vmcnt(0); expcnt and lgkmcnt left unconstrained).  On gfx950 a
// workgroup-scope release fence does not wait for global stores, so code that
// publishes data to other workgroups must wait explicitly.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Publish: wait until this wave's earlier (coherent) stores are performed,
// then the workgroup barrier; after it one thread may set a flag, and a
// workgroup that observes the flag reads the data with ld_coh.
__device__ __forceinline__ void wg_publish()
{
    wait_vmem();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
}

// Grid barrier for data exchanged with ld_coh/st_coh: only workgroup-scope
// fences (no whole-cache maintenance); the counter uses relaxed agent-scope
// atomics.  Returns false when the wait gave up.
__device__ __forceinline__ bool grid_sync_coh(unsigned *ctr, unsigned target, unsigned *err)
{
    __shared__ int gs_ok;
    wg_publish();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        int ok = 1;
        while (ld_relaxed(ctr) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > SKEW_SPIN_LIMIT) {
                atomicOr(err, 1u);
                ok = 0;
                break;
            }
        }
        gs_ok = ok;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    return gs_ok != 0;
}

// Grid-wide barrier for kernels whose workgroups are resident together: a monotonic counter
// that every workgroup increments once per barrier; `target` is the count at
// which this barrier opens.  Returns false when the wait gave up.
__device__ __forceinline__ bool grid_sync(unsigned *ctr, unsigned target, unsigned *err)
{
    __shared__ int gs_ok;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        add_release(ctr, 1u);
        unsigned spins = 0;
        int ok = 1;
        // spin with relaxed loads (an acquire load would invalidate caches on
        // every iteration); one acquire fence once the count is reached
        while (ld_relaxed(ctr) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > SKEW_SPIN_LIMIT) {
                atomicOr(err, 1u);
                ok = 0;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        gs_ok = ok;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return gs_ok != 0;
}

// Sums of np partial arrays (stride pst) for the 16 elements a thread owns in
// a 64 x 64 block: thread (tx, ty) = (tid % 64, tid / 64) owns row tx and
// columns ty + 4q; off(i, j) < 0 marks an element outside the array.  The
// loads of four partials are issued together; the summation order over p is
// sequential, so the result does not depend on the batching.
template <class OFF>
__device__ __forceinline__ void sum_partials_2d(const double *__restrict__ P, int np, size_t pst, const OFF &off,
                                                double acc[16])
{
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    int o[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        o[q] = off(tx, ty + 4 * q);
        acc[q] = 0.0;
    }
    int p = 0;
    for (; p + 4 <= np; p += 4) {
        double t[4][16];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < 16; ++q) t[u][q] = (o[q] >= 0) ? P[(size_t)(p + u) * pst + o[q]] : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] += t[u][q];
    }
    for (; p < np; ++p) {
        double t[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) t[q] = (o[q] >= 0) ? P[(size_t)p * pst + o[q]] : 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] += t[q];
    }
}

// 1/d for a normal d: the hardware estimate refined by two Newton steps
// r <- r (2 - d r), each of which squares the relative error, so the result
// is within an ulp or two of the rounded quotient.
__device__ __forceinline__ double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}

// Wavefront maximum (64 lanes) via cross-lane shuffles.
__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Tile t of the lower triangle of a tile grid, row by row: (I, J), J <= I.
__device__ __forceinline__ void tri_index(int t, int &I, int &J)
{
    int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    I = i;
    J = t - i * (i + 1) / 2;
}

// Wavefront sum (64 lanes) via cross-lane shuffles.
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

static inline unsigned cdiv(unsigned a, unsigned b) { return (a + b - 1) / b; }
