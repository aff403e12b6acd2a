// Device helpers shared by the kernels of liblpcg (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lpcg {

constexpr int kWave = 64;

// A substitution writes each solution entry exactly once.  Before a solve the
// output vector is filled with this bit pattern (a NaN payload that FP32
// arithmetic never produces: generated NaNs are canonicalised below), so the
// entry itself serves as its ready flag and no separate flag or fence is
// needed between value and flag.
constexpr uint32_t kUnset = 0x7fffffffu;
constexpr uint32_t kCanonNan = 0x7fc00000u;

__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_agent_i(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent_i(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t publishable(float v) {
    uint32_t b = __float_as_uint(v);
    return (v != v) ? kCanonNan : b;
}

// FP64 partial sums handed from every block to the block that finishes last
// follow the same rule: the slot is preset to kPartUnset, the value is stored
// with one agent-scope atomic store and is its own ready flag.
constexpr uint64_t kPartUnset = 0x7ff4000000000badull;  // signalling-NaN payload, never computed
constexpr uint64_t kCanonNan64 = 0x7ff8000000000000ull;

__device__ __forceinline__ uint64_t ld_agent_u64(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent_u64(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void publish_partial(double *part, int i, double v) {
    const uint64_t b = (v != v) ? kCanonNan64 : (uint64_t)__double_as_longlong(v);
    st_agent_u64(reinterpret_cast<uint64_t *>(part) + i, b);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Next work item of a wave from a shared counter, as a wave-uniform (scalar)
// value.  Every lane executes the atomic (the first active lane adds 1, the
// others add 0) so there is no single-lane branch the compiler could fuse with
// other single-lane code, and readfirstlane makes the result an SGPR, so the
// loop exit on it is a uniform scalar branch.  (A lane-0-only atomic followed
// by a cross-lane broadcast is not safe: the optimiser may rotate the loop so
// that the other lanes re-broadcast a stale register and never leave it.)
__device__ __forceinline__ int wave_ticket(int *ticket) {
    const int leader = __builtin_amdgcn_readfirstlane(lane_id());
    const int old = atomicAdd(ticket, lane_id() == leader ? 1 : 0);
    return __builtin_amdgcn_readfirstlane(old);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Sum over a block of BS threads, fixed reduction tree; result valid in all
// threads.  lds must hold BS / 64 elements.
template <int BS, typename T>
__device__ __forceinline__ T block_sum(T v, T *lds) {
    static_assert(BS % kWave == 0, "block size");
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if (lane_id() == 0) lds[w] = v;
    __syncthreads();
    T s = 0;
#pragma unroll
    for (int i = 0; i < BS / kWave; ++i) s += lds[i];
    return s;
}

// Sum of np published partials in a fixed order (result in all threads);
// waits for each slot to be published and rearms it with kPartUnset.  Each
// thread issues the loads of up to kPubBatch of its slots at once and
// re-polls only the ones still unset, so the wait costs about one memory
// round trip rather than one per slot.  Eight slots per thread cover 2048
// partials of a 256-thread block in one batch and keep the kernels that
// contain the reducer at or under 64 VGPRs (eight waves per SIMD; sixteen
// slots needed about 75, which capped them at six).
constexpr int kPubBatch = 8;
template <int BS>
__device__ __forceinline__ double reduce_published(double *part, int np, double *lds) {
    uint64_t *q = reinterpret_cast<uint64_t *>(part);
    double s = 0.0;
    for (int base = 0; base < np; base += BS * kPubBatch) {
        uint64_t v[kPubBatch];
#pragma unroll
        for (int t = 0; t < kPubBatch; ++t) {
            const int i = base + t * BS + (int)threadIdx.x;
            v[t] = i < np ? ld_agent_u64(q + i) : 0ull;
        }
        for (;;) {
            bool pending = false;
#pragma unroll
            for (int t = 0; t < kPubBatch; ++t) {
                const int i = base + t * BS + (int)threadIdx.x;
                if (i < np && v[t] == kPartUnset) {
                    v[t] = ld_agent_u64(q + i);
                    pending = pending || v[t] == kPartUnset;
                }
            }
            if (!pending) break;
            __builtin_amdgcn_s_sleep(1);
        }
#pragma unroll
        for (int t = 0; t < kPubBatch; ++t) {
            const int i = base + t * BS + (int)threadIdx.x;
            if (i < np) {
                s += __longlong_as_double((long long)v[t]);
                st_agent_u64(q + i, kPartUnset);
            }
        }
    }
    return block_sum<BS>(s, lds);
}

// Two published arrays of np slots each, summed as reduce_published sums
// each (every thread takes its slots in the same order, so the sums are the
// same bit for bit), with their loads issued together and one wait for both.
template <int BS>
__device__ __forceinline__ void reduce_published2(double *pa, double *pb, int np, double *lds, double &sa,
                                                  double &sb) {
    constexpr int H = kPubBatch / 2;
    uint64_t *qa = reinterpret_cast<uint64_t *>(pa);
    uint64_t *qb = reinterpret_cast<uint64_t *>(pb);
    double s0 = 0.0, s1 = 0.0;
    for (int base = 0; base < np; base += BS * H) {
        uint64_t va[H], vb[H];
#pragma unroll
        for (int t = 0; t < H; ++t) {
            const int i = base + t * BS + (int)threadIdx.x;
            va[t] = i < np ? ld_agent_u64(qa + i) : 0ull;
            vb[t] = i < np ? ld_agent_u64(qb + i) : 0ull;
        }
        for (;;) {
            bool pending = false;
#pragma unroll
            for (int t = 0; t < H; ++t) {
                const int i = base + t * BS + (int)threadIdx.x;
                if (i < np && va[t] == kPartUnset) {
                    va[t] = ld_agent_u64(qa + i);
                    pending = pending || va[t] == kPartUnset;
                }
                if (i < np && vb[t] == kPartUnset) {
                    vb[t] = ld_agent_u64(qb + i);
                    pending = pending || vb[t] == kPartUnset;
                }
            }
            if (!pending) break;
            __builtin_amdgcn_s_sleep(1);
        }
#pragma unroll
        for (int t = 0; t < H; ++t) {
            const int i = base + t * BS + (int)threadIdx.x;
            if (i < np) {
                s0 += __longlong_as_double((long long)va[t]);
                s1 += __longlong_as_double((long long)vb[t]);
                st_agent_u64(qa + i, kPartUnset);
                st_agent_u64(qb + i, kPartUnset);
            }
        }
    }
    sa = block_sum<BS>(s0, lds);
    sb = block_sum<BS>(s1, lds);
}

// Deterministic reduction of np partial sums (fixed order), result in all
// threads of the block.
template <int BS>
__device__ __forceinline__ double reduce_partials(const double *part, int np, double *lds) {
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += BS) s += part[i];
    return block_sum<BS>(s, lds);
}

}  // namespace lpcg
