// Microbenchmarks of the primitives the worklist kernels are built from:
// achievable HBM bandwidth (stream copy), random agent-scope atomics, a
// single contended counter, release/acquire fences, and random gathers with
// plain and agent-coherent loads.  They provide the measured ceilings the
// kernels are compared against.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "atos.h"
#include "atos_device.h"

using namespace atos;

namespace {

__device__ inline uint32_t mix32(uint64_t x) {
    x ^= x >> 33;
    x *= 0xFF51AFD7ED558CCDull;
    x ^= x >> 33;
    x *= 0xC4CEB9FE1A85EC53ull;
    x ^= x >> 33;
    return (uint32_t)x;
}

// dst[i] = src[i] over n 16-byte words
__global__ void mb_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// iters random agent-scope FP32 adds into a[0..m)
__global__ void mb_atomic_add_f32(float* a, uint64_t m, uint64_t iters) {
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = t0; i < iters; i += (uint64_t)gridDim.x * blockDim.x)
        add_agent(a + (mix32(i) % m), 1.0f);
}

// iters random agent-scope FP64 adds into a[0..m), old values consumed (as
// the PageRank edge update, which tests the value it replaced)
__global__ void mb_atomic_add_f64(double* a, uint64_t m, uint64_t iters, uint32_t* sink) {
    double acc = 0.0;
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = t0; i < iters; i += (uint64_t)gridDim.x * blockDim.x)
        acc += add_agent(a + (mix32(i) % m), 1.0);
    if (acc == -1.0) *sink = 1u;
}

// iters random agent-scope FP64 additions into a[0..m) whose old value is
// not used (the no-return form of the atomic)
__global__ void mb_atomic_add_f64_noret(double* a, uint64_t m, uint64_t iters) {
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = t0; i < iters; i += (uint64_t)gridDim.x * blockDim.x)
        (void)add_agent(a + (mix32(i) % m), 1.0);
}

// iters random FP64 additions, each wavefront into the slice of a[0..m) that
// belongs to the XCD it runs on (m / 8 entries per XCD), with workgroup
// scope: an address is only ever touched from one XCD, so the additions can
// be performed in that XCD's L2 instead of at the device coherence point.
// The sum of a[] afterwards is `iters` when every addition was atomic.
__global__ void mb_atomic_add_f64_xcd(double* a, uint64_t m, uint64_t iters, uint32_t* sink) {
    const uint64_t slice = m / 8;
    double* base = a + (uint64_t)(xcc_id() & 7u) * slice;
    double acc = 0.0;
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = t0; i < iters; i += (uint64_t)gridDim.x * blockDim.x)
        acc += __hip_atomic_fetch_add(base + (mix32(i) % slice), 1.0, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
    if (acc == -1.0) *sink = 1u;
}

// iters random agent-scope u32 minimums into a[0..m), results consumed
__global__ void mb_atomic_min_u32(uint32_t* a, uint64_t m, uint64_t iters, uint32_t* sink) {
    uint32_t acc = 0;
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = t0; i < iters; i += (uint64_t)gridDim.x * blockDim.x)
        acc += min_agent(a + (mix32(i) % m), (uint32_t)(i & 0xFFFF));
    if (acc == 0xFFFFFFFFu) *sink = acc;
}

// one agent-scope add per wavefront per iteration on a single counter
__global__ void mb_same_address(unsigned long long* c, uint64_t iters) {
    for (uint64_t i = 0; i < iters; ++i)
        if (lane_id() == 0) add_agent(c, 1ull);
}

// release + acquire fence pair per wavefront, with one store between
__global__ void mb_fences(uint32_t* a, uint64_t iters) {
    uint32_t* p = a + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = 0; i < iters; ++i) {
        *p = (uint32_t)i;
        fence_release_agent();
        fence_acquire_agent();
    }
}

// iters random 4-byte gathers from a[0..m): plain (kind 0) or agent-coherent (kind 1)
template <int KIND>
__global__ void mb_gather(const uint32_t* a, uint64_t m, uint64_t iters, uint32_t* sink) {
    uint32_t acc = 0;
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = t0; i < iters; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t* p = a + (mix32(i) % m);
        acc += KIND == 0 ? *p : ld_agent(p);
    }
    if (acc == 0xFFFFFFFFu) *sink = acc;
}

// Message-passing litmus test across XCDs.  Pair p has a writer (block p)
// and a reader (block P + p, P = grid/2 chosen so that the pair sits on
// different XCDs under round-robin dispatch).  Per round i the reader first
// loads data (caching the old value), acknowledges, then spins on flag; the
// writer waits for the acknowledgement, stores data = i + 1, waits for the
// store to complete (s_waitcnt vmcnt(0)), then stores flag = i + 1.  The reader
// then loads data with an agent-scope load and counts a stale value.  Plain
// agent-scope loads/stores only (the primitives the worklist relies on);
// every spin is bounded.  words: [0] stale reads, [1] spin give-ups,
// [2] rounds completed; per pair 3 words (data, flag, ack) at 64 + 64*p.
__global__ void mb_litmus_mp(uint32_t* w, uint32_t rounds, uint32_t pairs, uint32_t spin_limit) {
    if (threadIdx.x != 0) return;
    const uint32_t b = blockIdx.x;
    const bool writer = b < pairs;
    const uint32_t p = writer ? b : b - pairs;
    if (p >= pairs) return;
    uint32_t* data = w + 64 + 64 * p;
    uint32_t* flag = data + 16;
    uint32_t* ack = data + 32;
    uint32_t stale = 0, giveups = 0, done = 0;
    for (uint32_t i = 0; i < rounds; ++i) {
        if (writer) {
            uint32_t spin = 0;
            while (ld_agent(ack) != i && ++spin < spin_limit) __builtin_amdgcn_s_sleep(1);
            if (spin >= spin_limit) { ++giveups; break; }
            st_agent(data, i + 1);
            wait_vmem();
            st_agent(flag, i + 1);
        } else {
            const uint32_t before = ld_agent(data);  // bring the old value into this XCD's caches
            st_agent(ack, i + (before == 0xFFFFFFFFu ? 1u : 0u));
            uint32_t spin = 0;
            while (ld_agent(flag) != i + 1 && ++spin < spin_limit) __builtin_amdgcn_s_sleep(1);
            if (spin >= spin_limit) { ++giveups; break; }
            if (ld_agent(data) != i + 1) ++stale;
            ++done;
        }
    }
    if (stale) atomicAdd(w + 0, stale);
    if (giveups) atomicAdd(w + 1, giveups);
    if (done) atomicAdd(w + 2, done);
}

// Device clock rate: spin until the constant-rate clock has advanced by
// `ticks` (at most `max_spins` reads), recording the start and end readings
// and the number of reads in words [0..2] (as uint64).
__global__ void mb_clock(uint64_t* out, uint64_t ticks, uint64_t max_spins) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const uint64_t t0 = now_ticks();
    uint64_t t = t0, spins = 0;
    while (t - t0 < ticks && spins < max_spins) {
        __builtin_amdgcn_s_sleep(4);
        t = now_ticks();
        ++spins;
    }
    out[0] = t0;
    out[1] = t;
    out[2] = spins;
}

}  // namespace

extern "C" atos_status atos_microbench(int32_t kind, void* d_buf, size_t bytes, int64_t iters,
                                       int32_t grid, int32_t block, void* stream, float* ms) {
    if (!d_buf || !ms || bytes < 4096 || iters < 0 || grid <= 0 || block <= 0 || block > 1024 ||
        (block % 64) != 0)
        return ATOS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return ATOS_EHIP;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return ATOS_EHIP;
    }
    char* buf = (char*)d_buf;
    const uint64_t words4 = bytes / 4;
    uint32_t* sink = (uint32_t*)buf;  // first word: sink for consumed results
    atos_status r = ATOS_OK;
    (void)hipEventRecord(a, s);
    switch (kind) {
        case ATOS_MB_COPY: {
            const uint64_t n16 = bytes / 2 / 16;  // first half -> second half
            hipLaunchKernelGGL(mb_copy, dim3(grid), dim3(block), 0, s, (const uint4*)buf,
                               (uint4*)(buf + n16 * 16), n16);
            break;
        }
        case ATOS_MB_ATOMIC_ADD_F32:
            hipLaunchKernelGGL(mb_atomic_add_f32, dim3(grid), dim3(block), 0, s, (float*)buf + 64,
                               words4 - 64, (uint64_t)iters);
            break;
        case ATOS_MB_ATOMIC_ADD_F64:
            hipLaunchKernelGGL(mb_atomic_add_f64, dim3(grid), dim3(block), 0, s, (double*)buf + 32,
                               words4 / 2 - 32, (uint64_t)iters, sink);
            break;
        case ATOS_MB_ATOMIC_ADD_F64_NORET:
            hipLaunchKernelGGL(mb_atomic_add_f64_noret, dim3(grid), dim3(block), 0, s,
                               (double*)buf + 32, words4 / 2 - 32, (uint64_t)iters);
            break;
        case ATOS_MB_ATOMIC_ADD_F64_XCD:
            hipLaunchKernelGGL(mb_atomic_add_f64_xcd, dim3(grid), dim3(block), 0, s,
                               (double*)buf + 32, (words4 / 2 - 32) / 8 * 8, (uint64_t)iters, sink);
            break;
        case ATOS_MB_ATOMIC_MIN_U32:
            hipLaunchKernelGGL(mb_atomic_min_u32, dim3(grid), dim3(block), 0, s, (uint32_t*)buf + 64,
                               words4 - 64, (uint64_t)iters, sink);
            break;
        case ATOS_MB_SAME_ADDRESS:
            hipLaunchKernelGGL(mb_same_address, dim3(grid), dim3(block), 0, s,
                               (unsigned long long*)(buf + 256), (uint64_t)iters);
            break;
        case ATOS_MB_FENCES:
            if ((uint64_t)grid * block + 64 > words4) {
                r = ATOS_EINVAL;
                break;
            }
            hipLaunchKernelGGL(mb_fences, dim3(grid), dim3(block), 0, s, (uint32_t*)buf + 64,
                               (uint64_t)iters);
            break;
        case ATOS_MB_GATHER_PLAIN:
            hipLaunchKernelGGL(mb_gather<0>, dim3(grid), dim3(block), 0, s,
                               (const uint32_t*)buf + 64, words4 - 64, (uint64_t)iters, sink);
            break;
        case ATOS_MB_GATHER_COHERENT:
            hipLaunchKernelGGL(mb_gather<1>, dim3(grid), dim3(block), 0, s,
                               (const uint32_t*)buf + 64, words4 - 64, (uint64_t)iters, sink);
            break;
        case ATOS_MB_LITMUS_MP: {
            // grid = 2 * pairs; counters in the first words (zeroed here)
            const uint32_t pairs = (uint32_t)grid / 2;
            if (pairs == 0 || 64 + 64ull * pairs + 64 > words4 || iters > 0xFFFFFFF0ll) {
                r = ATOS_EINVAL;
                break;
            }
            if (hipMemsetAsync(buf, 0, (64 + 64ull * pairs + 64) * 4, s) != hipSuccess) {
                r = ATOS_EHIP;
                break;
            }
            hipLaunchKernelGGL(mb_litmus_mp, dim3(2 * pairs), dim3(64), 0, s, (uint32_t*)buf,
                               (uint32_t)iters, pairs, 1u << 20);
            break;
        }
        case ATOS_MB_CLOCK:
            hipLaunchKernelGGL(mb_clock, dim3(1), dim3(64), 0, s, (uint64_t*)buf, (uint64_t)iters,
                               (uint64_t)1 << 26);
            break;
        default:
            r = ATOS_EINVAL;
    }
    if (r == ATOS_OK && hipGetLastError() != hipSuccess) r = ATOS_EHIP;
    (void)hipEventRecord(b, s);
    if (r == ATOS_OK) {
        if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(ms, a, b) != hipSuccess)
            r = ATOS_EHIP;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return r;
}
