// Device primitives for gfx950 (CDNA4): scoped atomics, fences, wavefront
// aggregation and the worklist ring word format.
//
// Memory model notes (LLVM AMDGPU memory model for GFX942/GFX950): each XCD
// has its own L2, so state shared by all workers (depths, residues, colours,
// ring slots, counters) is read with agent-scope atomic loads and updated
// with agent-scope atomic read-modify-writes.  Ordering between a worker's
// data updates and the ring slot that publishes a task uses an agent-scope
// release fence before the slot write and an acquire fence after the slot
// read, once per batch rather than per task.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define ATOS_DEV __device__ __forceinline__

namespace atos {

constexpr int kWave = 64;

// ------------------------------------------------------------ scoped atomics
template <class T>
ATOS_DEV T ld_agent(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
ATOS_DEV void st_agent(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
ATOS_DEV T add_agent(T* p, T v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
ATOS_DEV T min_agent(T* p, T v) {
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
ATOS_DEV T max_agent(T* p, T v) {
    return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
ATOS_DEV T or_agent(T* p, T v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
ATOS_DEV T exch_agent(T* p, T v) {
    return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
ATOS_DEV bool cas_agent(T* p, T expected, T desired) {
    return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

ATOS_DEV void fence_acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
ATOS_DEV void fence_release_agent() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
ATOS_DEV void fence_seqcst_agent() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent"); }

// ------------------------------------------------------------ wavefront helpers
ATOS_DEV uint64_t ballot(bool p) { return __ballot(p); }
ATOS_DEV uint32_t lane_id() { return __lane_id(); }
// number of set bits of m below this lane
ATOS_DEV uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
ATOS_DEV uint32_t first_lane_u32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Backoff while spinning: s_sleep(n) idles the wave for about 64*n cycles.
ATOS_DEV void backoff(uint32_t& spin) {
    if (spin < 8) {
        __builtin_amdgcn_s_sleep(1);
    } else if (spin < 64) {
        __builtin_amdgcn_s_sleep(4);
    } else {
        __builtin_amdgcn_s_sleep(16);
    }
    ++spin;
}

// 100 MHz constant-rate device clock (s_memrealtime).
ATOS_DEV uint64_t now_ticks() { return wall_clock64(); }

// 32-bit hash of (seed, id): the murmur3 64-bit finaliser applied to the pair.
ATOS_DEV uint32_t priority_hash(uint64_t seed, uint32_t id) {
    uint64_t x = seed ^ (0x9E3779B97F4A7C15ull * ((uint64_t)id + 1));
    x ^= x >> 33;
    x *= 0xFF51AFD7ED558CCDull;
    x ^= x >> 33;
    x *= 0xC4CEB9FE1A85EC53ull;
    x ^= x >> 33;
    return (uint32_t)x;
}

// ------------------------------------------------------------ ring slot words
// A ring slot is one 64-bit word: [63:48] sequence tag, [47:32] task aux, [31:0]
// vertex.  For the ring position p (a monotonic 64-bit counter) on a ring of
// 2^k slots, lap(p) = p >> k; the slot of p is FREE for p when its tag is
// 2*lap(p) (mod 2^16) and FULL with p's task when its tag is 2*lap(p)+1.  A
// pusher turns FREE(p) into FULL(p) with a compare-and-swap; the popper of p
// turns FULL(p) into FREE(p + 2^k).  A zeroed ring is FREE for laps 0.
struct RingView {
    uint64_t* slots;
    uint64_t mask;
    uint32_t log2cap;

    ATOS_DEV uint64_t* slot(uint64_t pos) const { return slots + (pos & mask); }
    ATOS_DEV uint64_t free_word(uint64_t pos) const {
        return ((2ull * (pos >> log2cap)) & 0xFFFFull) << 48;
    }
    ATOS_DEV uint64_t full_word(uint64_t pos, uint64_t payload) const {
        return (((2ull * (pos >> log2cap) + 1ull) & 0xFFFFull) << 48) | (payload & 0xFFFFFFFFFFFFull);
    }
    ATOS_DEV bool is_full_for(uint64_t word, uint64_t pos) const {
        return (word >> 48) == ((2ull * (pos >> log2cap) + 1ull) & 0xFFFFull);
    }
};

ATOS_DEV uint64_t make_payload(uint32_t vertex, uint32_t aux) {
    return ((uint64_t)(aux & 0xFFFFu) << 32) | (uint64_t)vertex;
}
ATOS_DEV uint32_t payload_vertex(uint64_t w) { return (uint32_t)w; }
ATOS_DEV uint32_t payload_aux(uint64_t w) { return (uint32_t)(w >> 32) & 0xFFFFu; }

// ------------------------------------------------------------ workspace header
// Device-resident control block at the start of every workspace.  Hot
// counters sit on separate 128-byte lines.
enum : uint32_t {
    kStatusOverflow = 1u,
    kStatusTimeout = 2u,
    kStatusAbort = 4u,
    kStatusCorrupt = 8u,
};

constexpr uint64_t kCookie = 0x41544F5357534B31ull;  // "ATOSWSK1"

struct alignas(256) WsHeader {
    uint64_t head;  // next ring position a worker may claim
    uint64_t pad0[15];
    uint64_t tail;  // next ring position a pusher may reserve
    uint64_t pad1[15];
    uint64_t done;  // tasks fully processed (their pushes already reserved)
    uint64_t pad2[15];
    uint64_t check_cursor;  // PageRank sweep cursor (Check_Size variant)
    uint64_t pad3[15];
    uint32_t status;        // kStatus* bits of the current/last run
    uint32_t zero_pending;  // ring must be cleared by the init kernel of this run
    uint64_t cookie;        // kCookie ^ capacity when the ring is consistent
    uint64_t init_base;     // first ring position of this run
    uint64_t n_init;        // initial tasks of this run
    uint64_t capacity;
    uint64_t stat_popped;
    uint64_t stat_pushed;
    uint64_t stat_edges;
    uint64_t stat_rounds;
    int32_t scalar_out;     // small per-app result (e.g. colour count)
    uint32_t bsp_count;     // BSP: size of the next frontier
    uint64_t pad4[4];
};
static_assert(sizeof(WsHeader) % 256 == 0, "header alignment");

}  // namespace atos
