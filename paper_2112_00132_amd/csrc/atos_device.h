// Device primitives for gfx950 (CDNA4): scoped atomics, fences, wavefront
// aggregation and the worklist ring word format.
//
// Memory model notes (LLVM AMDGPU memory model for GFX942/GFX950): each XCD
// has its own L2, so state shared by all workers (depths, residues, colours,
// ring slots, counters) is read with agent-scope atomic loads and updated
// with agent-scope atomic stores and read-modify-writes, all of which the
// hardware performs at the device coherence point.  See wait_vmem() for how
// publication is ordered without L2-wide fences.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
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
ATOS_DEV T and_agent(T* p, T v) {
    return __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// Wait until this wavefront's outstanding vector memory operations (loads,
// stores, atomics) have completed: s_waitcnt vmcnt(0) (expcnt and lgkmcnt
// left free).  Every location the workers share is accessed only through
// agent-scope atomics (global_* ... sc1, performed at the device coherence
// point), so once such an operation has completed it is visible to every
// later agent-scope access on any XCD; the worklist publishes a task only
// after this wait, and a popper reads a task's data only through loads that
// depend on the slot it read.  This replaces agent-scope release/acquire
// fences, which write back / invalidate the whole L2 of the XCD
// (buffer_wbl2 / buffer_inv) and serialise chip-wide.
ATOS_DEV void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// XCD (XCC) this wavefront runs on.
ATOS_DEV uint32_t xcc_id() {
    uint32_t x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
    return x & 0xFu;
}

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
// Long-idle workers poll about every 3.4 us: hundreds of idle workers polling
// the same few ring counters faster than that slow down the pushes and pops
// of the workers that have work (a lone road-grid BFS on one shared ring).
ATOS_DEV void backoff(uint32_t& spin) {
    if (spin < 8) {
        __builtin_amdgcn_s_sleep(1);
    } else if (spin < 64) {
        __builtin_amdgcn_s_sleep(4);
    } else if (spin < 256) {
        __builtin_amdgcn_s_sleep(16);
    } else {
        __builtin_amdgcn_s_sleep(127);
    }
    ++spin;
}

// 100 MHz constant-rate device clock (s_memrealtime).
ATOS_DEV uint64_t now_ticks() { return wall_clock64(); }

// A deadline on the device clock that tolerates jumps of that clock.  On
// MI355X a kernel started after the GPU had been idle for a while has read a
// start time tens of seconds behind the clock's later readings (its
// deadline then passed at once).  A worker reads the clock at least every
// few milliseconds, so a step of more than a second between two of its
// readings is a jump of the clock, not time it spent: the deadline moves by
// the step.
struct Deadline {
    uint64_t at, last;
    static constexpr uint64_t kJumpTicks = 100000000ull;  // 1 s at 100 MHz

    ATOS_DEV void start(uint64_t timeout_ticks) {
        last = now_ticks();
        at = last + timeout_ticks;
    }
    ATOS_DEV bool passed() {
        const uint64_t now = now_ticks();
        if (now > last + kJumpTicks) at += now - last;  // forward jump: not elapsed time
        else if (now < last) at -= last - now;          // backward step: keep the remaining time
        last = now;
        return now > at;
    }
};

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

constexpr int kMaxQueues = 8;  // one worklist ring per XCD at most

// Counters of one worklist ring; each on its own 128-byte line.
struct alignas(128) QueueCtl {
    uint64_t head;  // next ring position a worker may claim
    uint64_t pad0[15];
    uint64_t tail;  // next ring position a pusher may reserve
    uint64_t pad1[15];
    uint64_t done;  // tasks completed by workers of this queue's XCD
    uint64_t pad2[15];
    uint64_t init_base;  // first ring position of this run
    uint64_t n_init;     // initial tasks placed in this ring
    uint64_t limit;      // discrete launches: positions below this are this launch's work
    uint64_t pad3[13];
};

// Hub board: tasks whose neighbour list is too long for one worker are
// posted here and processed in fixed-size chunks by any worker.
constexpr int kBoardEntries = 256;
constexpr uint32_t kBoardFree = 0u, kBoardPosting = 1u, kBoardOpen = 2u;
constexpr uint64_t kBoardOffsetBits = 40;  // cursor = generation << 40 | next edge offset
// Offset of a closed cursor: above any edge offset, and far enough below 2^40
// that the fetch-adds of claimers racing a close never carry into the generation.
constexpr uint64_t kBoardClosed = 1ull << 39;

struct alignas(64) HubEntry {
    uint32_t state;     // kBoardFree / kBoardPosting / kBoardOpen
    uint32_t vertex;
    uint32_t aux;
    uint32_t val;
    uint64_t end;       // one past the task's last edge (CSR offset)
    uint64_t cursor;    // generation (24 bits) | next unclaimed edge offset (40 bits)
    uint64_t finished;  // edges processed so far
    uint64_t total;     // edges of the task
    uint64_t acc;       // the task's 64-bit accumulator word from prepare
    uint64_t pad;
};
static_assert(sizeof(HubEntry) == 64, "hub entry size");
// Reduction words of a posted task whose application has a finish step: every
// chunk ORs its accumulator words in, and the chunk that completes the task
// runs finish on the union.
constexpr int kBoardRedWords = 4;

struct alignas(256) WsHeader {
    uint32_t status;        // kStatus* bits of the current/last run
    uint32_t zero_pending;  // rings must be cleared by the init kernel of this run
    uint64_t cookie;        // kCookie ^ capacity ^ queues when the rings are consistent
    uint64_t capacity;      // slots per ring
    uint32_t n_queues;
    int32_t scalar_out;     // small per-app result (e.g. colour count)
    uint64_t stat_popped;
    uint64_t stat_pushed;
    uint64_t stat_edges;
    uint64_t stat_rounds;
    uint64_t stat_push_retries;  // failed FREE->FULL attempts (slot of the previous lap still held)
    uint64_t stat_idle;          // worker loop iterations without a task
    uint64_t stat_steals;        // windows claimed from another XCD's ring
    uint32_t bsp_count;     // BSP: size of the next frontier
    uint32_t board_open;    // hub board entries currently posted
    uint64_t stat_hub_posts;  // tasks posted to the hub board
    uint64_t board_mask[kBoardEntries / 64];  // bit e set while entry e is open
    uint64_t pad1[18 - kBoardEntries / 64];
    uint64_t check_cursor;  // PageRank sweep cursor (Check_Size variant)
    uint64_t stat_comb_adds;     // PageRank: residue updates combined in a worker's LDS table
    uint64_t stat_comb_atomics;  // PageRank: device atomics that flushed those tables
    uint32_t comb_min_degree;    // PageRank: every vertex of at least this degree is combined,
    uint32_t comb_count;         //   in slots [0, comb_base) (slots taken)
    uint32_t comb_part_degree;   // and vertices of degree in [this, comb_min_degree) while slots
    uint32_t comb_part_count;    //   [comb_base, table size) last (slots taken)
    uint32_t comb_base;
    uint32_t comb_pad;
    uint64_t pad2[10];
    QueueCtl q[kMaxQueues];
    HubEntry board[kBoardEntries];
    uint64_t board_red[kBoardEntries][kBoardRedWords];
};
static_assert(sizeof(WsHeader) % 256 == 0, "header alignment");
static_assert(sizeof(WsHeader) <= 32768, "header size");
static_assert(offsetof(WsHeader, q) <= 4096, "cookie and status sit in the first 4096 bytes");

// Flags in a trace record's task count.
constexpr uint32_t kTraceHubChunk = 0x80000000u;  // a chunk of a hub task
constexpr uint32_t kTraceBspLevel = 0x40000000u;  // a level of a level-synchronous run

// Per-batch trace buffer (layout of the public atos_trace_record buffer).
struct TraceRec {
    uint64_t t_begin;
    uint64_t t_end;
    uint32_t worker;
    uint32_t tasks;
    uint32_t edges;
    uint32_t vertex;
};
struct alignas(64) TraceBuf {
    uint64_t count;
    uint64_t capacity;
    uint64_t clock_khz;
    uint64_t reserved[5];
    TraceRec rec[1];  // [capacity]
};
static_assert(sizeof(TraceRec) == 32, "trace record size");
static_assert(offsetof(TraceBuf, rec) == 64, "trace header size");

}  // namespace atos
