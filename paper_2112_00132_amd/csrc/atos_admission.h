// Admission control of the serving daemon (host side, plain C++): query slots,
// worklist-entry budgets and the first-fit heap that holds per-query state in
// the server's device arena.  Kept free of HIP so that it can be tested on
// its own.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>
#include <vector>

namespace atos {
namespace host {

// First-fit allocator over [base, base + bytes) of an arena; freed blocks
// merge with free neighbours.
struct Heap {
    std::map<size_t, size_t> free;  // offset -> bytes

    void reset(size_t base, size_t bytes) {
        free.clear();
        if (bytes) free[base] = bytes;
    }
    bool alloc(size_t bytes, size_t& off) {
        for (auto it = free.begin(); it != free.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const size_t rest = it->second - bytes;
            free.erase(it);
            if (rest) free[off + bytes] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto next = free.lower_bound(off);
        if (next != free.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free.erase(next);
        }
        if (next != free.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free[off] = bytes;
    }
};

// Slots and worklist budgets.  With one pool per ring (a query's tasks all go
// to the ring of its slot, slot % pools), a query takes a free slot of the
// least used pool that still has room for its entries; with a single pool,
// any free slot.  Admission also needs room in the heap.
struct Admission {
    uint32_t pools = 1;
    uint64_t pool_cap = 0;                          // entries per pool
    std::vector<uint64_t> pool_used;
    std::vector<std::vector<uint32_t>> pool_slots;  // free slots per pool
    Heap heap;

    void init(uint32_t slots, uint32_t n_pools, uint64_t cap, size_t heap_base, size_t heap_bytes) {
        pools = n_pools ? n_pools : 1u;
        pool_cap = cap;
        pool_used.assign(pools, 0);
        pool_slots.assign(pools, {});
        for (uint32_t i = slots; i-- > 0;) pool_slots[i % pools].push_back(i);
        heap.reset(heap_base, heap_bytes);
    }
    // false: no slot, entries or memory for it now (the caller retries later)
    bool admit(uint64_t entries, size_t bytes, uint32_t& slot, size_t& off) {
        uint32_t pool = pools;
        for (uint32_t p = 0; p < pools; ++p)
            if (!pool_slots[p].empty() && pool_used[p] + entries <= pool_cap &&
                (pool == pools || pool_used[p] < pool_used[pool]))
                pool = p;
        if (pool == pools) return false;
        if (!heap.alloc(bytes, off)) return false;
        slot = pool_slots[pool].back();
        pool_slots[pool].pop_back();
        pool_used[pool] += entries;
        return true;
    }
    void release(uint32_t slot, uint64_t entries, size_t off, size_t bytes) {
        heap.release(off, bytes);
        pool_slots[slot % pools].push_back(slot);
        pool_used[slot % pools] -= entries;
    }
};

}  // namespace host
}  // namespace atos
