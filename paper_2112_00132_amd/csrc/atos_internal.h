// Host-side definitions shared by the translation units of libatos: the
// graph record behind atos_graph_t and small launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>

#include "atos.h"

namespace atos {
namespace host {

constexpr int kInitBlock = 256;

struct GraphRec {
    const void* offs;
    int off64;
    const int32_t* cols;
    int64_t n, m, max_deg;
    uint32_t flags;
    int device;
    int num_cu;
    int64_t clock_khz;  // device wall clock (s_memrealtime) rate
    uint32_t sqrt_class_degree;  // lowest degree of the ~sqrt(n) highest-degree vertices of
                                 // degree >= 64 (colouring's ordered class), 0 = none
};

#define HIP_TRY(expr)                                   \
    do {                                                \
        if ((expr) != hipSuccess) return ATOS_EHIP;     \
    } while (0)

inline uint64_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}
inline uint32_t log2u(uint64_t p) {
    uint32_t l = 0;
    while ((1ull << l) < p) ++l;
    return l;
}
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// grid for a grid-stride kernel of kInitBlock threads over `work` items
inline int init_grid(int64_t work, int num_cu) {
    int64_t g = (work + kInitBlock - 1) / kInitBlock;
    g = std::min<int64_t>(g, (int64_t)num_cu * 16);
    return (int)std::max<int64_t>(g, 1);
}

// workgroups of `kern` that fit on one CU at once (cached per kernel)
inline std::mutex& occupancy_mutex() {
    static std::mutex m;
    return m;
}
inline std::map<const void*, int>& occupancy_cache() {
    static std::map<const void*, int> c;
    return c;
}
template <class K>
int occupancy(K kern, int block) {
    std::lock_guard<std::mutex> lock(occupancy_mutex());
    auto& cache = occupancy_cache();
    auto it = cache.find((const void*)kern);
    if (it != cache.end()) return it->second;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, block, 0) != hipSuccess) nb = 1;
    nb = std::max(nb, 1);
    cache[(const void*)kern] = nb;
    return nb;
}

}  // namespace host
}  // namespace atos

struct atos_graph {
    atos::host::GraphRec r;
};
