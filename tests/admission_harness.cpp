// Drives the serving daemon's host admission control (atos_admission.h) from
// commands on stdin, for tests/test_admission.py (CPU only):
//   I slots pools cap heap_base heap_bytes   initialise
//   A entries bytes                          admit -> "ok slot off" or "again"
//   R slot entries off bytes                 release -> "ok"
//   S                                        state -> "used u0 u1 ...", "free off bytes ..."
#include <iostream>
#include <sstream>
#include <string>

#include "atos_admission.h"

int main() {
    atos::host::Admission adm;
    std::string line;
    while (std::getline(std::cin, line)) {
        std::istringstream in(line);
        char op = 0;
        in >> op;
        if (op == 'I') {
            uint32_t slots = 0, pools = 0;
            uint64_t cap = 0;
            size_t base = 0, bytes = 0;
            in >> slots >> pools >> cap >> base >> bytes;
            adm.init(slots, pools, cap, base, bytes);
            std::cout << "ok\n";
        } else if (op == 'A') {
            uint64_t entries = 0;
            size_t bytes = 0, off = 0;
            uint32_t slot = 0;
            in >> entries >> bytes;
            if (adm.admit(entries, bytes, slot, off))
                std::cout << "ok " << slot << " " << off << "\n";
            else
                std::cout << "again\n";
        } else if (op == 'R') {
            uint32_t slot = 0;
            uint64_t entries = 0;
            size_t off = 0, bytes = 0;
            in >> slot >> entries >> off >> bytes;
            adm.release(slot, entries, off, bytes);
            std::cout << "ok\n";
        } else if (op == 'S') {
            std::cout << "used";
            for (uint64_t u : adm.pool_used) std::cout << " " << u;
            std::cout << "\nfree";
            for (const auto& kv : adm.heap.free) std::cout << " " << kv.first << " " << kv.second;
            std::cout << "\n";
        }
        std::cout.flush();
    }
    return 0;
}
