// Internal declarations shared by the host compiler and the HIP runtime.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "sfa.h"

// Host-side result of sfa_compile: the canonical minimal DFA over byte
// classes and, when built, its D-SFA.
struct sfa_compiled {
    uint32_t n_dfa = 0, n_sfa = 0, n_classes = 0, q0 = 0;
    uint32_t n_positions = 0, over_cap = 0;
    double dfa_seconds = 0, sfa_seconds = 0;
    uint8_t byte_class[256] = {};
    std::vector<uint32_t> dfa_next;   // [n_dfa * n_classes]
    std::vector<uint8_t> dfa_accept;  // [n_dfa]
    std::vector<uint32_t> sfa_next;   // [n_sfa * n_classes]
    std::vector<uint32_t> sfa_map;    // [n_sfa * n_dfa]
};

// Record a message for sfa_last_error() and return the status.
sfa_status sfa_fail(sfa_status st, const std::string &msg);
