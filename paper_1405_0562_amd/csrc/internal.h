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
    uint32_t n_positions = 0, over_cap = 0, lazy = 0;
    double dfa_seconds = 0, sfa_seconds = 0;
    uint8_t byte_class[256] = {};
    std::vector<uint32_t> dfa_next;   // [n_dfa * n_classes]
    std::vector<uint8_t> dfa_accept;  // [n_dfa]
    std::vector<uint32_t> sfa_next;   // [n_sfa * n_classes]
    std::vector<uint32_t> sfa_map;    // [n_sfa * n_dfa]
    // N-SFA (built from the position automaton): the "DFA" above is the
    // reachable subset automaton, each of its states is a set of NFA states
    uint32_t nsfa = 0, n_nfa = 0, words = 0;
    std::vector<uint64_t> nfa_sets;   // [n_dfa * words]
    std::vector<uint64_t> nfa_final;  // [words]
};

// Record a message for sfa_last_error() and return the status.
sfa_status sfa_fail(sfa_status st, const std::string &msg);

// A stride-S walk image, copied as one block into LDS by the walk kernel:
//   [pair-class table u8[65536] (S >= 2)] [byte-class table u8[256]]
//   [rows: n_sfa x (C^S (+ C if S >= 2)) u16 entries]
// Class and pair-class entries hold column offsets in bytes (2 * index).
// Entry values are row offsets in bytes (state id * row bytes), so one
// transition is a single LDS load at (current row offset + column * 2).
// Columns 0..C^S-1 hold delta_s applied to an S-byte word whose class digits
// c_0..c_{S-1} (first byte most significant, base C) form the column index;
// for S >= 2 the last C columns hold the single-byte transition (used for
// unaligned heads and short tails).
struct Image {
    uint32_t present = 0;
    uint32_t bytes = 0;       // total image bytes
    uint32_t row_bytes = 0;   // RS
    uint32_t one_off = 0;     // byte offset of the single-byte columns in a row
    uint64_t off = 0;         // offset in the device buffer
};

struct Layout {
    uint32_t n_dfa = 0, n_sfa = 0, C = 0, q0 = 0;
    uint32_t next_w = 0, map_w = 0;
    uint64_t off_cls = 0;    // u16[256]: cls[b] * next_w   (global-table walk)
    uint64_t off_dcls = 0;   // u16[256]: cls[b] * 2        (speculative kernel)
    uint64_t off_acc = 0;    // u8[n_dfa]
    uint64_t off_dnext = 0;  // u16[n_dfa * C]
    uint64_t off_next = 0;   // next_w bytes [n_sfa * C]: state ids (global-table walk)
    uint64_t off_map = 0;    // map_w bytes [n_sfa * n_dfa]
    uint64_t off_mul = 0;    // u8[n_sfa * n_sfa]: product table, id of f_a . f_b (when mul_bytes > 0)
    uint32_t mul_bytes = 0;  // 0: no product table (compositions go through the mappings)
    Image img[3];            // strides 1, 2, 4
    uint64_t total = 0;
    uint64_t next_bytes = 0;
    uint32_t hot_rows = 0;   // global-table walk: leading rows of sfa_next staged in LDS
    uint64_t off_himg = 0;   // global-table walk: hot image (u8 classes[256], (hot_rows + 1) x C u16 entries)
    uint32_t himg_bytes = 0;
    uint32_t renumbered = 0; // 1: D-SFA ids were renumbered by visit count
    uint32_t partial = 0;    // 1: on-the-fly D-SFA with unbuilt transitions (largest id of next_w)
    uint32_t vector_redo = 0; // 1: global walk re-walks cold words with vector loads (set by pack)
};

inline int stride_index(uint32_t S) { return S == 1 ? 0 : S == 2 ? 1 : S == 4 ? 2 : -1; }

// A loaded table: layout of the caller's device buffer plus the packed host image.
struct sfa_table {
    Layout L;
    uint8_t *d_base = nullptr;
    int device = 0;
    uint32_t lds_per_block = 0;
    uint32_t num_cus = 0;
    std::vector<uint8_t> image;
};
