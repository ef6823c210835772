// Device side of the single-stream matcher for gfx950: launch arguments,
// the ordered composition of chunk results (reverse composition, Section 2.1;
// Lemma 1 and Theorem 2, Section 4.3), and the walk kernels of Algorithm 5
// (Section 5.2).  The kernel templates are instantiated in translation units
// of their own (one per stride or table-entry width), so they compile in
// parallel; the host runtime reaches them through dispatch_shape and
// dispatch_global.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"
#include "internal.h"

namespace sfa_rt {


constexpr uint32_t kBlock = 256;             // threads per block of the walk kernels
constexpr uint32_t kGlobalBlock = 1024;      // threads per block of the global-table walk's wide default
constexpr uint32_t kGlobalSpecialBlock = 512; // its other default (short inputs, complete D-SFAs with vector re-walks)
constexpr uint32_t kLdsBlock = 512;          // default threads per block of the LDS walk
constexpr uint64_t kShortChunk = 4096;       // chunk bytes up to which the stride-4 walk uses 512 threads
constexpr uint32_t kSpecWaves = 4;           // waves (chunks) per speculative block
constexpr uint32_t kDefaultLdsBudget = 96 * 1024;
constexpr uint32_t kScratchLds = 16 * 1024;  // LDS for group mappings in the composition
constexpr uint32_t kMaxIds = 8 * kBlock;     // piece states per block (K * block threads <= 2048)
constexpr uint32_t kGlobalMaxClasses = 128;  // global-table walk: column byte offsets fit u8
constexpr uint32_t kPairTable = 65536;       // byte-pair class table entries (u8)
constexpr uint32_t kSpecStage = 16 * 1024;  // speculative blocks: LDS region for the grid composition
constexpr uint32_t kMulMax = 16 * 1024;      // product table bytes at most (u8 ids: n_sfa <= 128)
constexpr uint32_t kIdRun = 4096;            // product mode: blocks per level-1 run
constexpr uint64_t kWsHeader = 4096;         // workspace control words: [0] top level, [1 + r] level-1 run r
constexpr uint32_t kMaxRuns = kWsHeader / 4 - 1;
constexpr uint32_t kVectorRedo = 8;          // global walk: cold pieces of a wave above which the word is re-walked with vector loads
constexpr uint32_t kGroupPairsPerThread = 12; // (group, state) chains a thread follows together from global rows

inline uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// Byte-pair class table layout.  Entry h = b0 | b1 << 8 (b0 first in the
// text) sits at h with its bits 2..7 XORed with bits 0..5 of b1: the LDS
// bank of an entry then depends on both bytes, not on b0 alone (text over a
// small alphabet would otherwise put every lookup of a wave in a few banks).
// A permutation within each 256-entry block, so the table stays 64 KiB.
__host__ __device__ inline uint32_t pair_slot(uint32_t h) { return h ^ ((h >> 6) & 0xfcu); }
// Both pair slots of a 4-byte word at once: low half and high half of the result.
__host__ __device__ inline uint32_t pair_slots(uint32_t w) { return w ^ ((w >> 6) & 0x00fc00fcu); }


// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

using sfa_dev::copy16;

// LDS loads at a byte address of the block's dynamic LDS.  The walk
// kernels declare no static LDS, so their dynamic LDS starts at address 0
// (prepare_kernel checks this on the host before a kernel's first launch),
// and an address built from an integer needs no base: a row offset and a
// column then fold into one v_add_lshl_u32, and constant offsets into the
// load's offset field.
typedef const __attribute__((address_space(3))) uint8_t lds_u8_t;
typedef const __attribute__((address_space(3))) uint16_t lds_u16_t;
__device__ __forceinline__ uint32_t lds_u8(uint32_t addr) { return *(lds_u8_t *)(uintptr_t)addr; }
__device__ __forceinline__ uint32_t lds_u16(uint32_t addr) { return *(lds_u16_t *)(uintptr_t)addr; }

struct MatchArgs {
    const uint8_t *in;
    uint64_t n;
    uint64_t chunk_len;      // L >= ceil(n / n_chunks)
    uint32_t n_chunks;
    uint32_t n_dfa;
    uint32_t q0;
    uint32_t row_bytes;      // bytes per table row
    uint32_t one_off;        // LDS walk: byte offset of the single-byte columns
    uint32_t wide_mul;       // LDS walk, stride 4: C*C (first pair's weight in the column index)
    uint32_t img_bytes;      // LDS walk: image bytes; speculative: DFA table bytes
    uint32_t groups;         // G: groups per block in the block composition
    uint32_t groups1;        // G for a level-1 grid composition (one run of super_blocks blocks)
    uint32_t final_groups;   // G for the top grid composition
    uint32_t region_bytes;   // LDS bytes at offset 0 free once the walk is over (multiple of 16)
    uint32_t map_lds;        // 1: the mapping rows are copied into that region for the block composition
    uint32_t map_bytes;      // bytes of the mapping rows
    uint32_t map_stride;     // u16 entries per stored block or group mapping (n_dfa rounded up to 8)
    uint32_t super_blocks;   // blocks per level-1 run; n_super == 1: one level
    uint32_t n_super;        // level-1 runs (the top composition composes n_super mappings)
    uint32_t stage1;         // 1: level-1 compositions stage their block mappings in LDS
    uint32_t stage2;         // 1: the top composition stages its mappings in LDS
    uint32_t lanes_per_chunk;  // LPC: consecutive lanes sharing one chunk (walk kernels)
    uint32_t hot_rows;       // global-table walk: rows 0..hot_rows-1 staged in LDS
    uint32_t n_classes;      // global-table walk: C
    uint32_t cold;           // global-table walk: H, the cold row
    uint32_t mul_off;        // global-table walk: LDS offset of the product table (then the flag word)
    const uint8_t *gtab;     // global-table walk: D-SFA transitions, NT ids [n_sfa * C]
    const uint16_t *cls;     // speculative: u16[256] class column offsets
    const uint8_t *img;      // LDS image, hot image of the global walk, or u16 DFA table
    const uint8_t *map;      // mapping rows
    const uint8_t *accept;   // u8[n_dfa]
    uint32_t *counter;       // workspace control words: [0] top, [1 + r] level-1 run r
    uint16_t *block_maps;    // [gridDim.x * map_stride]
    uint16_t *group_maps;    // [n_super * map_stride] when n_super > 1
    const uint8_t *mul;      // product table u8[n_sfa * n_sfa] (product mode), else null
    uint32_t n_sfa;
    uint32_t mul_lds;        // LDS bytes of the product table copy (multiple of 16); 0: mapping mode
    uint32_t *block_ids;     // product mode: [gridDim.x] block products
    uint32_t *run_ids;       // product mode: [n_super] run products
    sfa_result *out;
    // partial (on-the-fly) D-SFA, global-table walk: a piece that reaches an
    // unbuilt transition parks on row cold + 1 and leaves a ParkRec
    uint32_t partial;
    struct ParkRec *park;    // [gridDim.x * K * TB], piece e of block b at b * K * TB + e
    const uint16_t *dnext;   // DFA transitions u16 [n_dfa * C] (class offsets in cls)
    uint32_t group_lds;      // global walk: the block composition's groups at LDS offset 0 (the freed region)
};

// A parked piece: it reached an unbuilt D-SFA transition at byte pos, in
// D-SFA state `state` (built); its bytes run to end.  When the mapping of
// `state` takes at most kParkVals distinct values, the piece's lane follows
// each of them through the DFA over bytes [pos, end) once, after its walk:
// vals[i] ends in res[i] (nvals of them; kParkMany: more values, every start
// state is followed in the composition instead).
constexpr uint32_t kParkVals = 4, kParkMany = 0xFFFFFFFFu;
struct ParkRec {
    uint64_t pos, end;
    uint32_t state, nvals;
    uint16_t vals[kParkVals], res[kParkVals];
    uint32_t pad[2];
};

// piece id of a parked piece among the block's piece ids
constexpr uint32_t kParkedId = 0xFFFFFFFFu;

// The mapping of parked piece e (of this block, E pieces per block) applied
// to x: x through the mapping of the state the piece stopped in (`map_at`),
// then through the DFA over the rest of the piece (the speculative walk of
// Algorithm 3, for the one start state x).
template <typename MapAt>
__device__ __forceinline__ uint32_t parked_apply(const MatchArgs &a, MapAt map_at, uint32_t E, uint32_t e, uint32_t x) {
    const ParkRec *r = a.park + (size_t)blockIdx.x * E + e;
    const uint64_t pos = __hip_atomic_load(&r->pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t end = __hip_atomic_load(&r->end, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t st = __hip_atomic_load(&r->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t nv = __hip_atomic_load(&r->nvals, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t y = map_at(st, x);
    if (nv != kParkMany) {
        // the piece's lane followed every value of the mapping: look y up
        const uint32_t *w = (const uint32_t *)r->vals;   // vals, then res: four u32 words
        uint32_t v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = __hip_atomic_load(w + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t out = y;
#pragma unroll
        for (uint32_t i = 0; i < kParkVals; ++i) {
            const uint32_t vi = (v[i / 2] >> (16 * (i & 1))) & 0xffffu;
            const uint32_t ri = (v[2 + i / 2] >> (16 * (i & 1))) & 0xffffu;
            out = (i < nv && vi == y) ? ri : out;
        }
        return out;
    }
    const uint8_t *dn = (const uint8_t *)a.dnext;
    const uint32_t rb = 2 * a.n_classes;
    for (uint64_t i = pos; i < end; ++i) y = *(const uint16_t *)(dn + y * rb + a.cls[a.in[i]]);
    return y;
}

// The lane of a parked piece completes its record: the piece's end, and the
// distinct values of its state's mapping (if at most kParkVals) each
// followed through the DFA over the rest of the piece, all together.
__device__ __forceinline__ void finish_parked(const MatchArgs &a, ParkRec *r, uint64_t end) {
    r->end = end;
    const uint64_t pos = r->pos;
    const uint32_t st = r->state, n = a.n_dfa;
    uint32_t v[kParkVals], nv = 0;
    for (uint32_t q = 0; q < n && nv <= kParkVals; ++q) {
        const uint32_t y = n <= 256 ? a.map[(size_t)st * n + q] : ((const uint16_t *)a.map)[(size_t)st * n + q];
        bool seen = false;
#pragma unroll
        for (uint32_t i = 0; i < kParkVals; ++i) seen |= i < nv && v[i] == y;
        if (!seen) {
            if (nv < kParkVals) {
#pragma unroll
                for (uint32_t i = 0; i < kParkVals; ++i) v[i] = i == nv ? y : v[i];
            }
            ++nv;
        }
    }
    if (nv > kParkVals) {
        r->nvals = kParkMany;
        return;
    }
    const uint8_t *dn = (const uint8_t *)a.dnext;
    const uint32_t rb = 2 * a.n_classes;
    uint32_t y[kParkVals];
#pragma unroll
    for (uint32_t i = 0; i < kParkVals; ++i) y[i] = i < nv ? v[i] : v[0];
    for (uint64_t i = pos; i < end; ++i) {
        const uint32_t c = a.cls[a.in[i]];
#pragma unroll
        for (uint32_t j = 0; j < kParkVals; ++j) y[j] = *(const uint16_t *)(dn + y[j] * rb + c);
    }
#pragma unroll
    for (uint32_t i = 0; i < kParkVals; ++i) {
        r->vals[i] = (uint16_t)(i < nv ? v[i] : 0);
        r->res[i] = (uint16_t)(i < nv ? y[i] : 0);
    }
    r->nvals = nv;
}

// Phase 1 of a composition: the elements 0..E-1 (mappings, in text order) are
// cut into G groups of R consecutive elements; for every (group g, start
// state q) pair, q is followed through the group's mappings, the earlier
// mapping first (reverse composition, f . g = g o f), and the end state is
// stored at out[g * n + q].  `get(e, x)` is mapping e applied to x.  P
// pairs per thread are followed together to hide load latency.
template <int P = 4, typename Get, typename Out>
__device__ __forceinline__ void follow_groups(Get get, uint32_t E, uint32_t R, uint32_t G, uint32_t n,
                                              Out *out) {
    const uint32_t items = G * n;
    for (uint32_t base = threadIdx.x; base < items; base += P * blockDim.x) {
        uint32_t it[P], x[P], e0[P], e1[P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
            it[i] = min(base + (uint32_t)i * blockDim.x, items - 1);
            const uint32_t g = it[i] / n;
            x[i] = it[i] - g * n;
            e0[i] = g * R;
            e1[i] = min(E, e0[i] + R);
        }
        for (uint32_t r = 0; r < R; ++r) {
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const uint32_t e = e0[i] + r;
                const uint32_t y = get(min(e, E - 1), x[i]);
                x[i] = e < e1[i] ? y : x[i];
            }
        }
#pragma unroll
        for (int i = 0; i < P; ++i)
            if (base + (uint32_t)i * blockDim.x < items) out[it[i]] = x[i];
    }
}

// Block composition: the block's E piece states (D-SFA ids in text order,
// s_ids) become the block mapping M[q], written to out_map (u16).  The
// mapping rows are read from LDS (copied over the walk-table region) when
// they fit.
template <typename MT, bool PARTIAL = false>
__device__ __forceinline__ void compose_block(const MatchArgs &a, uint8_t *smem, const uint32_t *s_ids, uint32_t E,
                              uint32_t *scratch, uint16_t *__restrict__ out_map) {
    const uint32_t n = a.n_dfa, G = a.groups, R = E / G;
    uint32_t *target = scratch;
    if (a.map_lds) {
        copy16((uint4 *)smem, (const uint4 *)a.map, (a.map_bytes + 15) / 16);
        __syncthreads();
        const MT *m = (const MT *)smem;
        auto map_at = [&](uint32_t id, uint32_t x) -> uint32_t { return m[id * n + x]; };
        auto get = [&](uint32_t e, uint32_t x) -> uint32_t {
            const uint32_t id = s_ids[e];
            if constexpr (PARTIAL)
                if (id == kParkedId) return parked_apply(a, map_at, E, e, x);
            return map_at(id, x);
        };
        if (G == 1) {
            follow_groups(get, E, R, 1, n, out_map);
            return;
        }
        follow_groups(get, E, R, G, n, target);
    } else {
        const MT *__restrict__ m = (const MT *)a.map;
        auto map_at = [&](uint32_t id, uint32_t x) -> uint32_t { return m[(size_t)id * n + x]; };
        auto get = [&](uint32_t e, uint32_t x) -> uint32_t {
            const uint32_t id = s_ids[e];
            if constexpr (PARTIAL)
                if (id == kParkedId) return parked_apply(a, map_at, E, e, x);
            return map_at(id, x);
        };
        if (G == 1) {
            follow_groups(get, E, R, 1, n, out_map);
            return;
        }
        // rows from global memory: more chains at once to cover the latency,
        // as many as the thread has pairs (up to kGroupPairsPerThread; a slot
        // past the last pair repeats it, loads included)
        const uint32_t per = (G * n + blockDim.x - 1) / blockDim.x;
        if (a.group_lds && per > 8)
            follow_groups<kGroupPairsPerThread>(get, E, R, G, n, target);
        else if (a.group_lds && per > 6)
            follow_groups<8>(get, E, R, G, n, target);
        else if (a.group_lds && per > 5)
            follow_groups<6>(get, E, R, G, n, target);
        else if (a.group_lds && per > 4)
            follow_groups<5>(get, E, R, G, n, target);
        else
            follow_groups(get, E, R, G, n, target);
    }
    __syncthreads();
    // phase 2: every start state through the G group mappings
    for (uint32_t q = threadIdx.x; q < n; q += blockDim.x) {
        uint32_t x = q;
        for (uint32_t g = 0; g < G; ++g) x = scratch[g * n + x];
        out_map[q] = (uint16_t)x;
    }
}

// Composition of `count` mappings in text order, `get(e, x)` being mapping e
// applied to x, in G groups.  With `out` the whole composed mapping is
// written there (u16); otherwise thread 0 returns its value at q0.
template <typename Get>
__device__ __forceinline__ uint32_t compose_rows(Get get, uint32_t count, uint32_t G, uint32_t n, uint32_t q0, uint32_t *scratch,
                                 uint16_t *out) {
    uint32_t x = q0;
    if (G == 1) {
        if (out) follow_groups(get, count, count, 1, n, out);
        else if (threadIdx.x == 0)
            for (uint32_t e = 0; e < count; ++e) x = get(e, x);
        return x;
    }
    follow_groups(get, count, (count + G - 1) / G, G, n, scratch);
    __syncthreads();
    if (out) {
        for (uint32_t q = threadIdx.x; q < n; q += blockDim.x) {
            uint32_t y = q;
            for (uint32_t g = 0; g < G; ++g) y = scratch[g * n + y];
            out[q] = (uint16_t)y;
        }
    } else if (threadIdx.x == 0) {
        for (uint32_t g = 0; g < G; ++g) x = scratch[g * n + x];
    }
    return x;
}

// Composes `count` stored mappings (u16 rows of a.map_stride entries, text
// order) starting at src; staged: the rows are first copied to LDS offset 0.
__device__ __forceinline__ uint32_t compose_stored(const MatchArgs &a, uint8_t *smem, uint32_t *scratch, const uint16_t *src,
                                   uint32_t count, uint32_t G, uint32_t staged, uint16_t *out) {
    const uint32_t n = a.n_dfa, ns = a.map_stride;
    if (staged) {
        copy16((uint4 *)smem, (const uint4 *)src, count * ns / 8);
        __syncthreads();
        const uint16_t *m = (const uint16_t *)smem;
        return compose_rows([&](uint32_t e, uint32_t y) -> uint32_t { return m[e * ns + y]; }, count, G, n, a.q0,
                            scratch, out);
    }
    const uint16_t *__restrict__ m = src;
    return compose_rows([&](uint32_t e, uint32_t y) -> uint32_t { return m[(size_t)e * ns + y]; }, count, G, n,
                        a.q0, scratch, out);
}

// s_waitcnt immediate that waits for vmcnt(0) only (gfx9 encoding: expcnt
// and lgkmcnt fields left at their maxima).
constexpr int kWaitVmcnt0 = 0x0F70;

// Counts this block's arrival at a counter that wraps back to zero after
// `count` arrivals (atomicInc limit).  True in the last block to arrive,
// which then sees every earlier block's stores.  Publication: every wave
// waits until its own stores are acknowledged by the L2, then one wave
// issues the agent-scope release (an L2 write-back) before the count; a
// release in every wave would write the L2 back once per wave.  The last
// block takes an agent-scope acquire.  s_last is one LDS word used for
// nothing else.
__device__ __forceinline__ bool arrive(uint32_t *counter, uint32_t count, uint32_t *s_last) {
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
    if (threadIdx.x < 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (threadIdx.x == 0) {
            const uint32_t prev = atomicInc(counter, count - 1);
            *s_last = (prev == count - 1) ? 1u : 0u;
        }
    }
    __syncthreads();
    if (!*s_last) return false;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

// Grid composition, after this block stored its mapping in block_maps.  One
// level: the last block to finish composes all block mappings in block order
// and applies the result to q0.  Two levels: the last block of each run of
// super_blocks consecutive blocks composes the run into a group mapping, and
// the last run to finish composes the group mappings.
__device__ __forceinline__ void block_done(const MatchArgs &a, uint8_t *smem, uint32_t *scratch, uint32_t *s_last) {
    const uint32_t B = gridDim.x;
    const uint16_t *top = a.block_maps;
    uint32_t top_count = B;
    if (a.n_super > 1) {
        const uint32_t r = blockIdx.x / a.super_blocks, first = r * a.super_blocks;
        const uint32_t count = min(a.super_blocks, B - first);
        if (!arrive(a.counter + 1 + r, count, s_last)) return;
        compose_stored(a, smem, scratch, a.block_maps + (size_t)first * a.map_stride, count, a.groups1, a.stage1,
                       a.group_maps + (size_t)r * a.map_stride);
        top = a.group_maps;
        top_count = a.n_super;
    }
    if (!arrive(a.counter, top_count, s_last)) return;
    const uint32_t x = compose_stored(a, smem, scratch, top, top_count, a.final_groups, a.stage2, nullptr);
    if (threadIdx.x == 0) {
        a.out->state = x;
        a.out->accept = a.accept[x];
    }
}

// ---- product mode: chunk results composed as D-SFA ids ------------------
// mul (LDS) is the n_sfa x n_sfa product table: mul[a * ns + b] is the id
// of f_a . f_b.  Id 0 is the identity f_I, so padding with 0 is harmless.

// Ordered product x_0 . x_1 . ... . x_63 of the ids held by a wave's lanes
// (lane order = text order).  Butterfly: at distance o the lane whose bit o
// is clear holds the left operand; every lane ends with the whole product.
__device__ __forceinline__ uint32_t wave_product(uint32_t x, const uint8_t *mul, uint32_t ns) {
    const uint32_t lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_xor((int)x, o, 64);
        const bool hi = (lane & (uint32_t)o) != 0;
        x = mul[(hi ? y : x) * ns + (hi ? x : y)];
    }
    return x;
}

// Ordered product of the ids held by the block's threads (thread order);
// the result is valid in thread 0.  s_w: one LDS word per wave.
__device__ __forceinline__ uint32_t block_product(uint32_t x, const uint8_t *mul, uint32_t ns, uint32_t *s_w) {
    x = wave_product(x, mul, ns);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x / 64] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        x = s_w[0];
        for (uint32_t w = 1; w < blockDim.x / 64; ++w) x = mul[x * ns + s_w[w]];
    }
    return x;
}

// Ordered product of ids[0 .. count) (global memory); thread t takes a run
// of consecutive ids.  Valid in thread 0.
__device__ __forceinline__ uint32_t product_of_ids(const uint32_t *ids, uint32_t count, const uint8_t *mul, uint32_t ns,
                                   uint32_t *s_w) {
    const uint32_t c = (count + blockDim.x - 1) / blockDim.x;
    const uint32_t b0 = min(count, threadIdx.x * c), b1 = min(count, b0 + c);
    uint32_t x = 0;
    for (uint32_t i = b0; i < b1; i += 8) {
        uint32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = ids[min(i + u, b1 - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u) x = i + u < b1 ? mul[x * ns + v[u]] : x;
    }
    return block_product(x, mul, ns, s_w);
}

// Grid step of product mode, after block_product (x valid in thread 0): as
// block_done, with one id per block or run instead of a mapping; the last
// block applies the final D-SFA state's mapping to q0.
__device__ __forceinline__ void finish_ids(const MatchArgs &a, uint32_t x, const uint8_t *mul, uint32_t *s_w, uint32_t *s_last) {
    const uint32_t B = gridDim.x, ns = a.n_sfa;
    if (threadIdx.x == 0) a.block_ids[blockIdx.x] = x;
    const uint32_t *top = a.block_ids;
    uint32_t top_count = B;
    if (a.n_super > 1) {
        const uint32_t r = blockIdx.x / a.super_blocks, first = r * a.super_blocks;
        const uint32_t count = min(a.super_blocks, B - first);
        if (!arrive(a.counter + 1 + r, count, s_last)) return;
        const uint32_t y = product_of_ids(a.block_ids + first, count, mul, ns, s_w);
        if (threadIdx.x == 0) a.run_ids[r] = y;
        top = a.run_ids;
        top_count = a.n_super;
    }
    if (!arrive(a.counter, top_count, s_last)) return;
    const uint32_t f = product_of_ids(top, top_count, mul, ns, s_w);
    if (threadIdx.x == 0) {
        const size_t at = (size_t)f * a.n_dfa + a.q0;
        const uint32_t q = a.n_dfa <= 256 ? a.map[at] : ((const uint16_t *)a.map)[at];
        a.out->state = q;
        a.out->accept = a.accept[q];
    }
}

__device__ __forceinline__ uint32_t word_of(const uint4 &v, int d) {
    return d == 0 ? v.x : d == 1 ? v.y : d == 2 ? v.z : v.w;
}

// Chunk bounds of this lane and its K pieces.  LPC consecutive lanes share a
// chunk: the chunk is cut into LPC * K pieces whose lengths are multiples of
// Q (so every piece starts at the same alignment) and lane part j of the
// chunk walks pieces j*K .. j*K + K - 1, i.e. piece order is text order.
template <int K, int Q, int TB>
__device__ __forceinline__ void lane_pieces(const MatchArgs &a, uint64_t &c0, uint64_t &c1, uint64_t *pos,
                                            uint64_t *end) {
    const uint64_t lane = (uint64_t)blockIdx.x * TB + threadIdx.x;
    const uint32_t lpc = a.lanes_per_chunk;
    const uint64_t chunk = lane / lpc;
    const uint32_t part = (uint32_t)(lane - chunk * lpc);
    // chunk c covers [b(c), b(c + 1)): b(0) = 0, b(c) = c * L - s, b(p) = n.
    // With L a multiple of 16, s = the input's misalignment puts every chunk
    // after the first on a 16-byte boundary (any split gives the same
    // result, Theorem 2 in Section 4.3)
    const uint64_t L = a.chunk_len;
    const uint64_t s = (L & 15) ? 0 : (uint64_t)((uintptr_t)a.in & 15);
    auto bound = [&](uint64_t c) -> uint64_t {
        return c == 0 ? 0 : c >= a.n_chunks ? a.n : min(a.n, c * L - s);
    };
    c0 = chunk < a.n_chunks ? bound(chunk) : a.n;
    c1 = chunk < a.n_chunks ? bound(chunk + 1) : a.n;
    const uint64_t len = c1 - c0;
    const uint64_t np = (uint64_t)lpc * K;
    const uint64_t piece = (((len + np - 1) / np) + Q - 1) / Q * Q;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        pos[k] = min(c1, c0 + ((uint64_t)part * K + k) * piece);
        end[k] = min(c1, pos[k] + piece);
    }
}

// LDS walk kernel, stride S (bytes per transition lookup), K pieces per lane,
// G bytes of each piece loaded per step, loads issued D - 1 steps ahead.  Lane l of block b owns chunk
// c = b*256 + l; its K piece states (in text order) join the block
// composition, then the grid composition.
template <int S, int K, int G, int D, int TB>
__global__ __launch_bounds__(TB) void k_sfa_lds(MatchArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    constexpr uint32_t CLS = (S >= 2) ? kPairTable : 0u;   // byte-class table
    constexpr uint32_t TAB = CLS + 256;                     // rows
    const uint32_t img = (a.img_bytes + 15) & ~15u;
    uint8_t *s_mul = smem + img;                            // product table (product mode)
    uint32_t *s_ids = (uint32_t *)(smem + img + a.mul_lds);
    uint32_t *s_flag = s_ids + K * TB;
    uint32_t *s_scr = s_flag + 4;
    uint64_t c0, c1, pos[K], end[K];
    lane_pieces<K, G, TB>(a, c0, c1, pos, end);
    // head: single bytes up to 16-byte alignment (the same for all pieces);
    // body[k]: where piece k's 16-byte aligned G-byte groups start
    const uint32_t head = c1 > c0 ? (uint32_t)((16 - ((uintptr_t)(a.in + pos[0]) & 15)) & 15) : 0u;
    uint64_t body[K], nb[K], maxnb = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        body[k] = min(end[k], pos[k] + head);
        nb[k] = (end[k] - body[k]) / G;
        maxnb = max(maxnb, nb[k]);
    }
    // ring of D load buffers: the loads of step j + D - 1 are issued before
    // step j is walked.  Piece 0 is the longest, so a piece past its last
    // group re-reads piece 0's first group (discarded).
    constexpr int V = G / 16;
    uint4 buf[D][K][V];
    // With a 2-deep ring the compiler would spread a step's loads over the
    // walk of the previous step; the 16-byte loads that share a 128-byte line
    // then reach the L2 microseconds apart and the line is fetched again
    // after an eviction (measured: 1.19x the input bytes).  Scheduling
    // barriers keep them together.
    auto issue = [&](uint4 (&dst)[K][V], uint64_t step) {
        if constexpr (D == 2) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint64_t base = (step < nb[k]) ? body[k] + (uint64_t)G * step : body[0];
#pragma unroll
            for (int v = 0; v < V; ++v) dst[k][v] = *(const uint4 *)(a.in + base + 16 * v);
        }
        if constexpr (D == 2) __builtin_amdgcn_sched_barrier(0);
    };
    // the first loads go out before the table is staged, so their latency
    // overlaps the staging
#pragma unroll
    for (int d = 0; d < D - 1; ++d)
        if ((uint64_t)d < maxnb) issue(buf[d], d);

    copy16((uint4 *)smem, (const uint4 *)a.img, img / 16, (blockIdx.x * 613u) % (img / 16));
    if (a.mul_lds) copy16((uint4 *)s_mul, (const uint4 *)a.mul, a.mul_lds / 16);
    __syncthreads();

    const uint32_t one = a.one_off, wide = a.wide_mul;
    auto row = [&](uint32_t off) -> uint32_t { return lds_u16(TAB + off); };
    // one byte: f <- delta_s[f, class(b)]
    auto step1 = [&](uint32_t st, uint32_t b) -> uint32_t { return row(st + one + lds_u8(CLS + b)); };

    uint32_t st[K];
#pragma unroll
    for (int k = 0; k < K; ++k) st[k] = 0;     // f_I

    if (c1 > c0) {
        for (uint32_t i = 0; i < head; ++i) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const bool act = pos[k] < end[k];
                const uint32_t t = step1(st[k], a.in[act ? pos[k] : c0]);
                st[k] = act ? t : st[k];
                pos[k] += act ? 1 : 0;
            }
        }
        if (maxnb) {
            auto walk = [&](const uint4 (&cur)[K][V], uint64_t step) {
                uint32_t t[K];
#pragma unroll
                for (int k = 0; k < K; ++k) t[k] = st[k];
#pragma unroll
                for (int v = 0; v < V; ++v) {
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        if constexpr (S == 1) {
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                uint32_t c[K];
#pragma unroll
                                for (int k = 0; k < K; ++k) c[k] = lds_u8(CLS + ((word_of(cur[k][v], d) >> (8 * i)) & 255u));
#pragma unroll
                                for (int k = 0; k < K; ++k) t[k] = row(t[k] + c[k]);
                            }
                        } else if constexpr (S == 2) {
                            uint32_t p0[K], p1[K];
#pragma unroll
                            for (int k = 0; k < K; ++k) {
                                const uint32_t w = pair_slots(word_of(cur[k][v], d));
                                p0[k] = lds_u8(w & 0xffffu);
                                p1[k] = lds_u8(w >> 16);
                            }
#pragma unroll
                            for (int k = 0; k < K; ++k) t[k] = row(t[k] + p0[k]);
#pragma unroll
                            for (int k = 0; k < K; ++k) t[k] = row(t[k] + p1[k]);
                        } else {
                            uint32_t p0[K], p1[K];
#pragma unroll
                            for (int k = 0; k < K; ++k) {
                                const uint32_t w = pair_slots(word_of(cur[k][v], d));
                                p0[k] = lds_u8(w & 0xffffu);
                                p1[k] = lds_u8(w >> 16);
                            }
#pragma unroll
                            for (int k = 0; k < K; ++k) t[k] = row(__umul24(p0[k], wide) + p1[k] + t[k]);
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < K; ++k) st[k] = (step < nb[k]) ? t[k] : st[k];
            };
            uint64_t j = 0;
            // steady state: every issued step exists, no bounds checks
            for (; j + 2 * D - 1 <= maxnb; j += D) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    issue(buf[(d + D - 1) % D], j + d + D - 1);
                    walk(buf[d], j + d);
                }
            }
            // last steps
            for (; j < maxnb; j += D) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    if (j + d < maxnb) {
                        if (j + d + D - 1 < maxnb) issue(buf[(d + D - 1) % D], j + d + D - 1);
                        walk(buf[d], j + d);
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < K; ++k) pos[k] += (uint64_t)G * nb[k];
        }
        // tail: fewer than G bytes per piece
        uint32_t maxtail = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) maxtail = max(maxtail, (uint32_t)(end[k] - pos[k]));
        for (uint32_t i = 0; i < maxtail; ++i) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const bool act = pos[k] < end[k];
                const uint32_t t = step1(st[k], a.in[act ? pos[k] : c0]);
                st[k] = act ? t : st[k];
                pos[k] += act ? 1 : 0;
            }
        }
    }
    const uint32_t rs = a.row_bytes;
    if (a.mul_lds) {
        uint32_t x = st[0] / rs;
#pragma unroll
        for (int k = 1; k < K; ++k) x = s_mul[x * a.n_sfa + st[k] / rs];
        finish_ids(a, block_product(x, s_mul, a.n_sfa, s_scr), s_mul, s_scr, s_flag);
        return;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) s_ids[threadIdx.x * K + k] = st[k] / rs;
    __syncthreads();   // the walk is over: the image region may be reused
    const uint32_t E = K * TB;
    uint16_t *bmap = a.block_maps + (size_t)blockIdx.x * a.map_stride;
    if (a.n_dfa <= 256)
        compose_block<uint8_t>(a, smem, s_ids, E, s_scr, bmap);
    else
        compose_block<uint16_t>(a, smem, s_ids, E, s_scr, bmap);
    block_done(a, smem, s_scr, s_flag);
}

// Global-table walk, for D-SFAs whose walk image does not fit in LDS
// (stride 1, at most 128 byte classes).  The loader renumbers the states so
// that the most visited come first and builds a hot image of rows 0..H-1
// plus one "cold" row H:
//   [2 * class of each byte, u8[256]] [H + 1 rows of C u16 entries]
// A row entry is the target u when u < H and H otherwise, and every entry of
// the cold row is H, so one transition is one LDS load at u * 2C + 2 * class,
// and a piece that steps onto a cold state stays on the cold row.  Pieces
// walk four bytes (one word) at a time this way; a piece that ends the word
// on the cold row walks the word again through the global table (ids of
// width NT, n_sfa x C entries), one lane at a time, with scalar loads: those
// are counted apart from the vector loads of the input ring, which complete
// in order, so a vector load would also wait for the input in flight.  While
// its state is cold, a piece keeps t = H and the state's id in cid.  The
// input is loaded as in the LDS walk: G bytes of each piece per step, loads
// issued D - 1 steps ahead (D = 1: the rolling ring described below).
//
// VEC: when more than kVectorRedo pieces of a wave end a word cold (tables
// whose visited states do not fit LDS), they re-walk it all at once with
// vector loads instead.  PARTIAL (on-the-fly D-SFA, the on-the-fly remark of
// Section 5.1): an unbuilt transition reads as the largest id of NT; the
// piece records where it stopped (ParkRec), moves to the parking row H + 1,
// and its mapping is completed after the walk (finish_parked) and in the
// block composition (parked_apply).
//
// LDS: [0, R) the hot image during the walk; once every wave has finished
// its walk, the piece ids and the composition scratch take the end of that
// region ([region_bytes, R)) and [0, region_bytes) is free for staging;
// [R, R + mul_lds) the product table (product mode); then the flag word.
template <int K, int G, int D, typename NT, int TB, bool PARTIAL, bool VEC>
__global__ __launch_bounds__(TB) void k_sfa_global(MatchArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    constexpr uint32_t ROWS = 256;                          // rows follow the class table
    const uint32_t img = (a.img_bytes + 15) & ~15u;
    uint8_t *s_mul = smem + a.mul_off;                      // product table (product mode)
    uint32_t *s_ids = (uint32_t *)(smem + a.region_bytes);  // after the walk
    uint32_t *s_scr = s_ids + K * TB;
    uint32_t *s_flag = (uint32_t *)(smem + a.mul_off + a.mul_lds);
    const uint32_t C = a.n_classes, H = a.hot_rows, cold = a.cold, RB = 2 * C;
    // partial D-SFA: a piece parks on row cold + 1 (its entries lead back to
    // it) once the scalar walk finds an unbuilt transition; never reached
    // otherwise (hot entries are at most cold)
    const uint32_t parked = cold + 1;
    constexpr uint32_t kUnbuilt = (uint32_t)(NT)~0u;

    uint64_t c0, c1, pos[K], end[K];
    lane_pieces<K, G, TB>(a, c0, c1, pos, end);
    const uint32_t head = c1 > c0 ? (uint32_t)((16 - ((uintptr_t)(a.in + pos[0]) & 15)) & 15) : 0u;
    // piece k's whole G-byte groups start `body[k]` bytes after c0 (a chunk
    // is shorter than 4 GiB); 32-bit offsets keep the walk's registers few
    const uint8_t *const cin = a.in + c0;
    uint32_t body[K], nb[K], maxnb = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint64_t b0 = min(end[k], pos[k] + head);
        body[k] = (uint32_t)(b0 - c0);
        nb[k] = (uint32_t)((end[k] - b0) / G);
        maxnb = max(maxnb, nb[k]);
    }
    // D >= 2: a ring of D steps of G bytes per piece, the loads of step j + D
    // - 1 issued before step j is walked.  D == 1: a rolling ring of three
    // half-line slots (G / 2 bytes) per piece: line j occupies two slots, and
    // once its first half is walked the whole of line j + 1 is loaded into
    // that slot and the spare one, so every line is requested whole (a line
    // read in two visits may leave the L2 in between) with 1.5 lines of
    // registers per piece instead of 2.
    constexpr int V = (D == 1 ? G / 2 : G) / 16;   // uint4 per ring slot
    constexpr int SLOTS = D == 1 ? 3 : D;
    uint4 buf[SLOTS][K][V];
    // loads of G bytes of step `step` into dst (D >= 2), or of line `step`
    // into the slots h0 (first half) and h1 (second half) (D == 1)
    auto issue = [&](uint4 (&dst)[K][V], uint32_t step) __attribute__((always_inline)) {
        if constexpr (D == 2) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t base = (step < nb[k]) ? body[k] + G * (uint32_t)step : body[0];
#pragma unroll
            for (int v = 0; v < V; ++v) dst[k][v] = *(const uint4 *)(cin + base + 16 * v);
        }
        if constexpr (D == 2) __builtin_amdgcn_sched_barrier(0);
    };
    auto issue_line = [&](uint4 (&h0)[K][V], uint4 (&h1)[K][V], uint32_t line) __attribute__((always_inline)) {
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t base = (line < nb[k]) ? body[k] + G * (uint32_t)line : body[0];
#pragma unroll
            for (int v = 0; v < V; ++v) h0[k][v] = *(const uint4 *)(cin + base + 16 * v);
#pragma unroll
            for (int v = 0; v < V; ++v) h1[k][v] = *(const uint4 *)(cin + base + G / 2 + 16 * v);
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    if constexpr (D == 1) {
        if (maxnb) issue_line(buf[0], buf[1], 0);
    } else {
#pragma unroll
        for (int d = 0; d < D - 1; ++d)
            if ((uint32_t)d < maxnb) issue(buf[d], d);
    }

    copy16((uint4 *)smem, (const uint4 *)a.img, img / 16, (blockIdx.x * 613u) % (img / 16));
    if (a.mul_lds) copy16((uint4 *)s_mul, (const uint4 *)a.mul, a.mul_lds / 16);
    __syncthreads();

    const uint8_t *__restrict__ tab = a.gtab;
    auto cls = [&](uint32_t b) __attribute__((always_inline)) -> uint32_t { return lds_u8(b); };
    auto row = [&](uint32_t u, uint32_t c2) __attribute__((always_inline)) -> uint32_t {
        return lds_u16(ROWS + __umul24(u, RB) + c2);
    };
    // Scalar walk through the global table from state s over the doubled
    // classes c2[b .. nc-1]; returns the new t and sets id to the new state.
    // At an unbuilt transition (partial D-SFA) it stops: returns the parking
    // row, id = the state before byte `at`, the byte's index.
    auto redo = [&](uint64_t s, const uint32_t *c2, int b, int nc, uint32_t &id, int &at_byte)
        __attribute__((always_inline)) -> uint32_t {
        for (int i = b; i < nc; ++i) {
            const uint64_t at = (s * C + (c2[i] >> 1)) * sizeof(NT);
            const uint32_t w = *(const __attribute__((address_space(4))) uint32_t *)(tab + (at & ~3ull));
            const uint32_t u = (w >> (8 * (uint32_t)(at & 3))) & kUnbuilt;
            if constexpr (PARTIAL) {
                if (u == kUnbuilt) {
                    id = (uint32_t)s;
                    at_byte = i;
                    return parked;
                }
            }
            s = u;
        }
        id = (uint32_t)s;
        return s < H ? (uint32_t)s : cold;
    };
    // park record of this lane's piece k: the byte at pos, in state id
    auto park_at = [&](int k, uint64_t pos, uint32_t id) __attribute__((always_inline)) {
        ParkRec *r = a.park + ((size_t)blockIdx.x * TB + threadIdx.x) * K + k;
        r->pos = pos;
        r->state = id;
    };
    // Four bytes of every piece (doubled classes c[i][k]): LDS walk, then the
    // pieces that ended on the cold row walk the whole word again from its
    // start (a fixed chain of four scalar loads: measured faster than a
    // shorter chain of run-time length from the last hot state).
    auto word = [&](uint32_t (&t)[K], uint32_t (&cid)[K], const uint32_t (&c)[4][K], uint32_t boff)
        __attribute__((always_inline)) {
        uint32_t t0[K];
#pragma unroll
        for (int k = 0; k < K; ++k) t0[k] = t[k];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int k = 0; k < K; ++k) t[k] = row(t[k], c[i][k]);
        uint64_t any = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) any |= __ballot(t[k] == cold);
        if (any) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                uint64_t m = __ballot(t[k] == cold);
                if (VEC && __builtin_popcountll(m) > kVectorRedo) {
                    // many pieces left the hot rows (a table whose visited
                    // states do not fit LDS): each walks its word again with
                    // vector loads, all at once; the wait for them also waits
                    // for the input loads in flight, which costs less than
                    // that many scalar chains one after another
                    if (t[k] == cold) {
                        uint64_t s = t0[k] == cold ? cid[k] : t0[k];
                        int at = -1;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            if (at < 0) {
                                const uint32_t u = *(const NT *)(tab + (s * C + (c[i][k] >> 1)) * sizeof(NT));
                                if (PARTIAL && u == kUnbuilt)
                                    at = i;
                                else
                                    s = u;
                            }
                        }
                        if (PARTIAL && at >= 0) {
                            park_at(k, (uint64_t)(cin - a.in) + body[k] + boff + (uint32_t)at, (uint32_t)s);
                            t[k] = parked;
                        } else {
                            t[k] = s < H ? (uint32_t)s : cold;
                        }
                        cid[k] = (uint32_t)s;
                    }
                    m = 0;
                }
                for (; m; m &= m - 1) {
                    const uint32_t l = (uint32_t)__builtin_ctzll(m);
                    uint32_t cl[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) cl[i] = __builtin_amdgcn_readlane(c[i][k], l);
                    const uint32_t s0 = __builtin_amdgcn_readlane(t0[k], l);
                    const uint64_t s = s0 == cold ? __builtin_amdgcn_readlane(cid[k], l) : s0;
                    uint32_t id;
                    int at = 0;
                    const uint32_t v = redo(s, cl, 0, 4, id, at);
                    const bool mine = __lane_id() == l;
                    if constexpr (PARTIAL)
                        if (v == parked && mine) park_at(k, (uint64_t)(cin - a.in) + body[k] + boff + (uint32_t)at, id);
                    t[k] = mine ? v : t[k];
                    cid[k] = mine ? id : cid[k];
                }
            }
        }
    };

    uint32_t st[K], sid[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        st[k] = H ? 0u : cold;     // f_I is id 0
        sid[k] = 0;
    }
    // single bytes (unaligned heads, short tails) of the pieces still inside
    auto singles = [&](uint32_t count) __attribute__((always_inline)) {
        for (uint32_t i = 0; i < count; ++i) {
            bool act[K];
            uint32_t c[K], nt[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                act[k] = pos[k] < end[k];
                c[k] = cls(a.in[act[k] ? pos[k] : c0]);
                nt[k] = row(st[k], c[k]);
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                for (uint64_t m = __ballot(act[k] && nt[k] == cold); m; m &= m - 1) {
                    const uint32_t l = (uint32_t)__builtin_ctzll(m);
                    const uint32_t cl = __builtin_amdgcn_readlane(c[k], l);
                    const uint32_t sl = __builtin_amdgcn_readlane(st[k], l);
                    const uint64_t s = sl == cold ? __builtin_amdgcn_readlane(sid[k], l) : sl;
                    uint32_t id;
                    int at = 0;
                    const uint32_t v = redo(s, &cl, 0, 1, id, at);
                    const bool mine = __lane_id() == l;
                    if constexpr (PARTIAL)
                        if (v == parked && mine) park_at(k, pos[k], id);
                    nt[k] = mine ? v : nt[k];
                    sid[k] = mine ? id : sid[k];
                }
                st[k] = act[k] ? nt[k] : st[k];
                pos[k] += act[k] ? 1 : 0;
            }
        }
    };
    if (c1 > c0) {
        singles(head);
        if (maxnb) {
            auto classes = [&](uint32_t (&c)[4][K], const uint4 (&cur)[K][V], int w) __attribute__((always_inline)) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int k = 0; k < K; ++k) c[i][k] = cls((word_of(cur[k][w / 4], w % 4) >> (8 * i)) & 255u);
            };
            // cur holds bytes [boff, boff + 16 V) of every piece's body
            auto walk = [&](const uint4 (&cur)[K][V], uint32_t step_no, uint32_t boff) __attribute__((always_inline)) {
                uint32_t t[K], id[K];
#pragma unroll
                for (int k = 0; k < K; ++k) t[k] = st[k], id[k] = sid[k];
                // the class columns of the next word are read while this word
                // is walked, unless the registers are short (the rolling ring
                // with four pieces, or with two in 1024-thread blocks: there
                // the prefetch costs spills, 1.68 against 1.65 ms on 4 GiB of
                // keyword text)
                constexpr bool ahead = !(D == 1 && (K >= 4 || TB >= 1024));
                uint32_t cc[4][K];
                classes(cc, cur, 0);
#pragma unroll
                for (int w = 0; w < 4 * V; ++w) {
                    if constexpr (ahead) {
                        uint32_t cn[4][K];
                        if (w + 1 < 4 * V) classes(cn, cur, w + 1);
                        word(t, id, cc, boff + 4 * w);
                        if (w + 1 < 4 * V) {
#pragma unroll
                            for (int i = 0; i < 4; ++i)
#pragma unroll
                                for (int k = 0; k < K; ++k) cc[i][k] = cn[i][k];
                        }
                    } else {
                        if (w) classes(cc, cur, w);
                        word(t, id, cc, boff + 4 * w);
                    }
                }
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const bool in = step_no < nb[k];   // a piece past its last step walked a stand-in
                    st[k] = in ? t[k] : st[k];
                    sid[k] = in ? id[k] : sid[k];
                }
            };
            uint32_t j = 0;
            if constexpr (D == 1) {
                // lines j (slots 0, 1) and j + 1 (slots 0, 2)
                for (; j + 2 <= maxnb; j += 2) {
                    walk(buf[0], j, G * j);
                    issue_line(buf[0], buf[2], j + 1);
                    walk(buf[1], j, G * j + G / 2);
                    walk(buf[0], j + 1, G * (j + 1));
                    if (j + 2 < maxnb) issue_line(buf[0], buf[1], j + 2);
                    walk(buf[2], j + 1, G * (j + 1) + G / 2);
                }
                if (j < maxnb) {
                    walk(buf[0], j, G * j);
                    walk(buf[1], j, G * j + G / 2);
                }
            } else {
                for (; j + 2 * D - 1 <= maxnb; j += D) {
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        issue(buf[(d + D - 1) % D], j + d + D - 1);
                        walk(buf[d], j + d, G * (j + d));
                    }
                }
                for (; j < maxnb; j += D) {
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        if (j + d < maxnb) {
                            if (j + d + D - 1 < maxnb) issue(buf[(d + D - 1) % D], j + d + D - 1);
                            walk(buf[d], j + d, G * (j + d));
                        }
                    }
                }
            }
        }
        // tail: fewer than G bytes per piece (the piece bounds are computed
        // again rather than kept live through the walk)
        lane_pieces<K, G, TB>(a, c0, c1, pos, end);
#pragma unroll
        for (int k = 0; k < K; ++k) pos[k] = c0 + body[k] + (uint64_t)G * nb[k];
        uint32_t maxtail = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) maxtail = max(maxtail, (uint32_t)(end[k] - pos[k]));
        singles(maxtail);
    }
    // D-SFA ids of the piece states (a parked piece: kParkedId, its record
    // completed with the piece's end); every wave is done with the hot image
    // before its region takes the ids and the composition scratch
    uint32_t ids[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        ids[k] = st[k] == cold ? sid[k] : st[k];
        if constexpr (PARTIAL) {
            if (st[k] == parked) {
                ids[k] = kParkedId;
                finish_parked(a, a.park + ((size_t)blockIdx.x * TB + threadIdx.x) * K + k, end[k]);
            }
        }
    }
    __syncthreads();
    if (a.mul_lds) {
        uint32_t x = ids[0];
#pragma unroll
        for (int k = 1; k < K; ++k) x = s_mul[x * a.n_sfa + ids[k]];
        finish_ids(a, block_product(x, s_mul, a.n_sfa, s_scr), s_mul, s_scr, s_flag);
        return;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) s_ids[threadIdx.x * K + k] = ids[k];
    __syncthreads();
    const uint32_t E = K * TB;
    uint16_t *bmap = a.block_maps + (size_t)blockIdx.x * a.map_stride;
    // mapping rows in global memory: the groups take the freed hot-image region
    uint32_t *gscr = a.group_lds ? (uint32_t *)smem : s_scr;
    if (a.n_dfa <= 256)
        compose_block<uint8_t, PARTIAL>(a, smem, s_ids, E, gscr, bmap);
    else
        compose_block<uint16_t, PARTIAL>(a, smem, s_ids, E, gscr, bmap);
    block_done(a, smem, s_scr, s_flag);
}

// ---------------------------------------------------------------------------
// host-side launch
// ---------------------------------------------------------------------------
// Supported (pieces K, load bytes G, prefetch depth D, block threads TB)
// shapes of the LDS walk.  K * G * D bounds the load buffers in registers.
#define SFA_LDS_SHAPES(X) \
    X(1, 64, 2, 256) X(1, 128, 2, 256) X(1, 128, 4, 256) X(2, 64, 2, 256) X(2, 64, 4, 256) \
    X(2, 128, 2, 256) X(2, 128, 3, 256) X(2, 128, 4, 256) X(3, 128, 3, 256) X(4, 64, 2, 256) X(8, 32, 2, 256) \
    X(1, 64, 2, 512) X(1, 128, 2, 512) X(1, 128, 3, 512) X(1, 128, 4, 512) X(2, 64, 2, 512) X(2, 64, 4, 512) \
    X(2, 128, 2, 512) X(2, 128, 3, 512) X(4, 32, 2, 512) X(4, 64, 2, 512) \
    X(1, 32, 2, 1024) X(1, 64, 2, 1024) X(1, 128, 2, 1024) X(2, 32, 2, 1024) X(2, 64, 2, 1024)

// Supported (pieces K, load bytes G, prefetch depth D, block threads TB)
// shapes of the global-table walk; each keeps its load ring in registers.
// 128-byte steps read every input line whole (shorter steps read a line in
// several visits, between which it may leave the L2).
#define SFA_GLOBAL_SHAPES(X) \
    X(1, 64, 2, 256) X(2, 64, 2, 256) X(4, 32, 2, 256) X(4, 64, 2, 256) \
    X(1, 128, 2, 256) X(2, 128, 2, 256) X(4, 128, 2, 256) \
    X(1, 64, 2, 512) X(2, 64, 2, 512) X(4, 32, 2, 512) X(4, 64, 2, 512) \
    X(1, 128, 2, 512) X(2, 128, 2, 512) X(2, 128, 3, 512) \
    X(2, 128, 1, 512) X(3, 128, 1, 512) X(4, 128, 1, 512) \
    X(1, 64, 2, 1024) X(2, 64, 2, 1024) X(1, 128, 2, 1024) X(2, 128, 1, 1024)

// Shapes of the global-table walk for a partial (on-the-fly) D-SFA or a
// table whose walk often leaves the hot rows (vector re-walks): the default
// plans and the shapes they fall back to for short chunks.
#define SFA_SPECIAL_SHAPES(X) X(4, 128, 1, 512) X(2, 128, 1, 512) X(1, 64, 2, 512) X(2, 128, 1, 1024)

// Once per kernel and device (runtime.hip): checks that the kernel has no
// static LDS (its dynamic LDS starts at address 0, which lds_u8/lds_u16
// assume) and allows it the device's whole LDS as dynamic LDS.
hipError_t prepare_kernel(const void *fn);

template <typename F>
hipError_t launch(F fn, uint32_t blocks, uint32_t threads, size_t lds, hipStream_t s, const MatchArgs &a) {
    hipError_t e = prepare_kernel((const void *)fn);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

// Launch of the LDS walk k_sfa_lds<S, K, G, D, TB> for a supported shape
// (SFA_LDS_SHAPES); hipErrorInvalidValue for any other.  Instantiated for
// S = 1, 2, 4 in walk_lds_s1.hip, walk_lds_s2.hip, walk_lds_s4.hip.
template <int S>
hipError_t dispatch_shape(uint32_t K, uint32_t G, uint32_t D, uint32_t TB, uint32_t blocks, size_t lds, hipStream_t s,
                          const MatchArgs &a) {
#define SFA_SHAPE_LAUNCH(k, g, d, tb) \
    if (K == k && G == g && D == d && TB == tb) return launch(k_sfa_lds<S, k, g, d, tb>, blocks, tb, lds, s, a);
    SFA_LDS_SHAPES(SFA_SHAPE_LAUNCH)
#undef SFA_SHAPE_LAUNCH
    return hipErrorInvalidValue;
}

// Launch of the global-table walk k_sfa_global<K, G, D, NT, TB> for a
// supported shape (SFA_GLOBAL_SHAPES).  Instantiated for NT = u8, u16, u32
// in walk_global_u8.hip, walk_global_u16.hip, walk_global_u32.hip.
template <typename NT>
hipError_t dispatch_global(uint32_t K, uint32_t G, uint32_t D, uint32_t TB, uint32_t blocks, size_t lds,
                           hipStream_t s, const MatchArgs &a) {
#define SFA_SHAPE_LAUNCH(k, g, d, tb) \
    if (K == k && G == g && D == d && TB == tb) return launch(k_sfa_global<k, g, d, NT, tb, false, false>, blocks, tb, lds, s, a);
    SFA_GLOBAL_SHAPES(SFA_SHAPE_LAUNCH)
#undef SFA_SHAPE_LAUNCH
    return hipErrorInvalidValue;
}

// The same for a partial D-SFA and/or vector re-walks (SFA_SPECIAL_SHAPES),
// instantiated for the three id widths in walk_partial.hip (partial) and
// walk_vector.hip (complete tables with vector re-walks).
template <typename NT, bool PARTIAL, bool VEC>
hipError_t dispatch_special(uint32_t K, uint32_t G, uint32_t D, uint32_t TB, uint32_t blocks, size_t lds,
                            hipStream_t s, const MatchArgs &a) {
#define SFA_SHAPE_LAUNCH(k, g, d, tb) \
    if (K == k && G == g && D == d && TB == tb) \
        return launch(k_sfa_global<k, g, d, NT, tb, PARTIAL, VEC>, blocks, tb, lds, s, a);
    SFA_SPECIAL_SHAPES(SFA_SHAPE_LAUNCH)
#undef SFA_SHAPE_LAUNCH
    return hipErrorInvalidValue;
}

#define SFA_DISPATCH_SHAPE(S) \
    template hipError_t dispatch_shape<S>(uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, size_t, hipStream_t, \
                                          const MatchArgs &)
#define SFA_DISPATCH_GLOBAL(NT) \
    template hipError_t dispatch_global<NT>(uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, size_t, hipStream_t, \
                                            const MatchArgs &)
extern SFA_DISPATCH_SHAPE(1);
extern SFA_DISPATCH_SHAPE(2);
extern SFA_DISPATCH_SHAPE(4);
extern SFA_DISPATCH_GLOBAL(uint8_t);
extern SFA_DISPATCH_GLOBAL(uint16_t);
extern SFA_DISPATCH_GLOBAL(uint32_t);
#define SFA_DISPATCH_SPECIAL(NT, P, V) \
    template hipError_t dispatch_special<NT, P, V>(uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, size_t, \
                                                   hipStream_t, const MatchArgs &)
extern SFA_DISPATCH_SPECIAL(uint8_t, true, false);
extern SFA_DISPATCH_SPECIAL(uint16_t, true, false);
extern SFA_DISPATCH_SPECIAL(uint32_t, true, false);
extern SFA_DISPATCH_SPECIAL(uint8_t, true, true);
extern SFA_DISPATCH_SPECIAL(uint16_t, true, true);
extern SFA_DISPATCH_SPECIAL(uint32_t, true, true);
extern SFA_DISPATCH_SPECIAL(uint8_t, false, true);
extern SFA_DISPATCH_SPECIAL(uint16_t, false, true);
extern SFA_DISPATCH_SPECIAL(uint32_t, false, true);

}  // namespace sfa_rt
