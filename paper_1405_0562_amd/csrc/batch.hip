// Batched matching: many (document, table) jobs in one persistent launch.
//
// Every document is cut into pieces of P bytes.  A work unit is one piece of
// one job; units are numbered document by document, piece by piece, and the
// jobs of a document fastest, so that neighbouring lanes walk the same bytes
// through different tables.  Each unit is walked from the identity mapping
// through its table (Algorithm 5, Section 5.2, with the pieces as chunks) and
// leaves one D-SFA state.  A job's result is its start state followed through
// the mappings of its pieces in text order (the sequential reduction of
// Algorithm 5; any division of a document composes, Theorem 2 of Section 4.3).
//
// One kernel, k_batch: a grid of resident blocks stages the tables in LDS
// once (the class columns of all tables interleaved, so that the lanes
// walking one piece through different tables read neighbouring bytes, then
// every table's rows), then every wave walks its share of the work items
// (runs of 64 * K consecutive units, dealt to the waves in turn) on its own:
// no block barriers, so a wave that follows a chain of mappings delays only
// itself.  After the walk of an item:
//   * a job of one piece is finished by the lane that walked it;
//   * a job whose pieces all lie in the item is finished by the lane holding
//     its last piece, which reads the other pieces' states from the other
//     lanes' registers;
//   * for a job whose pieces lie in several items, the wave computes the
//     mapping of the job's pieces in this item for every start state
//     (reverse composition, Section 2.1), stores it and counts one arrival
//     on the job's counter; the wave whose arrival completes the job follows
//     the start state through the job's item mappings in order.
// Counters are reset by the arrival that completes them, so a workspace
// serves every launch of its plan and the launch can be captured in a graph
// and replayed.  The host plan is built once (sfa_batch_create) and uploaded
// once (sfa_batch_upload).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "device.h"
#include "internal.h"
#include "walk.h"

namespace {

constexpr uint32_t kTB = 256;
constexpr uint32_t kLdsBudget = 96 * 1024;

struct BTable {
    const uint8_t *img;     // stride-1 image: [classes u8[256] (2*class)] [rows u16 (row byte offsets)]
    const uint8_t *map;     // mapping rows, map_w bytes per entry
    const uint8_t *accept;  // u8[n_dfa]
    uint32_t img_bytes, row_bytes;
    uint32_t lds_off;       // LDS tables: byte offset of this table's rows in LDS
    uint32_t n_dfa, q0, map_w, pad0, pad1;
};

struct BDoc {
    uint64_t off, len;
    uint64_t unit_base;     // first unit of this document
    uint32_t np;            // pieces (an empty document has one empty piece)
    uint32_t m;             // jobs of this document
    uint32_t job_base;      // first job of this document (sorted order)
    uint32_t pad;
};

struct BJob {
    uint32_t doc, table, out_index;
    uint32_t gjob;          // index into the spanning-job list (jobs whose pieces lie in several items), or UINT32_MAX
};

struct BGroupJob {
    uint64_t gmap_base;     // first u32 of this job's item mappings (n_items x n_dfa)
    uint32_t job;
    uint32_t n_items;       // items holding pieces of the job: its arrivals
    uint32_t n_dfa, pad;
};

struct BatchArgs {
    const uint8_t *data;
    const BTable *tables;
    const BDoc *docs;
    const BJob *jobs;
    const BGroupJob *gjobs;
    uint32_t *jcnt;          // arrival counters of the spanning jobs
    uint32_t *gmaps;         // item mappings of the spanning jobs
    sfa_result *out;
    uint64_t n_units;
    uint32_t n_witems;       // work items: ceil(n_units / (64 * K)), one wave each
    uint32_t n_docs, n_jobs, n_gjobs, n_tables;
    uint32_t piece;
    uint32_t seg;            // lanes per leader segment: a power of two >= min(64, largest n_dfa)
    uint32_t lds_tables;     // 1: tables staged in LDS (class columns at 0, rows at each table's lds_off)
    uint32_t lds_bytes;      // staged bytes (multiple of 16; 0 without LDS tables)
    const uint8_t *lds_image;  // lds_tables: the LDS contents, contiguous
};

inline uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

}  // namespace

struct sfa_batch {
    uint32_t n_tables = 0, n_docs = 0, n_jobs = 0, n_gjobs = 0;
    uint32_t piece = 0, K = 1;
    uint32_t lds_tables = 0, lds_bytes = 0, seg = 1;
    uint64_t n_units = 0, n_items = 0, n_map_entries = 0;
    uint32_t num_cus = 0;
    int device = 0;
    // occupancy of the plan's kernel, filled at its first launch
    mutable const void *occ_fn = nullptr;
    mutable size_t occ_lds = 0;
    mutable int occ_per_cu = 1;
    // workspace layout: [reserved][tables][docs][jobs][spanning jobs][job
    // counters][LDS contents] are uploaded; [item mappings] are written by
    // the kernel
    uint64_t off_tables = 0, off_docs = 0, off_jobs = 0, off_gjobs = 0, off_jcnt = 0, off_lds = 0, off_gmaps = 0,
             total = 0;
    std::vector<uint8_t> blob;   // bytes [0, off_gmaps) of the workspace
};

namespace {

// Last document whose first unit is <= u (documents without units share the
// next document's base and are never selected).
__device__ __forceinline__ uint32_t find_doc(const BDoc *docs, uint32_t n_docs, uint64_t u) {
    uint32_t lo = 0, hi = n_docs;   // invariant: docs[lo].unit_base <= u, answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (docs[mid].unit_base <= u)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

template <typename MT>
__device__ __forceinline__ uint32_t map_entry(const uint8_t *map, uint32_t f, uint32_t n, uint32_t q) {
    return ((const MT *)map)[(size_t)f * n + q];
}

__device__ __forceinline__ uint32_t apply_map(const BTable &t, uint32_t f, uint32_t q) {
    return t.map_w == 1 ? map_entry<uint8_t>(t.map, f, t.n_dfa, q) : map_entry<uint16_t>(t.map, f, t.n_dfa, q);
}

// Item mappings are exchanged between blocks (on any XCD)
// with agent-scope loads and stores (coherent per access, the sc1 bit): a
// writer waits until its stores are acknowledged before it counts its
// arrival, and the arrival that completes a counter reads them afterwards.
// No L2-wide write-back or invalidation is needed, so the tables and input
// lines cached in the L2 stay there.
__device__ __forceinline__ void put_shared(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t get_shared(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The start state of job j followed through its item mappings in order
// (called by a whole wave, j uniform).  For n <= 64 the mappings are read 64 /
// n at a time per register (contiguous entries, coalesced), 16 registers per
// round trip, and the state is carried across them with lane reads.
__device__ __forceinline__ void compose_job(const BatchArgs &a, uint32_t j, uint32_t lane) {
    const BJob job = a.jobs[j];
    const BGroupJob gj = a.gjobs[job.gjob];
    const BTable tab = a.tables[job.table];
    const uint32_t n = gj.n_dfa, N = gj.n_items;
    const uint32_t *gm = a.gmaps + gj.gmap_base;
    uint32_t q = tab.q0;
    if (n <= 64) {
        const uint32_t mpr = 64 / n;           // mappings per register
        const uint32_t span = 16 * mpr;        // mappings per round trip
        for (uint32_t b0 = 0; b0 < N; b0 += span) {
            uint32_t v[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint32_t i = b0 + r * mpr + lane / n;
                v[r] = (lane < mpr * n && i < N) ? get_shared(&gm[(uint64_t)(b0 + r * mpr) * n + lane]) : 0u;
            }
#pragma unroll
            for (int r = 0; r < 16; ++r)
                for (uint32_t g = 0; g < mpr && b0 + r * mpr + g < N; ++g)
                    q = __builtin_amdgcn_readlane(v[r], g * n + q);
        }
    } else {
        for (uint32_t i = 0; i < N; ++i) q = get_shared(&gm[(uint64_t)i * n + q]);
    }
    if (lane == 0) {
        a.out[job.out_index].state = q;
        a.out[job.out_index].accept = tab.accept[q];
    }
}

template <int K, bool LDS>
__global__ __launch_bounds__(kTB) void k_batch(BatchArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    if constexpr (LDS) sfa_dev::copy16((uint4 *)smem, (const uint4 *)a.lds_image, a.lds_bytes / 16);
    __syncthreads();
    // From here every wave works on its own, on work items (64 * K
    // consecutive units) w, w + W, w + 2W, ... (W waves in the grid): no
    // shared item counter (same-address atomics serialise), and a wave that
    // follows a chain of mappings delays only itself.
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t W = gridDim.x * (kTB / 64);
    for (uint32_t item = blockIdx.x * (kTB / 64) + threadIdx.x / 64; item < a.n_witems; item += W) {
        // ---- walk this item's units: lane l walks units (item*K + k)*64 + l
        uint64_t pos[K], end[K], unit[K];
        uint32_t st[K], rb[K], tb[K], tc[K], jk[K], pc[K];
        const uint8_t *gt[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            unit[k] = ((uint64_t)item * K + k) * 64 + lane;
            pos[k] = end[k] = 0;
            st[k] = 0;
            rb[k] = 2;
            tb[k] = 0;
            tc[k] = 0;
            jk[k] = UINT32_MAX;
            pc[k] = 0;
            gt[k] = a.tables[0].img;
            if (unit[k] < a.n_units) {
                const uint32_t d = find_doc(a.docs, a.n_docs, unit[k]);
                const BDoc doc = a.docs[d];
                const uint64_t local = unit[k] - doc.unit_base;
                const uint64_t p = local / doc.m;
                const uint32_t slot = (uint32_t)(local - p * doc.m);
                jk[k] = doc.job_base + slot;
                pc[k] = (uint32_t)p;
                const uint32_t t = a.jobs[jk[k]].table;
                pos[k] = doc.off + min(doc.len, p * a.piece);
                end[k] = doc.off + min(doc.len, (p + 1) * (uint64_t)a.piece);
                rb[k] = a.tables[t].row_bytes;
                tb[k] = a.tables[t].lds_off;
                tc[k] = t;
                gt[k] = a.tables[t].img;
            }
        }
        auto step = [&](int k, uint32_t s, uint32_t b) -> uint32_t {
            if constexpr (LDS) {
                // class columns interleaved by table: the lanes walking one
                // piece through different tables read neighbouring bytes
                return sfa_rt::lds_u16(tb[k] + s + sfa_rt::lds_u8(b * a.n_tables + tc[k]));
            } else {
                const uint8_t *base = gt[k];
                return *(const uint16_t *)(base + 256 + s + base[b]);
            }
        };
        // head bytes up to 16-byte alignment, per unit
        uint32_t maxhead = 0, head[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            head[k] = (uint32_t)min<uint64_t>((16 - ((uintptr_t)(a.data + pos[k]) & 15)) & 15, end[k] - pos[k]);
            maxhead = max(maxhead, head[k]);
        }
        for (uint32_t i = 0; i < maxhead; ++i) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const bool act = i < head[k];
                const uint32_t b = act ? a.data[pos[k] + i] : 0u;
                const uint32_t t = step(k, st[k], b);
                st[k] = act ? t : st[k];
            }
        }
        uint64_t nb[K], maxnb = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            pos[k] += head[k];
            nb[k] = (end[k] - pos[k]) / 16;
            maxnb = max(maxnb, nb[k]);
        }
        // body: 16-byte loads, the next step's issued before this one is
        // walked; a unit past its last 16 bytes re-reads its first (discarded)
        auto load = [&](uint4 (&v)[K], uint64_t j) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint64_t addr = (j < nb[k]) ? pos[k] + 16 * j : pos[k];
                v[k] = (nb[k] > 0) ? *(const uint4 *)(a.data + addr) : make_uint4(0, 0, 0, 0);
            }
        };
        uint4 cur[K];
        if (maxnb) load(cur, 0);
        for (uint64_t j = 0; j < maxnb; ++j) {
            uint4 nxt[K];
            if (j + 1 < maxnb) load(nxt, j + 1);
            uint32_t t[K];
#pragma unroll
            for (int k = 0; k < K; ++k) t[k] = st[k];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const uint32_t w = i < 4 ? cur[k].x : i < 8 ? cur[k].y : i < 12 ? cur[k].z : cur[k].w;
                    t[k] = step(k, t[k], (w >> (8 * (i & 3))) & 255u);
                }
            }
#pragma unroll
            for (int k = 0; k < K; ++k) st[k] = (j < nb[k]) ? t[k] : st[k];
            if (j + 1 < maxnb) {
#pragma unroll
                for (int k = 0; k < K; ++k) cur[k] = nxt[k];
            }
        }
        // tail
#pragma unroll
        for (int k = 0; k < K; ++k) pos[k] += 16 * nb[k];
        for (uint32_t i = 0; i < 16; ++i) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const bool act = pos[k] + i < end[k];
                const uint32_t b = act ? a.data[pos[k] + i] : 0u;
                const uint32_t t = step(k, st[k], b);
                st[k] = act ? t : st[k];
            }
        }

        // ---- results.  Lane l's unit k is unit i0 + k * 64 + l.
        //  * a job of one piece: the lane that walked it finishes it;
        //  * a job whose pieces all lie in this item: the lane holding its
        //    last piece follows the start state through the pieces' states,
        //    read from the other lanes' registers;
        //  * a job that spans items: the lane holding its last piece in this
        //    item leads; the wave computes the mapping of the job's pieces in
        //    this item for every start state (reverse composition,
        //    Section 2.1), stores it and counts one arrival on the job's
        //    counter; the arrival that completes the job follows the start
        //    state through the job's item mappings in order.
        const uint64_t i0 = (uint64_t)item * K * 64, i1 = min(a.n_units, i0 + (uint64_t)K * 64);
        uint32_t sid[K], loc = 0, lead = 0;   // bit k: unit k composes (loc) or leads (lead)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            sid[k] = st[k] / rb[k];
            if (jk[k] == UINT32_MAX) continue;
            const BJob job = a.jobs[jk[k]];
            const BDoc doc = a.docs[job.doc];
            if (doc.np == 1) {
                const BTable tab = a.tables[job.table];
                const uint32_t q = apply_map(tab, sid[k], tab.q0);
                a.out[job.out_index].state = q;
                a.out[job.out_index].accept = tab.accept[q];
            } else if (job.gjob == UINT32_MAX) {
                if (pc[k] == doc.np - 1) loc |= 1u << k;
            } else if (pc[k] == doc.np - 1 || unit[k] + doc.m >= i1) {
                lead |= 1u << k;
            }
        }
        // the state id of unit i0 + off, from the lane that walked it (every
        // lane takes part: the reads are cross-lane permutes)
        auto state_at = [&](uint32_t off) __attribute__((always_inline)) -> uint32_t {
            const uint32_t src = off & 63u, reg = off >> 6;
            uint32_t v = 0;
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const uint32_t x = (uint32_t)__shfl((int)sid[r], (int)src, 64);
                v = (uint32_t)r == reg ? x : v;
            }
            return v;
        };
        if (__ballot(loc != 0)) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const bool mine = (loc >> k) & 1u;
                uint32_t q = 0, np = 0, m = 1, out_index = 0, f = 0;
                BTable tab{};
                if (mine) {
                    const BJob job = a.jobs[jk[k]];
                    const BDoc doc = a.docs[job.doc];
                    tab = a.tables[job.table];
                    out_index = job.out_index;
                    q = tab.q0;
                    np = doc.np;
                    m = doc.m;
                    f = (uint32_t)(doc.unit_base + (jk[k] - doc.job_base) - i0);   // first piece, in this item
                }
                for (uint32_t p = 0; __ballot(mine && p < np); ++p) {
                    const uint32_t v = state_at(mine ? f + p * m : lane);
                    if (mine && p < np) q = apply_map(tab, v, q);
                }
                if (mine) {
                    a.out[out_index].state = q;
                    a.out[out_index].accept = tab.accept[q];
                }
            }
        }
        if (__ballot(lead != 0)) {
            // leaders in segments of `seg` lanes (a power of two that holds
            // the largest start-state count, at most 64), 64 / seg at a time;
            // lane x of a segment follows start state x (x, x + 64, ... when
            // a table has more than 64 DFA states)
            const uint32_t seg = a.seg, per = 64 / seg, sl = lane / seg, x0 = lane % seg;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                uint64_t lm = __ballot((lead >> k) & 1u);
                while (lm) {
                    uint32_t my = 64;   // the lane of this segment's leader
                    for (uint32_t g = 0; g < per && lm; ++g) {
                        const uint32_t l = (uint32_t)__builtin_ctzll(lm);
                        lm &= lm - 1;
                        my = g == sl ? l : my;
                    }
                    const bool act = my < 64;
                    const uint32_t j = (uint32_t)__shfl((int)jk[k], (int)(act ? my : lane), 64);
                    const uint32_t pl = (uint32_t)__shfl((int)pc[k], (int)(act ? my : lane), 64);
                    uint32_t n = 0, pa = 0, m = 1, f = 0, slot = 0, n_arr = 0, gjob = 0;
                    uint64_t gbase = 0;
                    BTable tab{};
                    if (act) {
                        const BJob job = a.jobs[j];
                        const BDoc doc = a.docs[job.doc];
                        const BGroupJob gj = a.gjobs[job.gjob];
                        tab = a.tables[job.table];
                        n = gj.n_dfa;
                        m = doc.m;
                        const uint64_t first = doc.unit_base + (j - doc.job_base);
                        pa = i0 > first ? (uint32_t)((i0 - first + m - 1) / m) : 0u;   // first piece in this item
                        f = (uint32_t)(first + (uint64_t)pa * m - i0);
                        n_arr = gj.n_items;
                        slot = m < K * 64 ? item - (uint32_t)(first / (K * 64)) : pl;
                        gbase = gj.gmap_base + (uint64_t)slot * n;
                        gjob = job.gjob;
                    }
                    const uint32_t steps = act ? pl - pa + 1 : 0;
                    for (uint32_t xb = 0; __ballot(act && xb < n); xb += seg) {
                        uint32_t x = min(xb + x0, n ? n - 1 : 0u);
                        for (uint32_t i = 0; __ballot(i < steps); ++i) {
                            const uint32_t v = state_at(i < steps ? f + i * m : lane);
                            if (i < steps) x = apply_map(tab, v, x);
                        }
                        if (act && xb + x0 < n) put_shared(&a.gmaps[gbase + xb + x0], x);
                    }
                    __builtin_amdgcn_s_waitcnt(sfa_rt::kWaitVmcnt0);   // this lane's entries are acknowledged
                    // one arrival per segment; a segment's lanes all wrote before
                    // it (the wave runs in lockstep past the wait above)
                    uint32_t done = 0;
                    if (act && x0 == 0) {
                        uint32_t *cnt = &a.jcnt[gjob];
                        if (atomicAdd(cnt, 1u) == n_arr - 1) {
                            *cnt = 0;   // the job is complete: its counter starts over for the next launch
                            done = 1;
                        }
                    }
                    for (uint64_t dm = __ballot(done); dm; dm &= dm - 1) {
                        const uint32_t l = (uint32_t)__builtin_ctzll(dm);
                        compose_job(a, __builtin_amdgcn_readlane(j, l), lane);
                    }
                }
            }
        }
    }
}

template <int K, bool LDS>
hipError_t launch_batch(const sfa_batch *b, hipStream_t s, const BatchArgs &a, size_t lds) {
    auto fn = k_batch<K, LDS>;
    hipError_t e = sfa_rt::prepare_kernel((const void *)fn);
    if (e != hipSuccess) return e;
    // blocks per CU: queried once per plan (the kernel and its LDS size are
    // fixed by the plan), so a replayed or repeated launch does no host query
    if (b->occ_fn != (const void *)fn || b->occ_lds != lds) {
        int per_cu = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kTB, lds);
        if (e != hipSuccess) return e;
        b->occ_fn = (const void *)fn;
        b->occ_lds = lds;
        b->occ_per_cu = std::max(1, per_cu);
    }
    // every resident wave takes items in turn (the grid is never larger
    // than what fits at once, so no wave waits for a slot)
    const uint64_t resident = (uint64_t)b->occ_per_cu * std::max(1u, b->num_cus);
    const uint64_t grid = std::min<uint64_t>((a.n_witems + kTB / 64 - 1) / (kTB / 64), resident);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(kTB), lds, s, a);
    return hipGetLastError();
}

}  // namespace

extern "C" sfa_status sfa_batch_create(const sfa_table *const *tables, uint32_t n_tables, const uint64_t *doc_off,
                                       uint32_t n_docs, const uint32_t *jobs, uint32_t n_jobs,
                                       const sfa_batch_options *opts, sfa_batch **out) {
    if (!out) return sfa_fail(SFA_ERR_INVALID_ARG, "null out");
    *out = nullptr;
    if (!tables || n_tables == 0 || !doc_off || (n_jobs && !jobs))
        return sfa_fail(SFA_ERR_INVALID_ARG, "null or empty batch argument");
    const uint32_t piece = (opts && opts->piece_bytes) ? opts->piece_bytes : 4096;
    const uint32_t K = (opts && opts->units_per_lane) ? opts->units_per_lane : 2;
    if (piece < 16 || (piece & 15)) return sfa_fail(SFA_ERR_INVALID_ARG, "piece_bytes must be a multiple of 16");
    if (K != 1 && K != 2 && K != 4) return sfa_fail(SFA_ERR_INVALID_ARG, "units_per_lane must be 1, 2 or 4");
    if (opts && opts->reserved) return sfa_fail(SFA_ERR_INVALID_ARG, "sfa_batch_options.reserved must be 0");
    int dev = -1;
    for (uint32_t t = 0; t < n_tables; ++t) {
        const sfa_table *tb = tables[t];
        if (!tb) return sfa_fail(SFA_ERR_INVALID_ARG, "null table");
        if (tb->L.n_sfa == 0) return sfa_fail(SFA_ERR_NO_SFA, "batched matching needs D-SFA tables");
        if (!tb->L.img[0].present)
            return sfa_fail(SFA_ERR_INVALID_ARG, "table too large for batched matching (no stride-1 image)");
        if (t == 0) dev = tb->device;
        if (tb->device != dev) return sfa_fail(SFA_ERR_INVALID_ARG, "tables on different devices");
    }
    for (uint32_t d = 0; d < n_docs; ++d)
        if (doc_off[d + 1] < doc_off[d]) return sfa_fail(SFA_ERR_INVALID_ARG, "doc_off must be non-decreasing");
    for (uint32_t j = 0; j < n_jobs; ++j)
        if (jobs[2 * j] >= n_docs || jobs[2 * j + 1] >= n_tables)
            return sfa_fail(SFA_ERR_INVALID_ARG, "job references a missing document or table");
    sfa_batch *b = new (std::nothrow) sfa_batch();
    if (!b) return sfa_fail(SFA_ERR_HOST_ALLOC, "out of host memory");
    try {
        b->n_tables = n_tables;
        b->n_jobs = n_jobs;
        b->piece = piece;
        b->K = K;
        b->device = dev;
        // jobs sorted by document (stable), original index kept for the output
        std::vector<uint32_t> order(n_jobs);
        std::iota(order.begin(), order.end(), 0u);
        std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return jobs[2 * x] < jobs[2 * y]; });
        std::vector<BTable> bt(n_tables);
        // LDS layout: the class columns of all tables, byte b of table t at
        // b * n_tables + t (the lanes of one piece, one per table, read
        // neighbouring bytes), then every table's rows, 16-byte aligned
        uint64_t lds_off = (256ull * n_tables + 15) & ~15ull;
        for (uint32_t t = 0; t < n_tables; ++t) {
            const sfa_table *tb = tables[t];
            const Image &im = tb->L.img[0];
            bt[t].img = tb->d_base + im.off;
            bt[t].map = tb->d_base + tb->L.off_map;
            bt[t].accept = tb->d_base + tb->L.off_acc;
            bt[t].img_bytes = im.bytes;
            bt[t].row_bytes = im.row_bytes;
            bt[t].lds_off = (uint32_t)std::min<uint64_t>(lds_off, UINT32_MAX);
            bt[t].n_dfa = tb->L.n_dfa;
            bt[t].q0 = tb->L.q0;
            bt[t].map_w = tb->L.map_w;
            lds_off += ((uint64_t)im.bytes - 256 + 15) & ~15ull;
        }
        const bool force_global = opts && opts->force_global;
        b->lds_tables = (!force_global && lds_off <= kLdsBudget) ? 1 : 0;
        b->lds_bytes = b->lds_tables ? (uint32_t)lds_off : 0;
        // documents that have jobs, in document order
        const uint64_t IK = 64ull * K;   // units per work item
        std::vector<BDoc> docs;
        std::vector<BJob> bj(n_jobs);
        std::vector<BGroupJob> gj;
        uint64_t units = 0, gmap = 0;
        uint32_t max_dfa = 1;
        for (uint32_t i = 0; i < n_jobs;) {
            const uint32_t d = jobs[2 * order[i]];
            uint32_t e = i;
            while (e < n_jobs && jobs[2 * order[e]] == d) ++e;
            BDoc doc{};
            doc.off = doc_off[d];
            doc.len = doc_off[d + 1] - doc_off[d];
            doc.unit_base = units;
            doc.np = (uint32_t)std::max<uint64_t>(1, (doc.len + piece - 1) / piece);   // empty: one empty piece
            doc.m = e - i;
            doc.job_base = i;
            units += (uint64_t)doc.np * doc.m;
            const uint32_t di = (uint32_t)docs.size();
            for (uint32_t k = i; k < e; ++k) {
                const uint32_t t = jobs[2 * order[k] + 1];
                bj[k] = BJob{di, t, order[k], UINT32_MAX};
                const uint64_t first = doc.unit_base + (k - i);
                const uint64_t fi = first / IK, li = (first + (uint64_t)(doc.np - 1) * doc.m) / IK;
                if (fi != li) {
                    // pieces in several items: one mapping per item holding
                    // some of them (every item from the first to the last
                    // when pieces are less than an item apart, else one
                    // item per piece)
                    BGroupJob g{};
                    g.gmap_base = gmap;
                    g.job = k;
                    g.n_items = doc.m < IK ? (uint32_t)(li - fi + 1) : doc.np;
                    g.n_dfa = bt[t].n_dfa;
                    gmap += (uint64_t)g.n_items * g.n_dfa;
                    max_dfa = std::max(max_dfa, g.n_dfa);
                    bj[k].gjob = (uint32_t)gj.size();
                    gj.push_back(g);
                }
            }
            docs.push_back(doc);
            i = e;
        }
        if (gj.size() >= UINT32_MAX) throw std::bad_alloc();
        b->n_docs = (uint32_t)docs.size();
        b->n_gjobs = (uint32_t)gj.size();
        b->n_units = units;
        b->n_map_entries = gmap;
        b->n_items = (units + IK - 1) / IK;   // work items: 64 * K units, one wave each
        if (b->n_items >= UINT32_MAX) throw std::bad_alloc();
        b->seg = 1;
        while (b->seg < std::min(64u, max_dfa)) b->seg *= 2;
        b->num_cus = tables[0]->num_cus;
        uint64_t off = 256;   // [0, 256): reserved
        b->off_tables = off;
        off = align256(off + sizeof(BTable) * bt.size());
        b->off_docs = off;
        off = align256(off + sizeof(BDoc) * std::max<size_t>(1, docs.size()));
        b->off_jobs = off;
        off = align256(off + sizeof(BJob) * std::max<size_t>(1, bj.size()));
        b->off_gjobs = off;
        off = align256(off + sizeof(BGroupJob) * std::max<size_t>(1, gj.size()));
        b->off_jcnt = off;
        off = align256(off + 4 * std::max<size_t>(1, gj.size()));
        b->off_lds = off;
        off = align256(off + b->lds_bytes);
        b->off_gmaps = off;
        off = align256(off + 4 * std::max<uint64_t>(1, gmap));
        b->total = off;
        b->blob.assign(b->off_gmaps, 0);   // counters start at zero
        auto put = [&](uint64_t at, const void *src, size_t bytes) {
            if (bytes) std::memcpy(&b->blob[at], src, bytes);
        };
        put(b->off_tables, bt.data(), sizeof(BTable) * bt.size());
        put(b->off_docs, docs.data(), sizeof(BDoc) * docs.size());
        put(b->off_jobs, bj.data(), sizeof(BJob) * bj.size());
        put(b->off_gjobs, gj.data(), sizeof(BGroupJob) * gj.size());
        if (b->lds_tables)   // the LDS contents, from the tables' packed host images ([classes][rows])
            for (uint32_t t = 0; t < n_tables; ++t) {
                const Image &im = tables[t]->L.img[0];
                const uint8_t *src = tables[t]->image.data() + im.off;
                for (uint32_t c = 0; c < 256; ++c) b->blob[b->off_lds + (uint64_t)c * n_tables + t] = src[c];
                put(b->off_lds + bt[t].lds_off, src + 256, im.bytes - 256);
            }
    } catch (const std::bad_alloc &) {
        delete b;
        return sfa_fail(SFA_ERR_HOST_ALLOC, "out of host memory");
    }
    *out = b;
    return SFA_OK;
}

extern "C" sfa_status sfa_batch_get_info(const sfa_batch *b, sfa_batch_info *out) {
    if (!b || !out) return sfa_fail(SFA_ERR_INVALID_ARG, "null argument");
    std::memset(out, 0, sizeof(*out));
    out->n_jobs = b->n_jobs;
    out->n_docs = b->n_docs;
    out->n_units = b->n_units;
    out->n_item_map_entries = b->n_map_entries;
    out->piece_bytes = b->piece;
    out->units_per_lane = b->K;
    out->tables_in_lds = b->lds_tables;
    out->workspace_bytes = b->total;
    return SFA_OK;
}

extern "C" sfa_status sfa_batch_workspace_bytes(const sfa_batch *b, size_t *out_bytes) {
    if (!b || !out_bytes) return sfa_fail(SFA_ERR_INVALID_ARG, "null argument");
    *out_bytes = (size_t)b->total;
    return SFA_OK;
}

extern "C" sfa_status sfa_batch_upload(const sfa_batch *b, void *d_ws, size_t ws_bytes, void *stream) {
    if (!b || !d_ws) return sfa_fail(SFA_ERR_INVALID_ARG, "null argument");
    if (((uintptr_t)d_ws & 255) != 0) return sfa_fail(SFA_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < b->total) return sfa_fail(SFA_ERR_BUFFER_TOO_SMALL, "workspace smaller than sfa_batch_workspace_bytes");
    hipError_t e = hipMemcpyAsync(d_ws, b->blob.data(), b->blob.size(), hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e != hipSuccess) return sfa_fail(SFA_ERR_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    return SFA_OK;
}

extern "C" sfa_status sfa_match_batch(const sfa_batch *b, const uint8_t *d_data, void *d_ws, size_t ws_bytes,
                                    sfa_result *d_out, void *stream) {
    if (!b || !d_ws || (b->n_jobs && !d_out)) return sfa_fail(SFA_ERR_INVALID_ARG, "null argument");
    if (b->n_units && !d_data) return sfa_fail(SFA_ERR_INVALID_ARG, "null data");
    if (((uintptr_t)d_ws & 255) != 0) return sfa_fail(SFA_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < b->total) return sfa_fail(SFA_ERR_BUFFER_TOO_SMALL, "workspace smaller than sfa_batch_workspace_bytes");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
        return sfa_fail(SFA_ERR_INVALID_ARG, "batch tables were loaded on another device");
    uint8_t *ws = (uint8_t *)d_ws;
    BatchArgs a{};
    a.data = d_data;
    a.tables = (const BTable *)(ws + b->off_tables);
    a.docs = (const BDoc *)(ws + b->off_docs);
    a.jobs = (const BJob *)(ws + b->off_jobs);
    a.gjobs = (const BGroupJob *)(ws + b->off_gjobs);
    a.jcnt = (uint32_t *)(ws + b->off_jcnt);
    a.gmaps = (uint32_t *)(ws + b->off_gmaps);
    a.out = d_out;
    a.n_units = b->n_units;
    a.n_witems = (uint32_t)b->n_items;
    a.n_docs = b->n_docs;
    a.n_jobs = b->n_jobs;
    a.n_gjobs = b->n_gjobs;
    a.n_tables = b->n_tables;
    a.piece = b->piece;
    a.seg = b->seg;
    a.lds_tables = b->lds_tables;
    a.lds_bytes = b->lds_tables ? b->lds_bytes : 0;
    a.lds_image = ws + b->off_lds;
    hipStream_t s = (hipStream_t)stream;
    // LDS: the staged table images only
    const size_t lds = a.lds_bytes;
    hipError_t e;
    if (b->lds_tables) {
        if (b->K == 4) e = launch_batch<4, true>(b, s, a, lds);
        else if (b->K == 2) e = launch_batch<2, true>(b, s, a, lds);
        else e = launch_batch<1, true>(b, s, a, lds);
    } else {
        if (b->K == 4) e = launch_batch<4, false>(b, s, a, lds);
        else if (b->K == 2) e = launch_batch<2, false>(b, s, a, lds);
        else e = launch_batch<1, false>(b, s, a, lds);
    }
    if (e != hipSuccess) return sfa_fail(SFA_ERR_HIP, std::string("batch launch: ") + hipGetErrorString(e));
    return SFA_OK;
}

extern "C" void sfa_batch_free(sfa_batch *b) { delete b; }
