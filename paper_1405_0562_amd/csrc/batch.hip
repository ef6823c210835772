// Batched matching: many (document, table) jobs in one launch sequence.
//
// Every document is cut into pieces of P bytes.  A work unit is one piece of
// one job; units are numbered document by document, piece by piece, and the
// jobs of a document fastest, so that neighbouring lanes walk the same bytes
// through different tables.  Each unit is walked from the identity mapping
// through its table (Algorithm 5, Section 5.2, with the pieces as chunks) and
// leaves one D-SFA state.  A job's result is its start state followed through
// the mappings of its pieces in text order (the sequential reduction of
// Algorithm 5); jobs with more than `group` pieces first compose groups of
// pieces for every start state (reverse composition, Section 2.1), so the
// final chain has at most ceil(pieces / group) steps.
//
// Launches: k_batch_walk -> k_batch_groups (only if some job needs groups)
// -> k_batch_compose.  The host plan is built once (sfa_batch_create) and
// uploaded once (sfa_batch_upload); sfa_match_batch only launches kernels, so
// it can be captured in a graph and replayed.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "device.h"
#include "internal.h"

namespace {

constexpr uint32_t kTB = 256;
constexpr uint32_t kLdsBudget = 96 * 1024;

struct BTable {
    const uint8_t *img;     // stride-1 image: [classes u8[256] (2*class)] [rows u16 (row byte offsets)]
    const uint8_t *map;     // mapping rows, map_w bytes per entry
    const uint8_t *accept;  // u8[n_dfa]
    uint32_t img_bytes, row_bytes, lds_off, n_dfa, q0, map_w, pad0, pad1;
};

struct BDoc {
    uint64_t off, len;
    uint64_t unit_base;     // first unit of this document
    uint32_t np;            // pieces
    uint32_t m;             // jobs of this document
    uint32_t job_base;      // first job of this document (sorted order)
    uint32_t pad;
};

struct BJob {
    uint32_t doc, table, out_index, gjob;   // gjob: index into the group-job list, or UINT32_MAX
};

struct BGroupJob {
    uint64_t item_base;     // first (group, state) item of this job
    uint64_t gmap_base;     // first u32 of this job's group mappings
    uint32_t job, n_groups, n_dfa, pad;
};

struct BatchArgs {
    const uint8_t *data;
    const BTable *tables;
    const BDoc *docs;
    const BJob *jobs;
    const BGroupJob *gjobs;
    uint32_t *unit_state;
    uint32_t *gmaps;
    sfa_result *out;
    uint64_t n_units;
    uint64_t n_items;
    uint32_t n_docs, n_jobs, n_gjobs, n_tables;
    uint32_t piece, group;
    uint32_t lds_tables;     // 1: table images staged in LDS at lds_off
    uint32_t lds_bytes;
    const uint8_t *lds_image;  // lds_tables: all staged images, contiguous (lds_bytes, multiple of 16)
};

inline uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

}  // namespace

struct sfa_batch {
    uint32_t n_tables = 0, n_docs = 0, n_jobs = 0, n_gjobs = 0;
    uint32_t piece = 0, group = 0, K = 1;
    uint32_t lds_tables = 0, lds_bytes = 0;
    uint64_t n_units = 0, n_items = 0;
    int device = 0;
    // workspace layout
    uint64_t off_tables = 0, off_docs = 0, off_jobs = 0, off_gjobs = 0, off_lds = 0, off_units = 0, off_gmaps = 0,
             total = 0;
    std::vector<uint8_t> blob;   // bytes [off_tables, off_units) of the workspace
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

// Walk kernel: lane t of block b walks units (b*K + k)*256 + t, k < K.
template <int K, bool LDS>
__global__ __launch_bounds__(kTB) void k_batch_walk(BatchArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    if constexpr (LDS) {
        sfa_dev::copy16((uint4 *)smem, (const uint4 *)a.lds_image, a.lds_bytes / 16);
        __syncthreads();
    }
    uint64_t pos[K], end[K], unit[K];
    uint32_t st[K], rb[K], tb[K];   // state (row byte offset), row bytes, table base (LDS offset)
    const uint8_t *gt[K];           // table base in global memory
#pragma unroll
    for (int k = 0; k < K; ++k) {
        unit[k] = ((uint64_t)blockIdx.x * K + k) * kTB + threadIdx.x;
        pos[k] = end[k] = 0;
        st[k] = 0;
        rb[k] = 2;
        tb[k] = 0;
        gt[k] = a.tables[0].img;
        if (unit[k] < a.n_units) {
            const uint32_t d = find_doc(a.docs, a.n_docs, unit[k]);
            const BDoc doc = a.docs[d];
            const uint64_t local = unit[k] - doc.unit_base;
            const uint64_t p = local / doc.m;
            const uint32_t slot = (uint32_t)(local - p * doc.m);
            const uint32_t t = a.jobs[doc.job_base + slot].table;
            pos[k] = doc.off + p * a.piece;
            end[k] = doc.off + min(doc.len, (p + 1) * (uint64_t)a.piece);
            rb[k] = a.tables[t].row_bytes;
            tb[k] = a.tables[t].lds_off;
            gt[k] = a.tables[t].img;
        }
    }
    auto step = [&](int k, uint32_t s, uint32_t b) -> uint32_t {
        if constexpr (LDS) {
            const uint8_t *base = smem + tb[k];
            return *(const uint16_t *)(base + 256 + s + base[b]);
        } else {
            const uint8_t *base = gt[k];
            return *(const uint16_t *)(base + 256 + s + base[b]);
        }
    };
    // head bytes up to 16-byte alignment, per unit
    uint32_t maxhead = 0;
    uint32_t head[K];
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
    // body: 16-byte loads; a unit past its groups re-reads its first group (discarded)
    for (uint64_t j = 0; j < maxnb; ++j) {
        uint4 v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint64_t addr = (j < nb[k]) ? pos[k] + 16 * j : pos[k];
            v[k] = (nb[k] > 0) ? *(const uint4 *)(a.data + addr) : make_uint4(0, 0, 0, 0);
        }
        uint32_t t[K];
#pragma unroll
        for (int k = 0; k < K; ++k) t[k] = st[k];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t w = i < 4 ? v[k].x : i < 8 ? v[k].y : i < 12 ? v[k].z : v[k].w;
                t[k] = step(k, t[k], (w >> (8 * (i & 3))) & 255u);
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) st[k] = (j < nb[k]) ? t[k] : st[k];
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
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (unit[k] < a.n_units) a.unit_state[unit[k]] = st[k] / rb[k];
}

template <typename MT>
__device__ __forceinline__ uint32_t map_entry(const uint8_t *map, uint32_t f, uint32_t n, uint32_t q) {
    return ((const MT *)map)[(size_t)f * n + q];
}

__device__ __forceinline__ uint32_t apply_map(const BTable &t, uint32_t f, uint32_t q) {
    return t.map_w == 1 ? map_entry<uint8_t>(t.map, f, t.n_dfa, q) : map_entry<uint16_t>(t.map, f, t.n_dfa, q);
}

__device__ __forceinline__ uint64_t unit_of(const BDoc &d, uint32_t slot, uint64_t p) {
    return d.unit_base + p * d.m + slot;
}

// Group mappings of long jobs: item (job, group g, start state x) follows x
// through the mappings of pieces [g*group, min(np, (g+1)*group)).
__global__ __launch_bounds__(kTB) void k_batch_groups(BatchArgs a) {
    const uint64_t item = (uint64_t)blockIdx.x * kTB + threadIdx.x;
    if (item >= a.n_items) return;
    uint32_t lo = 0, hi = a.n_gjobs;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a.gjobs[mid].item_base <= item)
            lo = mid;
        else
            hi = mid;
    }
    const BGroupJob gj = a.gjobs[lo];
    const uint64_t local = item - gj.item_base;
    const uint32_t g = (uint32_t)(local / gj.n_dfa), x0 = (uint32_t)(local - (uint64_t)g * gj.n_dfa);
    const BJob job = a.jobs[gj.job];
    const BDoc doc = a.docs[job.doc];
    const BTable tab = a.tables[job.table];
    const uint32_t slot = gj.job - doc.job_base;
    const uint64_t p0 = (uint64_t)g * a.group, p1 = min<uint64_t>(doc.np, p0 + a.group);
    uint32_t x = x0;
    for (uint64_t p = p0; p < p1; ++p) x = apply_map(tab, a.unit_state[unit_of(doc, slot, p)], x);
    a.gmaps[gj.gmap_base + local] = x;
}

// One thread per job: the start state through the job's pieces (or groups).
__global__ __launch_bounds__(kTB) void k_batch_compose(BatchArgs a) {
    const uint32_t j = blockIdx.x * kTB + threadIdx.x;
    if (j >= a.n_jobs) return;
    const BJob job = a.jobs[j];
    const BDoc doc = a.docs[job.doc];
    const BTable tab = a.tables[job.table];
    const uint32_t slot = j - doc.job_base;
    uint32_t q = tab.q0;
    if (job.gjob == UINT32_MAX) {
        for (uint64_t p = 0; p < doc.np; ++p) q = apply_map(tab, a.unit_state[unit_of(doc, slot, p)], q);
    } else {
        const BGroupJob gj = a.gjobs[job.gjob];
        for (uint32_t g = 0; g < gj.n_groups; ++g) q = a.gmaps[gj.gmap_base + (uint64_t)g * gj.n_dfa + q];
    }
    a.out[job.out_index].state = q;
    a.out[job.out_index].accept = tab.accept[q];
}

template <typename F>
hipError_t launch(F fn, uint64_t blocks, size_t lds, hipStream_t s, const BatchArgs &a) {
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(fn, dim3((uint32_t)blocks), dim3(kTB), lds, s, a);
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
    const uint32_t group = (opts && opts->group_pieces) ? opts->group_pieces : 32;
    const uint32_t K = (opts && opts->units_per_lane) ? opts->units_per_lane : 2;
    if (piece < 16 || (piece & 15)) return sfa_fail(SFA_ERR_INVALID_ARG, "piece_bytes must be a multiple of 16");
    if (K != 1 && K != 2 && K != 4) return sfa_fail(SFA_ERR_INVALID_ARG, "units_per_lane must be 1, 2 or 4");
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
        b->group = group;
        b->K = K;
        b->device = dev;
        // jobs sorted by document (stable), original index kept for the output
        std::vector<uint32_t> order(n_jobs);
        std::iota(order.begin(), order.end(), 0u);
        std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return jobs[2 * x] < jobs[2 * y]; });
        std::vector<BTable> bt(n_tables);
        uint32_t lds_off = 0;
        for (uint32_t t = 0; t < n_tables; ++t) {
            const sfa_table *tb = tables[t];
            const Image &im = tb->L.img[0];
            bt[t].img = tb->d_base + im.off;
            bt[t].map = tb->d_base + tb->L.off_map;
            bt[t].accept = tb->d_base + tb->L.off_acc;
            bt[t].img_bytes = im.bytes;
            bt[t].row_bytes = im.row_bytes;
            bt[t].lds_off = lds_off;
            bt[t].n_dfa = tb->L.n_dfa;
            bt[t].q0 = tb->L.q0;
            bt[t].map_w = tb->L.map_w;
            lds_off += (im.bytes + 15) & ~15u;
        }
        const bool force_global = opts && opts->force_global;
        b->lds_tables = (!force_global && lds_off <= kLdsBudget) ? 1 : 0;
        b->lds_bytes = b->lds_tables ? lds_off : 0;
        // documents that have jobs, in document order
        std::vector<BDoc> docs;
        std::vector<BJob> bj(n_jobs);
        std::vector<BGroupJob> gj;
        uint64_t units = 0, items = 0, gmap = 0;
        for (uint32_t i = 0; i < n_jobs;) {
            const uint32_t d = jobs[2 * order[i]];
            uint32_t e = i;
            while (e < n_jobs && jobs[2 * order[e]] == d) ++e;
            BDoc doc{};
            doc.off = doc_off[d];
            doc.len = doc_off[d + 1] - doc_off[d];
            doc.unit_base = units;
            doc.np = (uint32_t)((doc.len + piece - 1) / piece);
            doc.m = e - i;
            doc.job_base = i;
            units += (uint64_t)doc.np * doc.m;
            const uint32_t di = (uint32_t)docs.size();
            for (uint32_t k = i; k < e; ++k) {
                const uint32_t t = jobs[2 * order[k] + 1];
                bj[k] = BJob{di, t, order[k], UINT32_MAX};
                if (doc.np > group) {
                    BGroupJob g{};
                    g.item_base = items;
                    g.gmap_base = gmap;
                    g.job = k;
                    g.n_groups = (doc.np + group - 1) / group;
                    g.n_dfa = bt[t].n_dfa;
                    items += (uint64_t)g.n_groups * g.n_dfa;
                    gmap += (uint64_t)g.n_groups * g.n_dfa;
                    bj[k].gjob = (uint32_t)gj.size();
                    gj.push_back(g);
                }
            }
            docs.push_back(doc);
            i = e;
        }
        b->n_docs = (uint32_t)docs.size();
        b->n_gjobs = (uint32_t)gj.size();
        b->n_units = units;
        b->n_items = items;
        uint64_t off = 256;
        b->off_tables = off;
        off = align256(off + sizeof(BTable) * bt.size());
        b->off_docs = off;
        off = align256(off + sizeof(BDoc) * std::max<size_t>(1, docs.size()));
        b->off_jobs = off;
        off = align256(off + sizeof(BJob) * std::max<size_t>(1, bj.size()));
        b->off_gjobs = off;
        off = align256(off + sizeof(BGroupJob) * std::max<size_t>(1, gj.size()));
        b->off_lds = off;
        off = align256(off + b->lds_bytes);
        b->off_units = off;
        off = align256(off + 4 * std::max<uint64_t>(1, units));
        b->off_gmaps = off;
        off = align256(off + 4 * std::max<uint64_t>(1, gmap));
        b->total = off;
        b->blob.assign(b->off_units - b->off_tables, 0);
        auto put = [&](uint64_t at, const void *src, size_t bytes) {
            if (bytes) std::memcpy(&b->blob[at - b->off_tables], src, bytes);
        };
        put(b->off_tables, bt.data(), sizeof(BTable) * bt.size());
        put(b->off_docs, docs.data(), sizeof(BDoc) * docs.size());
        put(b->off_jobs, bj.data(), sizeof(BJob) * bj.size());
        put(b->off_gjobs, gj.data(), sizeof(BGroupJob) * gj.size());
        if (b->lds_tables)   // the LDS images of all tables, contiguous, from the tables' packed host images
            for (uint32_t t = 0; t < n_tables; ++t) {
                const Image &im = tables[t]->L.img[0];
                put(b->off_lds + bt[t].lds_off, tables[t]->image.data() + im.off, im.bytes);
            }
    } catch (const std::bad_alloc &) {
        delete b;
        return sfa_fail(SFA_ERR_HOST_ALLOC, "out of host memory");
    }
    if (b->lds_tables) {
        // allow dynamic LDS above 64 KiB for every instantiation
        const int lds = (int)b->lds_bytes;
        hipError_t e = hipFuncSetAttribute((const void *)k_batch_walk<1, true>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_batch_walk<2, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_batch_walk<4, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) {
            delete b;
            return sfa_fail(SFA_ERR_HIP, std::string("batch LDS attribute: ") + hipGetErrorString(e));
        }
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
    out->n_group_items = b->n_items;
    out->piece_bytes = b->piece;
    out->group_pieces = b->group;
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
    hipError_t e = hipMemcpyAsync((uint8_t *)d_ws + b->off_tables, b->blob.data(), b->blob.size(), hipMemcpyHostToDevice,
                                  (hipStream_t)stream);
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
    a.unit_state = (uint32_t *)(ws + b->off_units);
    a.gmaps = (uint32_t *)(ws + b->off_gmaps);
    a.out = d_out;
    a.n_units = b->n_units;
    a.n_items = b->n_items;
    a.n_docs = b->n_docs;
    a.n_jobs = b->n_jobs;
    a.n_gjobs = b->n_gjobs;
    a.n_tables = b->n_tables;
    a.piece = b->piece;
    a.group = b->group;
    a.lds_tables = b->lds_tables;
    a.lds_bytes = b->lds_bytes;
    a.lds_image = ws + b->off_lds;
    hipStream_t s = (hipStream_t)stream;
    const uint64_t lanes = (b->n_units + b->K - 1) / b->K;
    const uint64_t wblocks = (lanes + kTB - 1) / kTB;
    const size_t lds = b->lds_tables ? b->lds_bytes : 0;
    hipError_t e = hipSuccess;
    if (b->lds_tables) {
        if (b->K == 4) e = launch(k_batch_walk<4, true>, wblocks, lds, s, a);
        else if (b->K == 2) e = launch(k_batch_walk<2, true>, wblocks, lds, s, a);
        else e = launch(k_batch_walk<1, true>, wblocks, lds, s, a);
    } else {
        if (b->K == 4) e = launch(k_batch_walk<4, false>, wblocks, 0, s, a);
        else if (b->K == 2) e = launch(k_batch_walk<2, false>, wblocks, 0, s, a);
        else e = launch(k_batch_walk<1, false>, wblocks, 0, s, a);
    }
    if (e == hipSuccess) e = launch(k_batch_groups, (b->n_items + kTB - 1) / kTB, 0, s, a);
    if (e == hipSuccess) e = launch(k_batch_compose, (b->n_jobs + kTB - 1) / kTB, 0, s, a);
    if (e != hipSuccess) return sfa_fail(SFA_ERR_HIP, std::string("batch launch: ") + hipGetErrorString(e));
    return SFA_OK;
}

extern "C" void sfa_batch_free(sfa_batch *b) { delete b; }
