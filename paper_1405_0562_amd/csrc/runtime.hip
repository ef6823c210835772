// HIP runtime of the SFA matcher for gfx950: table packing and loading, the
// walk kernel (Algorithm 5, Section 5.2), the speculative kernel
// (Algorithm 3, Section 3) and the ordered composition of chunk mappings
// (reverse composition, Section 2.1; Lemma 1 and Theorem 2, Section 4.3).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

sfa_status sfa_fail(sfa_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

extern "C" const char *sfa_last_error(void) { return g_err.c_str(); }
extern "C" uint32_t sfa_abi_version(void) { return SFA_ABI_VERSION; }

extern "C" const char *sfa_status_string(sfa_status s) {
    switch (s) {
        case SFA_OK: return "ok";
        case SFA_ERR_INVALID_ARG: return "invalid argument";
        case SFA_ERR_PARSE: return "regex parse error";
        case SFA_ERR_DFA_TOO_LARGE: return "DFA too large";
        case SFA_ERR_OVER_CAP: return "D-SFA over the state cap";
        case SFA_ERR_NO_DEVICE: return "no HIP device";
        case SFA_ERR_UNSUPPORTED_ARCH: return "device is not gfx950";
        case SFA_ERR_BUFFER_TOO_SMALL: return "device buffer too small";
        case SFA_ERR_HIP: return "HIP runtime error";
        case SFA_ERR_NO_SFA: return "table has no D-SFA";
        case SFA_ERR_HOST_ALLOC: return "host allocation failed";
    }
    return "unknown status";
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return sfa_fail(SFA_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// device table layout
// ---------------------------------------------------------------------------
namespace {

constexpr uint32_t kBlock = 256;          // threads per block of the walk kernel
constexpr uint32_t kSpecWaves = 4;        // waves (chunks) per speculative block
constexpr uint32_t kDefaultLdsBudget = 96 * 1024;
constexpr uint32_t kScratchLds = 16 * 1024;  // LDS for group mappings in the composition
constexpr uint64_t kWsHeader = 256;       // control word area at the start of a workspace

inline uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

struct Layout {
    uint32_t n_dfa = 0, n_sfa = 0, C = 0, q0 = 0;
    uint32_t next_w = 0, map_w = 0;
    uint32_t in_lds = 0;
    uint64_t off_cls = 0;    // u16[256]: cls[b] * next_w      (walk kernel)
    uint64_t off_dcls = 0;   // u16[256]: cls[b] * 2            (speculative kernel)
    uint64_t off_acc = 0;    // u8[n_dfa]
    uint64_t off_dnext = 0;  // u16[n_dfa * C]
    uint64_t off_next = 0;   // next_w bytes [n_sfa * C]
    uint64_t off_map = 0;    // map_w bytes [n_sfa * n_dfa]
    uint64_t total = 0;
    uint32_t next_bytes = 0;  // bytes of the walk table
};

}  // namespace

struct sfa_table {
    Layout L;
    uint8_t *d_base = nullptr;
    int device = 0;
    uint32_t lds_per_block = 0;
    uint32_t num_cus = 0;
    std::vector<uint8_t> image;
};

namespace {

sfa_status check_device(int &dev, uint32_t &lds_per_block, uint32_t &num_cus) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0)
        return sfa_fail(SFA_ERR_NO_DEVICE, "no HIP device visible");
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return sfa_fail(SFA_ERR_UNSUPPORTED_ARCH, std::string("device arch is ") + prop.gcnArchName);
    lds_per_block = (uint32_t)prop.sharedMemPerBlock;
    num_cus = (uint32_t)prop.multiProcessorCount;
    return SFA_OK;
}

sfa_status validate(const sfa_table_desc *d) {
    if (!d) return sfa_fail(SFA_ERR_INVALID_ARG, "null descriptor");
    if (d->abi_version != SFA_ABI_VERSION) return sfa_fail(SFA_ERR_INVALID_ARG, "abi_version mismatch");
    if (d->n_dfa == 0 || d->n_dfa > 65535) return sfa_fail(SFA_ERR_INVALID_ARG, "n_dfa out of range");
    if (d->n_classes == 0 || d->n_classes > 256) return sfa_fail(SFA_ERR_INVALID_ARG, "n_classes out of range");
    if (d->q0 >= d->n_dfa) return sfa_fail(SFA_ERR_INVALID_ARG, "q0 out of range");
    if (d->n_sfa > 16777215u) return sfa_fail(SFA_ERR_INVALID_ARG, "n_sfa out of range");
    if (!d->byte_class || !d->dfa_next || !d->dfa_accept) return sfa_fail(SFA_ERR_INVALID_ARG, "null array");
    for (int b = 0; b < 256; ++b)
        if (d->byte_class[b] >= d->n_classes) return sfa_fail(SFA_ERR_INVALID_ARG, "byte_class out of range");
    const uint64_t nd = (uint64_t)d->n_dfa * d->n_classes;
    for (uint64_t i = 0; i < nd; ++i)
        if (d->dfa_next[i] >= d->n_dfa) return sfa_fail(SFA_ERR_INVALID_ARG, "dfa_next out of range");
    if (d->n_sfa) {
        if (!d->sfa_next || !d->sfa_map) return sfa_fail(SFA_ERR_INVALID_ARG, "null D-SFA array");
        const uint64_t ns = (uint64_t)d->n_sfa * d->n_classes;
        for (uint64_t i = 0; i < ns; ++i)
            if (d->sfa_next[i] >= d->n_sfa) return sfa_fail(SFA_ERR_INVALID_ARG, "sfa_next out of range");
        const uint64_t nm = (uint64_t)d->n_sfa * d->n_dfa;
        for (uint64_t i = 0; i < nm; ++i)
            if (d->sfa_map[i] >= d->n_dfa) return sfa_fail(SFA_ERR_INVALID_ARG, "sfa_map out of range");
        for (uint32_t q = 0; q < d->n_dfa; ++q)
            if (d->sfa_map[q] != q) return sfa_fail(SFA_ERR_INVALID_ARG, "D-SFA state 0 is not the identity");
    }
    return SFA_OK;
}

Layout plan(const sfa_table_desc *d, const sfa_load_options *o) {
    Layout L;
    L.n_dfa = d->n_dfa;
    L.n_sfa = d->n_sfa;
    L.C = d->n_classes;
    L.q0 = d->q0;
    L.next_w = d->n_sfa <= 256 ? 1 : d->n_sfa <= 65536 ? 2 : 4;
    L.map_w = d->n_dfa <= 256 ? 1 : 2;
    uint64_t off = 0;
    L.off_cls = off;
    off += 512;
    L.off_dcls = off;
    off += 512;
    off = align256(off);
    L.off_acc = off;
    off = align256(off + d->n_dfa);
    L.off_dnext = off;
    off = align256(off + 2ull * d->n_dfa * d->n_classes);
    L.off_next = off;
    L.next_bytes = (uint32_t)std::min<uint64_t>(UINT32_MAX, (uint64_t)L.next_w * d->n_sfa * d->n_classes);
    off = align256(off + (uint64_t)L.next_w * d->n_sfa * d->n_classes);
    L.off_map = off;
    off = align256(off + (uint64_t)L.map_w * d->n_sfa * d->n_dfa);
    L.total = off;
    uint32_t budget = (o && o->lds_budget) ? o->lds_budget : kDefaultLdsBudget;
    L.in_lds = (d->n_sfa && !(o && o->force_global) && (uint64_t)L.next_bytes <= budget) ? 1 : 0;
    return L;
}

template <typename T>
void put(std::vector<uint8_t> &img, uint64_t off, uint64_t i, T v) {
    std::memcpy(&img[off + i * sizeof(T)], &v, sizeof(T));
}

void pack(const sfa_table_desc *d, const Layout &L, std::vector<uint8_t> &img) {
    img.assign(L.total, 0);
    for (int b = 0; b < 256; ++b) {
        put<uint16_t>(img, L.off_cls, b, (uint16_t)(d->byte_class[b] * L.next_w));
        put<uint16_t>(img, L.off_dcls, b, (uint16_t)(d->byte_class[b] * 2));
    }
    for (uint32_t q = 0; q < d->n_dfa; ++q) img[L.off_acc + q] = d->dfa_accept[q] ? 1 : 0;
    for (uint64_t i = 0; i < (uint64_t)d->n_dfa * d->n_classes; ++i)
        put<uint16_t>(img, L.off_dnext, i, (uint16_t)d->dfa_next[i]);
    for (uint64_t i = 0; i < (uint64_t)d->n_sfa * d->n_classes; ++i) {
        uint32_t v = d->sfa_next[i];
        if (L.next_w == 1) put<uint8_t>(img, L.off_next, i, (uint8_t)v);
        else if (L.next_w == 2) put<uint16_t>(img, L.off_next, i, (uint16_t)v);
        else put<uint32_t>(img, L.off_next, i, v);
    }
    for (uint64_t i = 0; i < (uint64_t)d->n_sfa * d->n_dfa; ++i) {
        uint32_t v = d->sfa_map[i];
        if (L.map_w == 1) put<uint8_t>(img, L.off_map, i, (uint8_t)v);
        else put<uint16_t>(img, L.off_map, i, (uint16_t)v);
    }
}

}  // namespace

extern "C" sfa_status sfa_table_device_bytes(const sfa_table_desc *desc, const sfa_load_options *opts,
                                             size_t *out_bytes) {
    if (!out_bytes) return sfa_fail(SFA_ERR_INVALID_ARG, "null out_bytes");
    sfa_status st = validate(desc);
    if (st != SFA_OK) return st;
    *out_bytes = (size_t)plan(desc, opts).total;
    return SFA_OK;
}

extern "C" sfa_status sfa_load_table(const sfa_table_desc *desc, const sfa_load_options *opts, void *d_buf,
                                     size_t d_bytes, void *stream, sfa_table **out) {
    if (!out) return sfa_fail(SFA_ERR_INVALID_ARG, "null out");
    *out = nullptr;
    sfa_status st = validate(desc);
    if (st != SFA_OK) return st;
    if (!d_buf) return sfa_fail(SFA_ERR_INVALID_ARG, "null device buffer");
    if (((uintptr_t)d_buf & 255) != 0) return sfa_fail(SFA_ERR_INVALID_ARG, "device buffer must be 256-byte aligned");
    Layout L = plan(desc, opts);
    if (d_bytes < L.total) return sfa_fail(SFA_ERR_BUFFER_TOO_SMALL, "table buffer smaller than sfa_table_device_bytes");
    int dev;
    uint32_t lds, cus;
    st = check_device(dev, lds, cus);
    if (st != SFA_OK) return st;
    sfa_table *t = new (std::nothrow) sfa_table();
    if (!t) return sfa_fail(SFA_ERR_HOST_ALLOC, "out of host memory");
    try {
        pack(desc, L, t->image);
    } catch (const std::bad_alloc &) {
        delete t;
        return sfa_fail(SFA_ERR_HOST_ALLOC, "out of host memory");
    }
    if (L.in_lds && L.next_bytes + 512 + kScratchLds + 8 * kBlock * 4 > lds) L.in_lds = 0;
    t->L = L;
    t->d_base = (uint8_t *)d_buf;
    t->device = dev;
    t->lds_per_block = lds;
    t->num_cus = cus;
    hipError_t e = hipMemcpyAsync(d_buf, t->image.data(), L.total, hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e != hipSuccess) {
        delete t;
        return sfa_fail(SFA_ERR_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    }
    *out = t;
    return SFA_OK;
}

extern "C" sfa_status sfa_table_get_info(const sfa_table *t, sfa_table_info *out) {
    if (!t || !out) return sfa_fail(SFA_ERR_INVALID_ARG, "null argument");
    out->n_dfa = t->L.n_dfa;
    out->n_sfa = t->L.n_sfa;
    out->n_classes = t->L.C;
    out->q0 = t->L.q0;
    out->next_bytes = t->L.next_w;
    out->map_bytes = t->L.map_w;
    out->table_in_lds = t->L.in_lds;
    out->has_monoid = 0;
    out->device_bytes = t->L.total;
    return SFA_OK;
}

extern "C" sfa_status sfa_free_table(sfa_table *t) {
    delete t;
    return SFA_OK;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
namespace {

struct MatchArgs {
    const uint8_t *in;
    uint64_t n;
    uint64_t chunk_len;      // L = ceil(n / n_chunks)
    uint32_t n_chunks;
    uint32_t n_dfa;
    uint32_t q0;
    uint32_t row_bytes;      // C * next_w (walk) or C * 2 (speculative)
    uint32_t next_bytes;     // bytes of the walk table (staged into LDS when in_lds)
    uint32_t groups;         // G: groups per block in the block composition
    uint32_t final_groups;   // G for the grid composition
    const uint16_t *cls;     // u16[256]
    const uint8_t *next;     // walk table (or u16 dfa table for speculative)
    const uint8_t *map;      // mapping rows
    const uint8_t *accept;   // u8[n_dfa]
    uint32_t *counter;       // workspace control word
    uint32_t *block_maps;    // [gridDim.x * n_dfa]
    sfa_result *out;
};

template <typename MT>
__device__ __forceinline__ uint32_t map_at(const uint8_t *__restrict__ map, uint32_t f, uint32_t n_dfa, uint32_t q) {
    return ((const MT *)map)[(size_t)f * n_dfa + q];
}

// Composition of E element mappings given as rows of `map` (element e is
// D-SFA state ids[e]), in text order, into the block mapping M[q] (q < n_dfa):
//   phase 1: the E elements are cut into G consecutive groups; for every
//            (group, start state) pair one thread follows the start state
//            through the group's mappings (reverse composition applies the
//            earlier mapping first);
//   phase 2: every start state is followed through the G group mappings.
template <typename MT>
__device__ void compose_block(const uint32_t *ids, uint32_t E, const uint8_t *__restrict__ map, uint32_t n_dfa,
                              uint32_t G, uint32_t *scratch, uint32_t *__restrict__ out_map) {
    const uint32_t R = E / G;
    const uint32_t items = G * n_dfa;
    for (uint32_t it = threadIdx.x; it < items; it += blockDim.x) {
        const uint32_t g = it / n_dfa, q = it - g * n_dfa;
        uint32_t x = q;
        const uint32_t *e = ids + g * R;
        for (uint32_t i = 0; i < R; ++i) x = map_at<MT>(map, e[i], n_dfa, x);
        if (G == 1)
            out_map[q] = x;
        else
            scratch[it] = x;
    }
    if (G == 1) return;
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < n_dfa; q += blockDim.x) {
        uint32_t x = q;
        for (uint32_t g = 0; g < G; ++g) x = scratch[g * n_dfa + x];
        out_map[q] = x;
    }
}

// Grid-level step run by the last block to finish: composes the block
// mappings in block order, applies the result to q0 and writes the answer.
__device__ void finalize_grid(const MatchArgs &a, uint32_t *scratch) {
    const uint32_t B = gridDim.x, n = a.n_dfa;
    const uint32_t G = a.final_groups;   // groups of consecutive blocks
    const uint32_t R = (B + G - 1) / G;
    const uint32_t *bm = a.block_maps;
    if (G == 1) {
        if (threadIdx.x == 0) {
            uint32_t x = a.q0;
            for (uint32_t b = 0; b < B; ++b) x = __builtin_nontemporal_load(&bm[(size_t)b * n + x]);
            a.out->state = x;
            a.out->accept = a.accept[x];
        }
        return;
    }
    const uint32_t items = G * n;
    for (uint32_t it = threadIdx.x; it < items; it += blockDim.x) {
        const uint32_t g = it / n, q = it - g * n;
        uint32_t x = q;
        if (g > 0 || q == a.q0) {
            const uint32_t b0 = g * R, b1 = min(B, b0 + R);
            for (uint32_t b = b0; b < b1; ++b) x = __builtin_nontemporal_load(&bm[(size_t)b * n + x]);
        }
        scratch[it] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t x = a.q0;
        for (uint32_t g = 0; g < G; ++g) x = scratch[g * n + x];
        a.out->state = x;
        a.out->accept = a.accept[x];
    }
}

// Publish this block's mapping and let the last block compose the grid.
__device__ void block_done(const MatchArgs &a, uint32_t *scratch) {
    __shared__ uint32_t s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        // wraps to 0 after gridDim.x increments, leaving the word zero again
        const uint32_t prev = atomicInc(a.counter, gridDim.x - 1);
        s_last = (prev == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    finalize_grid(a, scratch);
}

__device__ __forceinline__ uint32_t byte_of(const uint4 &v, int i) {
    const uint32_t w = i < 4 ? v.x : i < 8 ? v.y : i < 12 ? v.z : v.w;
    return (w >> (8 * (i & 3))) & 0xffu;
}

// Walk kernel.  Lane l of block b owns chunk c = b*256 + l, walked from the
// identity (state 0) as K consecutive pieces in lock step; the K*256 piece
// states of the block are composed in text order, then across blocks.
template <int K, typename NT, typename MT, bool LDS>
__global__ __launch_bounds__(kBlock) void k_sfa_walk(MatchArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint16_t *s_cls = (uint16_t *)smem;                       // 512 B
    uint8_t *s_tab = smem + 512;                              // walk table when LDS
    const uint32_t tab_lds = LDS ? ((a.next_bytes + 15) & ~15u) : 0;
    uint32_t *s_ids = (uint32_t *)(smem + 512 + tab_lds);     // K*256 piece states
    uint32_t *s_scr = s_ids + K * kBlock;                     // composition scratch

    for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) s_cls[i] = a.cls[i];
    if constexpr (LDS) {
        const uint4 *src = (const uint4 *)a.next;
        uint4 *dst = (uint4 *)s_tab;
        for (uint32_t i = threadIdx.x; i < tab_lds / 16; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();

    const uint32_t rb = a.row_bytes;
    const uint64_t chunk = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    uint64_t c0 = a.n, c1 = a.n;
    if (chunk < a.n_chunks) {
        c0 = min(a.n, chunk * a.chunk_len);
        c1 = min(a.n, c0 + a.chunk_len);
    }
    const uint64_t len = c1 - c0;
    const uint64_t piece = (((len + K - 1) / K) + 15) & ~uint64_t(15);

    uint64_t pos[K], end[K];
    uint32_t st[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        pos[k] = min(c1, c0 + k * piece);
        end[k] = min(c1, pos[k] + piece);
        st[k] = 0;
    }
    // one D-SFA transition: f <- delta_s[f, class(b)]
    auto step = [&](uint32_t s, uint32_t b) -> uint32_t {
        if constexpr (LDS)
            return *(const NT *)(s_tab + s * rb + s_cls[b]);
        else
            return *(const NT *)(a.next + (size_t)s * rb + s_cls[b]);
    };
    if (len > 0) {
    // head: single bytes up to 16-byte alignment (same for all pieces)
    const uint32_t head = (uint32_t)((16 - ((uintptr_t)(a.in + c0) & 15)) & 15);
    for (uint32_t i = 0; i < head; ++i) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const bool act = pos[k] < end[k];
            const uint32_t b = a.in[act ? pos[k] : c0];
            const uint32_t t = step(st[k], b);
            st[k] = act ? t : st[k];
            pos[k] += act ? 1 : 0;
        }
    }
    // body: aligned 16-byte groups, next group loaded before the current one is walked
    uint64_t nb[K];
    uint64_t maxnb = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        nb[k] = (end[k] - pos[k]) / 16;
        maxnb = max(maxnb, nb[k]);
    }
    if (maxnb) {
        uint4 cur[K];
#pragma unroll
        for (int k = 0; k < K; ++k) cur[k] = *(const uint4 *)(a.in + (nb[k] ? pos[k] : pos[0]));
        for (uint64_t j = 0; j < maxnb; ++j) {
            uint4 nxt[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const bool more = j + 1 < nb[k];
                nxt[k] = *(const uint4 *)(a.in + (more ? pos[k] + 16 * (j + 1) : pos[0]));
            }
            uint32_t t[K];
#pragma unroll
            for (int k = 0; k < K; ++k) t[k] = st[k];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
#pragma unroll
                for (int k = 0; k < K; ++k) t[k] = step(t[k], byte_of(cur[k], i));
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                st[k] = (j < nb[k]) ? t[k] : st[k];
                cur[k] = nxt[k];
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) pos[k] += 16 * nb[k];
    }
    // tail: fewer than 16 bytes per piece
    for (uint32_t i = 0; i < 16; ++i) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const bool act = pos[k] < end[k];
            const uint32_t b = a.in[act ? pos[k] : c0];
            const uint32_t t = step(st[k], b);
            st[k] = act ? t : st[k];
            pos[k] += act ? 1 : 0;
        }
    }
    }  // len > 0
#pragma unroll
    for (int k = 0; k < K; ++k) s_ids[threadIdx.x * K + k] = st[k];
    __syncthreads();
    compose_block<MT>(s_ids, K * kBlock, a.map, a.n_dfa, a.groups, s_scr,
                      a.block_maps + (size_t)blockIdx.x * a.n_dfa);
    block_done(a, s_scr);
}

// Speculative kernel (Algorithm 3).  Wave w of block b walks chunk
// c = b*4 + w; lane j tracks the states q = j, j+64, ... (T[q] <- delta(T[q], sigma));
// the 4 chunk mappings are composed in order into the block mapping.
template <int S>
__global__ __launch_bounds__(kSpecWaves * 64) void k_spec_walk(MatchArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint16_t *s_cls = (uint16_t *)smem;                        // 512 B
    uint16_t *s_dn = (uint16_t *)(smem + 512);                 // u16 [n_dfa * C]
    const uint32_t dn_bytes = (a.next_bytes + 15) & ~15u;
    uint32_t *s_T = (uint32_t *)(smem + 512 + dn_bytes);       // [4][n_dfa]
    for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) s_cls[i] = a.cls[i];
    {
        const uint4 *src = (const uint4 *)a.next;
        uint4 *dst = (uint4 *)s_dn;
        for (uint32_t i = threadIdx.x; i < dn_bytes / 16; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
    const uint32_t wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const uint32_t n = a.n_dfa, rb = a.row_bytes;
    const uint64_t chunk = (uint64_t)blockIdx.x * kSpecWaves + wave;
    uint64_t c0 = a.n, c1 = a.n;
    if (chunk < a.n_chunks) {
        c0 = min(a.n, chunk * a.chunk_len);
        c1 = min(a.n, c0 + a.chunk_len);
    }
    uint32_t T[S];
#pragma unroll
    for (int s = 0; s < S; ++s) T[s] = min(lane + 64u * s, n - 1);   // clamped lanes are discarded
    const uint8_t *sp = (const uint8_t *)s_dn;
    auto step = [&](uint32_t q, uint32_t b) -> uint32_t { return *(const uint16_t *)(sp + q * rb + s_cls[b]); };
    uint64_t p = c0;
    for (; p < c1 && ((uintptr_t)(a.in + p) & 15); ++p) {
        const uint32_t b = a.in[p];
#pragma unroll
        for (int s = 0; s < S; ++s) T[s] = step(T[s], b);
    }
    for (; p + 16 <= c1; p += 16) {
        const uint4 v = *(const uint4 *)(a.in + p);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const uint32_t b = byte_of(v, i);
#pragma unroll
            for (int s = 0; s < S; ++s) T[s] = step(T[s], b);
        }
    }
    for (; p < c1; ++p) {
        const uint32_t b = a.in[p];
#pragma unroll
        for (int s = 0; s < S; ++s) T[s] = step(T[s], b);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const uint32_t q = lane + 64u * s;
        if (q < n) s_T[wave * n + q] = T[s];
    }
    __syncthreads();
    uint32_t *bm = a.block_maps + (size_t)blockIdx.x * n;
    for (uint32_t q = threadIdx.x; q < n; q += blockDim.x) {
        uint32_t x = q;
        for (uint32_t w = 0; w < kSpecWaves; ++w) x = s_T[w * n + x];
        bm[q] = x;
    }
    block_done(a, s_T);
}

// ---------------------------------------------------------------------------
// host-side launch
// ---------------------------------------------------------------------------
struct Plan {
    uint32_t n_chunks = 0, blocks = 0, K = 1, groups = 1, final_groups = 1;
    uint64_t chunk_len = 0;
    size_t ws_bytes = 0;
};

uint32_t pick_groups(uint32_t items_max, uint32_t n_dfa, uint32_t cap_groups) {
    // largest power of two G <= cap_groups with G * n_dfa * 4 <= kScratchLds
    uint32_t G = 1;
    while (G * 2 <= cap_groups && (uint64_t)G * 2 * n_dfa * 4 <= kScratchLds && G * 2 <= items_max) G *= 2;
    return G;
}

Plan make_plan(const sfa_table *t, uint64_t n, uint32_t n_chunks, bool speculative) {
    Plan P;
    const uint32_t per_block = speculative ? kSpecWaves : kBlock;
    if (n_chunks == 0) {
        const uint64_t target = speculative ? 4096 : 1024;   // bytes per chunk at least
        const uint64_t max_chunks = (uint64_t)std::max(1u, t->num_cus) * per_block * (speculative ? 8 : 1);
        uint64_t p = std::max<uint64_t>(1, (n + target - 1) / target);
        P.n_chunks = (uint32_t)std::min(p, max_chunks);
    } else {
        P.n_chunks = n_chunks;
    }
    P.chunk_len = n ? (n + P.n_chunks - 1) / P.n_chunks : 0;
    P.blocks = (uint32_t)((P.n_chunks + per_block - 1) / per_block);
    if (!speculative) {
        // pieces per lane: at least 256 bytes per piece
        uint64_t k = P.chunk_len / 256;
        P.K = k >= 8 ? 8 : k >= 4 ? 4 : k >= 2 ? 2 : 1;
        P.groups = pick_groups(P.K * kBlock, t->L.n_dfa, P.K * kBlock);
    }
    P.final_groups = pick_groups(P.blocks, t->L.n_dfa, P.blocks);
    P.ws_bytes = kWsHeader + (size_t)P.blocks * t->L.n_dfa * 4;
    return P;
}

template <int K, typename NT, typename MT, bool LDS>
hipError_t launch_walk(const MatchArgs &a, uint32_t blocks, size_t lds, hipStream_t s) {
    auto fn = k_sfa_walk<K, NT, MT, LDS>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(kBlock), lds, s, a);
    return hipGetLastError();
}

template <int K, typename NT, typename MT>
hipError_t dispatch_lds(const MatchArgs &a, bool lds_tab, uint32_t blocks, size_t lds, hipStream_t s) {
    return lds_tab ? launch_walk<K, NT, MT, true>(a, blocks, lds, s) : launch_walk<K, NT, MT, false>(a, blocks, lds, s);
}

template <int K, typename NT>
hipError_t dispatch_map(const MatchArgs &a, uint32_t map_w, bool lds_tab, uint32_t blocks, size_t lds, hipStream_t s) {
    return map_w == 1 ? dispatch_lds<K, NT, uint8_t>(a, lds_tab, blocks, lds, s)
                      : dispatch_lds<K, NT, uint16_t>(a, lds_tab, blocks, lds, s);
}

template <int K>
hipError_t dispatch_next(const MatchArgs &a, const Layout &L, uint32_t blocks, size_t lds, hipStream_t s) {
    const bool lt = L.in_lds != 0;
    if (L.next_w == 1) return dispatch_map<K, uint8_t>(a, L.map_w, lt, blocks, lds, s);
    if (L.next_w == 2) return dispatch_map<K, uint16_t>(a, L.map_w, lt, blocks, lds, s);
    return dispatch_map<K, uint32_t>(a, L.map_w, lt, blocks, lds, s);
}

sfa_status common_checks(const sfa_table *t, const uint8_t *d_in, uint64_t n, void *d_ws, size_t ws_bytes,
                         sfa_result *d_out, const Plan &P) {
    if (!t) return sfa_fail(SFA_ERR_INVALID_ARG, "null table");
    if (!d_out) return sfa_fail(SFA_ERR_INVALID_ARG, "null output");
    if (n && !d_in) return sfa_fail(SFA_ERR_INVALID_ARG, "null input");
    if (!d_ws) return sfa_fail(SFA_ERR_INVALID_ARG, "null workspace");
    if (((uintptr_t)d_ws & 255) != 0) return sfa_fail(SFA_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < P.ws_bytes) return sfa_fail(SFA_ERR_BUFFER_TOO_SMALL, "workspace smaller than sfa_match_workspace_bytes");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != t->device) return sfa_fail(SFA_ERR_INVALID_ARG, "table was loaded on another device");
    return SFA_OK;
}

MatchArgs base_args(const sfa_table *t, const uint8_t *d_in, uint64_t n, void *d_ws, sfa_result *d_out, const Plan &P) {
    MatchArgs a{};
    a.in = d_in;
    a.n = n;
    a.chunk_len = P.chunk_len;
    a.n_chunks = P.n_chunks;
    a.n_dfa = t->L.n_dfa;
    a.q0 = t->L.q0;
    a.groups = P.groups;
    a.final_groups = P.final_groups;
    a.accept = t->d_base + t->L.off_acc;
    a.map = t->d_base + t->L.off_map;
    a.counter = (uint32_t *)d_ws;
    a.block_maps = (uint32_t *)((uint8_t *)d_ws + kWsHeader);
    a.out = d_out;
    return a;
}

}  // namespace

extern "C" sfa_status sfa_match_workspace_bytes(const sfa_table *t, uint64_t n, uint32_t n_chunks, size_t *out_bytes) {
    if (!t || !out_bytes) return sfa_fail(SFA_ERR_INVALID_ARG, "null argument");
    Plan a = make_plan(t, n, n_chunks, false), b = make_plan(t, n, n_chunks, true);
    *out_bytes = std::max(a.ws_bytes, b.ws_bytes);
    return SFA_OK;
}

extern "C" sfa_status sfa_match(const sfa_table *t, const uint8_t *d_in, uint64_t n, uint32_t n_chunks, void *d_ws,
                                size_t ws_bytes, sfa_result *d_out, void *stream) {
    if (!t) return sfa_fail(SFA_ERR_INVALID_ARG, "null table");
    if (t->L.n_sfa == 0) return sfa_fail(SFA_ERR_NO_SFA, "table has no D-SFA; use sfa_match_speculative");
    Plan P = make_plan(t, n, n_chunks, false);
    sfa_status st = common_checks(t, d_in, n, d_ws, ws_bytes, d_out, P);
    if (st != SFA_OK) return st;
    MatchArgs a = base_args(t, d_in, n, d_ws, d_out, P);
    a.row_bytes = t->L.C * t->L.next_w;
    a.next_bytes = t->L.next_bytes;
    a.cls = (const uint16_t *)(t->d_base + t->L.off_cls);
    a.next = t->d_base + t->L.off_next;
    const size_t lds = 512 + (t->L.in_lds ? ((t->L.next_bytes + 15) & ~15u) : 0) + (size_t)P.K * kBlock * 4 +
                       std::max<size_t>(P.groups > 1 ? (size_t)P.groups * t->L.n_dfa * 4 : 0,
                                        P.final_groups > 1 ? (size_t)P.final_groups * t->L.n_dfa * 4 : 0);
    if (lds > t->lds_per_block) return sfa_fail(SFA_ERR_INVALID_ARG, "LDS plan exceeds the device limit");
    hipError_t e;
    switch (P.K) {
        case 8: e = dispatch_next<8>(a, t->L, P.blocks, lds, (hipStream_t)stream); break;
        case 4: e = dispatch_next<4>(a, t->L, P.blocks, lds, (hipStream_t)stream); break;
        case 2: e = dispatch_next<2>(a, t->L, P.blocks, lds, (hipStream_t)stream); break;
        default: e = dispatch_next<1>(a, t->L, P.blocks, lds, (hipStream_t)stream); break;
    }
    if (e != hipSuccess) return sfa_fail(SFA_ERR_HIP, std::string("walk launch: ") + hipGetErrorString(e));
    return SFA_OK;
}

extern "C" sfa_status sfa_match_speculative(const sfa_table *t, const uint8_t *d_in, uint64_t n, uint32_t n_chunks,
                                            void *d_ws, size_t ws_bytes, sfa_result *d_out, void *stream) {
    if (!t) return sfa_fail(SFA_ERR_INVALID_ARG, "null table");
    Plan P = make_plan(t, n, n_chunks, true);
    sfa_status st = common_checks(t, d_in, n, d_ws, ws_bytes, d_out, P);
    if (st != SFA_OK) return st;
    MatchArgs a = base_args(t, d_in, n, d_ws, d_out, P);
    a.row_bytes = t->L.C * 2;
    a.next_bytes = 2 * t->L.n_dfa * t->L.C;
    a.cls = (const uint16_t *)(t->d_base + t->L.off_dcls);
    a.next = t->d_base + t->L.off_dnext;
    const uint32_t nd = t->L.n_dfa;
    const size_t lds = 512 + ((a.next_bytes + 15) & ~15u) +
                       std::max<size_t>((size_t)kSpecWaves * nd * 4,
                                        P.final_groups > 1 ? (size_t)P.final_groups * nd * 4 : 0);
    if (lds > t->lds_per_block)
        return sfa_fail(SFA_ERR_INVALID_ARG, "DFA too large for the speculative kernel's LDS plan");
    const uint32_t S = (nd + 63) / 64;
    hipError_t e;
    const dim3 grid(P.blocks), block(kSpecWaves * 64);
    hipStream_t s = (hipStream_t)stream;
    auto go = [&](auto fn) -> hipError_t {
        if (lds > 64 * 1024) {
            hipError_t e2 = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e2 != hipSuccess) return e2;
        }
        hipLaunchKernelGGL(fn, grid, block, lds, s, a);
        return hipGetLastError();
    };
    if (S <= 1) e = go(k_spec_walk<1>);
    else if (S <= 2) e = go(k_spec_walk<2>);
    else if (S <= 4) e = go(k_spec_walk<4>);
    else if (S <= 8) e = go(k_spec_walk<8>);
    else if (S <= 16) e = go(k_spec_walk<16>);
    else return sfa_fail(SFA_ERR_INVALID_ARG, "speculative kernel supports at most 1024 DFA states");
    if (e != hipSuccess) return sfa_fail(SFA_ERR_HIP, std::string("speculative launch: ") + hipGetErrorString(e));
    return SFA_OK;
}
