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

#include "device.h"
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

constexpr uint32_t kBlock = 256;             // threads per block of the walk kernels
constexpr uint32_t kGlobalBlock = 512;       // default threads per block of the global-table walk
constexpr uint64_t kShortChunk = 4096;       // chunk bytes up to which the stride-4 walk uses 512 threads
constexpr uint32_t kSpecWaves = 4;           // waves (chunks) per speculative block
constexpr uint32_t kDefaultLdsBudget = 96 * 1024;
constexpr uint32_t kScratchLds = 16 * 1024;  // LDS for group mappings in the composition
constexpr uint32_t kMaxIds = 8 * kBlock;     // piece states per block (K * block threads <= 2048)
constexpr uint32_t kPairTable = 65536;       // byte-pair class table entries (u8)
constexpr uint32_t kSpecStage = 16 * 1024;  // speculative blocks: LDS region for the grid composition
constexpr uint32_t kMulMax = 16 * 1024;      // product table bytes at most (u8 ids: n_sfa <= 128)
constexpr uint32_t kIdRun = 4096;            // product mode: blocks per level-1 run
constexpr uint64_t kWsHeader = 4096;         // workspace control words: [0] top level, [1 + r] level-1 run r
constexpr uint32_t kMaxRuns = kWsHeader / 4 - 1;

inline uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// Byte-pair class table layout.  Entry h = b0 | b1 << 8 (b0 first in the
// text) sits at h with its bits 2..7 XORed with bits 0..5 of b1: the LDS
// bank of an entry then depends on both bytes, not on b0 alone (text over a
// small alphabet would otherwise put every lookup of a wave in a few banks).
// A permutation within each 256-entry block, so the table stays 64 KiB.
__host__ __device__ inline uint32_t pair_slot(uint32_t h) { return h ^ ((h >> 6) & 0xfcu); }
// Both pair slots of a 4-byte word at once: low half and high half of the result.
__host__ __device__ inline uint32_t pair_slots(uint32_t w) { return w ^ ((w >> 6) & 0x00fc00fcu); }

}  // namespace


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

uint64_t ipow(uint64_t b, uint32_t e) {
    uint64_t r = 1;
    while (e--) r *= b;
    return r;
}

// True when the product table is well defined for d: every D-SFA state is
// reachable from the identity (state 0), and the mapping rows agree with the
// transitions, sfa_map[sfa_next[s][c]][q] = dfa_next[sfa_map[s][q]][c], so
// that state ids compose like the mappings they stand for (Lemma 1).
bool product_defined(const sfa_table_desc *d) {
    const uint32_t m = d->n_sfa, C = d->n_classes, n = d->n_dfa;
    if (m == 0 || (uint64_t)m * C * n > (1u << 24)) return false;
    std::vector<uint8_t> seen(m, 0);
    std::vector<uint32_t> order{0};
    seen[0] = 1;
    for (size_t h = 0; h < order.size(); ++h)
        for (uint32_t c = 0; c < C; ++c) {
            const uint32_t t = d->sfa_next[(uint64_t)order[h] * C + c];
            if (!seen[t]) {
                seen[t] = 1;
                order.push_back(t);
            }
        }
    if (order.size() != m) return false;
    for (uint32_t s = 0; s < m; ++s)
        for (uint32_t c = 0; c < C; ++c) {
            const uint32_t *to = d->sfa_map + (uint64_t)d->sfa_next[(uint64_t)s * C + c] * n;
            const uint32_t *from = d->sfa_map + (uint64_t)s * n;
            for (uint32_t x = 0; x < n; ++x)
                if (to[x] != d->dfa_next[(uint64_t)from[x] * C + c]) return false;
        }
    return true;
}

// LDS bytes the walk kernel needs besides the image: piece states + scratch.
constexpr uint32_t kWalkExtraLds = kMaxIds * 4 + 16 + kScratchLds;

Layout plan(const sfa_table_desc *d, const sfa_load_options *o, uint32_t lds_limit) {
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
    L.next_bytes = (uint64_t)L.next_w * d->n_sfa * d->n_classes;
    off = align256(off + L.next_bytes);
    L.off_map = off;
    off = align256(off + (uint64_t)L.map_w * d->n_sfa * d->n_dfa);
    if (!(o && o->no_product) && (uint64_t)d->n_sfa * d->n_sfa <= kMulMax && product_defined(d)) {
        L.off_mul = off;
        L.mul_bytes = d->n_sfa * d->n_sfa;
        off = align256(off + L.mul_bytes);
    }
    const uint32_t extra = kWalkExtraLds + ((L.mul_bytes + 15) & ~15u);
    const bool allow_lds = d->n_sfa && !(o && o->force_global);
    const uint64_t budget = std::min<uint64_t>((o && o->lds_budget) ? o->lds_budget : kDefaultLdsBudget + kPairTable,
                                               lds_limit > extra ? lds_limit - extra : 0);
    for (uint32_t S : {1u, 2u, 4u}) {
        Image &im = L.img[stride_index(S)];
        if (!allow_lds) continue;
        if (S >= 2 && 2 * ((uint64_t)L.C * L.C - 1) > 255) continue;   // doubled pair index fits u8
        if (S == 1 && 2 * ((uint64_t)L.C - 1) > 255) continue;
        const uint64_t cs = ipow(L.C, S);
        const uint64_t cols = cs + (S >= 2 ? L.C : 0);
        const uint64_t rs = 2 * cols;
        if ((uint64_t)d->n_sfa * rs > 65536) continue;   // row offsets must fit u16
        const uint64_t bytes = (S >= 2 ? kPairTable : 0) + 256 + (uint64_t)d->n_sfa * rs;
        if (bytes > budget) continue;
        im.present = 1;
        im.bytes = (uint32_t)bytes;
        im.row_bytes = (uint32_t)rs;
        im.one_off = S >= 2 ? (uint32_t)(2 * cs) : 0;
        im.off = off;
        off = align256(off + bytes);
    }
    L.total = off;
    const bool any_img = L.img[0].present || L.img[1].present || L.img[2].present;
    if (d->n_sfa && !any_img) {
        // global-table walk: stage as many leading rows as the budget holds
        const uint64_t rb = (uint64_t)L.C * L.next_w;
        const uint64_t hb = std::min<uint64_t>((o && o->lds_budget) ? o->lds_budget : lds_limit,
                                               lds_limit > extra + 512 ? lds_limit - extra - 512 : 0);
        L.hot_rows = (uint32_t)std::min<uint64_t>(d->n_sfa, rb ? hb / rb : 0);
    }
    const uint32_t rn = o ? o->renumber : 0;
    L.renumbered = d->n_sfa > 1 && (rn == 1 || (rn == 0 && !any_img)) ? 1 : 0;
    return L;
}

// States of the small closed sets of the D-SFA's transition graph: strongly
// connected components with no edge leaving them, of at most kTrapScc states.
// A walk that enters one never leaves it, so it spends the rest of its chunk
// there, while a profiling walk may never reach it (the constant mapping to
// an accepting sink, entered once a keyword has been read, is the usual
// case).  Iterative Tarjan over the n_sfa x C graph; components in the order
// they complete.
constexpr uint32_t kTrapScc = 64, kTrapTotal = 1024;

std::vector<uint32_t> trap_states(const sfa_table_desc *d) {
    const uint32_t m = d->n_sfa, C = d->n_classes, none = ~0u;
    std::vector<uint32_t> index(m, none), low(m, 0), stack, out;
    std::vector<uint8_t> on(m, 0);
    std::vector<std::pair<uint32_t, uint32_t>> call;   // (state, next class to visit)
    uint32_t next_index = 0;
    for (uint32_t root = 0; root < m && out.size() < kTrapTotal; ++root) {
        if (index[root] != none) continue;
        call.push_back({root, 0});
        index[root] = low[root] = next_index++;
        stack.push_back(root);
        on[root] = 1;
        while (!call.empty()) {
            auto &[v, c] = call.back();
            if (c < C) {
                const uint32_t w = d->sfa_next[(uint64_t)v * C + c++];
                if (index[w] == none) {
                    index[w] = low[w] = next_index++;
                    stack.push_back(w);
                    on[w] = 1;
                    call.push_back({w, 0});
                } else if (on[w]) {
                    low[v] = std::min(low[v], index[w]);
                }
                continue;
            }
            const uint32_t done = v;
            call.pop_back();
            if (!call.empty()) low[call.back().first] = std::min(low[call.back().first], low[done]);
            if (low[done] != index[done]) continue;
            // done is the root of a component: pop it, then test that every edge stays inside
            size_t first = stack.size();
            while (stack[first - 1] != done) --first;
            --first;
            std::vector<uint32_t> comp(stack.begin() + first, stack.end());
            stack.resize(first);
            bool closed = comp.size() <= kTrapScc;
            for (uint32_t q : comp) on[q] = 2;      // 2: in the component being tested
            for (size_t i = 0; closed && i < comp.size(); ++i)
                for (uint32_t cc = 0; cc < C; ++cc)
                    if (on[d->sfa_next[(uint64_t)comp[i] * C + cc]] != 2) { closed = false; break; }
            for (uint32_t q : comp) on[q] = 0;
            if (closed && out.size() + comp.size() <= kTrapTotal) out.insert(out.end(), comp.begin(), comp.end());
        }
    }
    return out;
}

// Permutation of D-SFA ids for the hot-row walk: identity stays 0; then the
// states of the small closed sets above; then the rest by visit count in a
// profiling walk (descending, ties by id).  The walk follows the sample bytes
// (256 walkers over consecutive parts) or, without a sample, classes drawn
// uniformly (256 walkers x 2048 steps, xorshift generator).
std::vector<uint32_t> visit_order(const sfa_table_desc *d, const sfa_load_options *o) {
    const uint32_t m = d->n_sfa, C = d->n_classes;
    std::vector<uint64_t> count(m, 0);
    const uint32_t W = 256;
    if (o && o->profile_sample && o->profile_bytes) {
        const uint64_t part = std::max<uint64_t>(1, o->profile_bytes / W);
        for (uint32_t w = 0; w < W; ++w) {
            uint32_t s = 0;
            const uint64_t b0 = (uint64_t)w * part, b1 = std::min<uint64_t>(o->profile_bytes, b0 + part);
            for (uint64_t i = b0; i < b1; ++i) {
                s = d->sfa_next[(uint64_t)s * C + d->byte_class[o->profile_sample[i]]];
                ++count[s];
            }
        }
    } else {
        uint32_t x = 0x9e3779b9u;
        for (uint32_t w = 0; w < W; ++w) {
            uint32_t s = 0;
            for (uint32_t i = 0; i < 2048; ++i) {
                x ^= x << 13;
                x ^= x >> 17;
                x ^= x << 5;
                s = d->sfa_next[(uint64_t)s * C + (x % C)];
                ++count[s];
            }
        }
    }
    // closed sets rank above every visited state (a count no walk reaches)
    const uint64_t top = ~0ull;
    const std::vector<uint32_t> traps = trap_states(d);
    for (size_t i = 0; i < traps.size(); ++i) count[traps[i]] = top - i;
    std::vector<uint32_t> ids(m);
    for (uint32_t i = 0; i < m; ++i) ids[i] = i;
    std::stable_sort(ids.begin() + 1, ids.end(), [&](uint32_t a, uint32_t b) { return count[a] > count[b]; });
    std::vector<uint32_t> perm(m);   // old id -> new id
    for (uint32_t i = 0; i < m; ++i) perm[ids[i]] = i;
    return perm;
}

template <typename T>
void put(std::vector<uint8_t> &img, uint64_t off, uint64_t i, T v) {
    std::memcpy(&img[off + i * sizeof(T)], &v, sizeof(T));
}

void pack(const sfa_table_desc *d0, const sfa_load_options *o, const Layout &L, std::vector<uint8_t> &img) {
    img.assign(L.total, 0);
    const uint32_t C = L.C;
    // renumbered copies of the D-SFA arrays (new id = perm[old id])
    sfa_table_desc dd = *d0;
    std::vector<uint32_t> rnext, rmap;
    if (L.renumbered) {
        const std::vector<uint32_t> perm = visit_order(d0, o);
        const uint32_t m = d0->n_sfa, n = d0->n_dfa;
        rnext.resize((uint64_t)m * C);
        rmap.resize((uint64_t)m * n);
        for (uint32_t s = 0; s < m; ++s) {
            const uint32_t t = perm[s];
            for (uint32_t c = 0; c < C; ++c) rnext[(uint64_t)t * C + c] = perm[d0->sfa_next[(uint64_t)s * C + c]];
            std::memcpy(&rmap[(uint64_t)t * n], &d0->sfa_map[(uint64_t)s * n], sizeof(uint32_t) * n);
        }
        dd.sfa_next = rnext.data();
        dd.sfa_map = rmap.data();
    }
    const sfa_table_desc *d = &dd;
    for (int b = 0; b < 256; ++b) {
        put<uint16_t>(img, L.off_cls, b, (uint16_t)(d->byte_class[b] * L.next_w));
        put<uint16_t>(img, L.off_dcls, b, (uint16_t)(d->byte_class[b] * 2));
    }
    for (uint32_t q = 0; q < d->n_dfa; ++q) img[L.off_acc + q] = d->dfa_accept[q] ? 1 : 0;
    for (uint64_t i = 0; i < (uint64_t)d->n_dfa * C; ++i)
        put<uint16_t>(img, L.off_dnext, i, (uint16_t)d->dfa_next[i]);
    for (uint64_t i = 0; i < (uint64_t)d->n_sfa * C; ++i) {
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
    if (L.mul_bytes) {
        // breadth-first tree from the identity: parent of each state and the
        // class on the edge into it; then f_a . f_b = delta_s(f_a . f_parent(b),
        // class into b), filled in breadth-first order of b
        const uint32_t m = d->n_sfa;
        std::vector<uint32_t> order{0}, par(m, UINT32_MAX), pcls(m, 0);
        par[0] = 0;
        for (size_t h = 0; h < order.size(); ++h)
            for (uint32_t c = 0; c < C; ++c) {
                const uint32_t t = d->sfa_next[(uint64_t)order[h] * C + c];
                if (par[t] == UINT32_MAX) {
                    par[t] = order[h];
                    pcls[t] = c;
                    order.push_back(t);
                }
            }
        for (uint32_t a = 0; a < m; ++a) {
            uint8_t *row = &img[L.off_mul + (uint64_t)a * m];
            row[0] = (uint8_t)a;
            for (size_t h = 1; h < order.size(); ++h) {
                const uint32_t b = order[h];
                row[b] = (uint8_t)d->sfa_next[(uint64_t)row[par[b]] * C + pcls[b]];
            }
        }
    }
    for (uint32_t S : {1u, 2u, 4u}) {
        const Image &im = L.img[stride_index(S)];
        if (!im.present) continue;
        uint64_t o = im.off;
        if (S >= 2) {
            for (uint32_t h = 0; h < kPairTable; ++h)   // little endian: low byte comes first in the text
                img[o + pair_slot(h)] = (uint8_t)(2 * (d->byte_class[h & 255] * C + d->byte_class[h >> 8]));
            o += kPairTable;
        }
        for (int b = 0; b < 256; ++b) img[o + b] = (uint8_t)(2 * d->byte_class[b]);
        o += 256;
        const uint32_t cs = (uint32_t)ipow(C, S);
        const uint32_t cols = im.row_bytes / 2;
        for (uint32_t s = 0; s < d->n_sfa; ++s) {
            for (uint32_t col = 0; col < cs; ++col) {
                uint32_t t = s, rem = col, div = cs / C;
                for (uint32_t i = 0; i < S; ++i) {      // digits, most significant first
                    const uint32_t c = rem / div;
                    rem -= c * div;
                    div = div > 1 ? div / C : 1;
                    t = d->sfa_next[(uint64_t)t * C + c];
                }
                put<uint16_t>(img, o, (uint64_t)s * cols + col, (uint16_t)(t * im.row_bytes));
            }
            if (S >= 2)
                for (uint32_t c = 0; c < C; ++c)
                    put<uint16_t>(img, o, (uint64_t)s * cols + cs + c,
                                  (uint16_t)(d->sfa_next[(uint64_t)s * C + c] * im.row_bytes));
        }
    }
}

}  // namespace

extern "C" sfa_status sfa_table_device_bytes(const sfa_table_desc *desc, const sfa_load_options *opts,
                                             size_t *out_bytes) {
    if (!out_bytes) return sfa_fail(SFA_ERR_INVALID_ARG, "null out_bytes");
    sfa_status st = validate(desc);
    if (st != SFA_OK) return st;
    // the LDS limit of gfx950 (160 KiB per workgroup); the loader re-plans
    // with the device's reported limit, which can only shrink the layout
    *out_bytes = (size_t)plan(desc, opts, 160 * 1024).total;
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
    int dev;
    uint32_t lds, cus;
    st = check_device(dev, lds, cus);
    if (st != SFA_OK) return st;
    Layout L = plan(desc, opts, std::min<uint32_t>(lds, 160 * 1024));
    if (d_bytes < L.total) return sfa_fail(SFA_ERR_BUFFER_TOO_SMALL, "table buffer smaller than sfa_table_device_bytes");
    sfa_table *t = new (std::nothrow) sfa_table();
    if (!t) return sfa_fail(SFA_ERR_HOST_ALLOC, "out of host memory");
    try {
        pack(desc, opts, L, t->image);
    } catch (const std::bad_alloc &) {
        delete t;
        return sfa_fail(SFA_ERR_HOST_ALLOC, "out of host memory");
    }
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
    std::memset(out, 0, sizeof(*out));
    out->n_dfa = t->L.n_dfa;
    out->n_sfa = t->L.n_sfa;
    out->n_classes = t->L.C;
    out->q0 = t->L.q0;
    out->next_bytes = t->L.next_w;
    out->map_bytes = t->L.map_w;
    out->table_in_lds = t->L.img[0].present | t->L.img[1].present | t->L.img[2].present;
    out->hot_rows = t->L.hot_rows;
    out->strides = (t->L.img[0].present ? 2u : 0u) | (t->L.img[1].present ? 4u : 0u) | (t->L.img[2].present ? 16u : 0u);
    out->product_table = t->L.mul_bytes ? 1u : 0u;
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

using sfa_dev::copy16;

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
    const uint16_t *cls;     // global walk / speculative: u16[256] class column offsets
    const uint8_t *img;      // LDS image, global walk table, or u16 DFA table
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
};

// Phase 1 of a composition: the elements 0..E-1 (mappings, in text order) are
// cut into G groups of R consecutive elements; for every (group g, start
// state q) pair, q is followed through the group's mappings, the earlier
// mapping first (reverse composition, f . g = g o f), and the end state is
// stored at out[g * n + q].  `get(e, x)` is mapping e applied to x.  Four
// pairs per thread are followed together to hide load latency.
template <typename Get, typename Out>
__device__ __forceinline__ void follow_groups(Get get, uint32_t E, uint32_t R, uint32_t G, uint32_t n,
                                              Out *out) {
    const uint32_t items = G * n;
    for (uint32_t base = threadIdx.x; base < items; base += 4 * blockDim.x) {
        uint32_t it[4], x[4], e0[4], e1[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            it[i] = min(base + (uint32_t)i * blockDim.x, items - 1);
            const uint32_t g = it[i] / n;
            x[i] = it[i] - g * n;
            e0[i] = g * R;
            e1[i] = min(E, e0[i] + R);
        }
        for (uint32_t r = 0; r < R; ++r) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t e = e0[i] + r;
                const uint32_t y = get(min(e, E - 1), x[i]);
                x[i] = e < e1[i] ? y : x[i];
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (base + (uint32_t)i * blockDim.x < items) out[it[i]] = x[i];
    }
}

// Block composition: the block's E piece states (D-SFA ids in text order,
// s_ids) become the block mapping M[q], written to out_map (u16).  The
// mapping rows are read from LDS (copied over the walk-table region) when
// they fit.
template <typename MT>
__device__ __forceinline__ void compose_block(const MatchArgs &a, uint8_t *smem, const uint32_t *s_ids, uint32_t E,
                              uint32_t *scratch, uint16_t *__restrict__ out_map) {
    const uint32_t n = a.n_dfa, G = a.groups, R = E / G;
    uint32_t *target = scratch;
    if (a.map_lds) {
        copy16((uint4 *)smem, (const uint4 *)a.map, (a.map_bytes + 15) / 16);
        __syncthreads();
        const MT *m = (const MT *)smem;
        auto get = [&](uint32_t e, uint32_t x) -> uint32_t { return m[s_ids[e] * n + x]; };
        if (G == 1) {
            follow_groups(get, E, R, 1, n, out_map);
            return;
        }
        follow_groups(get, E, R, G, n, target);
    } else {
        const MT *__restrict__ m = (const MT *)a.map;
        auto get = [&](uint32_t e, uint32_t x) -> uint32_t { return m[(size_t)s_ids[e] * n + x]; };
        if (G == 1) {
            follow_groups(get, E, R, 1, n, out_map);
            return;
        }
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
    auto row = [&](uint32_t off) -> uint32_t { return *(const uint16_t *)(smem + TAB + off); };
    // one byte: f <- delta_s[f, class(b)]
    auto step1 = [&](uint32_t st, uint32_t b) -> uint32_t { return row(st + one + smem[CLS + b]); };

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
                                for (int k = 0; k < K; ++k) c[k] = smem[CLS + ((word_of(cur[k][v], d) >> (8 * i)) & 255u)];
#pragma unroll
                                for (int k = 0; k < K; ++k) t[k] = row(t[k] + c[k]);
                            }
                        } else if constexpr (S == 2) {
                            uint32_t p0[K], p1[K];
#pragma unroll
                            for (int k = 0; k < K; ++k) {
                                const uint32_t w = pair_slots(word_of(cur[k][v], d));
                                p0[k] = smem[w & 0xffffu];
                                p1[k] = smem[w >> 16];
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
                                p0[k] = smem[w & 0xffffu];
                                p1[k] = smem[w >> 16];
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

// Global-table walk (tables too large for an LDS image): stride 1, state
// ids of width NT.  The table's rows 0..hot_rows-1 (the most visited
// states, after the loader's renumbering) are staged in LDS; other rows are
// read through L1/L2.  Each byte step reads the next row of all K pieces
// from LDS at once (offsets clamped into the staged rows, so the K chains
// overlap), then pieces whose state is not staged reload the row from
// global memory (rare; exec-masked).  The input is loaded as in the LDS
// walk: G bytes of each piece per step, loads issued D - 1 steps ahead.
template <int K, int G, int D, typename NT, int TB>
__global__ __launch_bounds__(TB) void k_sfa_global(MatchArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint16_t *s_cls = (uint16_t *)smem;            // 512 B
    const uint32_t rb = a.row_bytes, H = a.hot_rows;
    const uint32_t hot_bytes = ((H * rb) + 15) & ~15u;
    uint8_t *s_hot = smem + 512;
    uint8_t *s_mul = s_hot + hot_bytes;                     // product table (product mode)
    uint32_t *s_ids = (uint32_t *)(s_mul + a.mul_lds);
    uint32_t *s_flag = s_ids + K * TB;
    uint32_t *s_scr = s_flag + 4;

    uint64_t c0, c1, pos[K], end[K];
    lane_pieces<K, G, TB>(a, c0, c1, pos, end);
    const uint32_t head = c1 > c0 ? (uint32_t)((16 - ((uintptr_t)(a.in + pos[0]) & 15)) & 15) : 0u;
    uint64_t body[K], nb[K], maxnb = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        body[k] = min(end[k], pos[k] + head);
        nb[k] = (end[k] - body[k]) / G;
        maxnb = max(maxnb, nb[k]);
    }
    constexpr int V = G / 16;
    uint4 buf[D][K][V];
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
#pragma unroll
    for (int d = 0; d < D - 1; ++d)
        if ((uint64_t)d < maxnb) issue(buf[d], d);

    for (uint32_t i = threadIdx.x; i < 256; i += TB) s_cls[i] = a.cls[i];
    copy16((uint4 *)s_hot, (const uint4 *)a.img, hot_bytes / 16);
    if (a.mul_lds) copy16((uint4 *)s_mul, (const uint4 *)a.mul, a.mul_lds / 16);
    __syncthreads();

    const uint8_t *__restrict__ tab = a.img;
    const uint32_t lim = hot_bytes >= (uint32_t)sizeof(NT) ? hot_bytes - (uint32_t)sizeof(NT) : 0u;
    // one byte of one piece (heads and tails)
    auto step1 = [&](uint32_t s, uint32_t b) -> uint32_t {
        const uint32_t off = __umul24(s, rb) + s_cls[b];
        if (s < H) return *(const NT *)(s_hot + off);
        return *(const NT *)(tab + off);
    };
    // one byte of every piece.  All K rows are read from LDS (at a clamped
    // offset); a piece outside the staged rows then takes its row from the
    // global table through a scalar load, one lane at a time.  Scalar loads
    // are counted apart from vector loads, so a miss does not wait for the
    // input loads in flight, as a vector load would (those complete in order).
    auto stepK = [&](uint32_t (&t)[K], const uint32_t (&col)[K]) {
        uint32_t off[K], v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) off[k] = __umul24(t[k], rb) + col[k];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = *(const NT *)(s_hot + min(off[k], lim));
        uint32_t bits = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) bits |= (t[k] >= H ? 1u : 0u) << k;
        for (uint64_t m = __ballot(bits != 0); m; m &= m - 1) {
            const uint32_t l = (uint32_t)__builtin_ctzll(m);
            const uint32_t lb = __builtin_amdgcn_readlane(bits, l);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (lb & (1u << k)) {
                    const uint32_t o = __builtin_amdgcn_readlane(off[k], l);
                    const uint32_t w = *(const __attribute__((address_space(4))) uint32_t *)(tab + (o & ~3u));
                    const uint32_t x = (w >> (8 * (o & 3u & ~(uint32_t)(sizeof(NT) - 1)))) & (uint32_t)(NT)~0u;
                    if (__lane_id() == l) v[k] = x;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) t[k] = v[k];
    };

    uint32_t st[K];
#pragma unroll
    for (int k = 0; k < K; ++k) st[k] = 0;
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
                        // the class columns of a word's four bytes do not depend on
                        // the walk: read them before its first step
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            uint32_t col[K];
#pragma unroll
                            for (int k = 0; k < K; ++k) col[k] = s_cls[(word_of(cur[k][v], d) >> (8 * i)) & 255u];
                            stepK(t, col);
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < K; ++k) st[k] = (step < nb[k]) ? t[k] : st[k];
            };
            uint64_t j = 0;
            for (; j + 2 * D - 1 <= maxnb; j += D) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    issue(buf[(d + D - 1) % D], j + d + D - 1);
                    walk(buf[d], j + d);
                }
            }
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
    if (a.mul_lds) {
        uint32_t x = st[0];
#pragma unroll
        for (int k = 1; k < K; ++k) x = s_mul[x * a.n_sfa + st[k]];
        finish_ids(a, block_product(x, s_mul, a.n_sfa, s_scr), s_mul, s_scr, s_flag);
        return;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) s_ids[threadIdx.x * K + k] = st[k];
    __syncthreads();
    const uint32_t E = K * TB;
    uint16_t *bmap = a.block_maps + (size_t)blockIdx.x * a.map_stride;
    if (a.n_dfa <= 256)
        compose_block<uint8_t>(a, smem, s_ids, E, s_scr, bmap);
    else
        compose_block<uint16_t>(a, smem, s_ids, E, s_scr, bmap);
    block_done(a, smem, s_scr, s_flag);
}

// Speculative kernel (Algorithm 3).  Wave w of block b walks chunk
// c = b*4 + w; lane j tracks the states q = j, j+64, ... (T[q] <- delta(T[q], sigma));
// the 4 chunk mappings are composed in order into the block mapping.
template <int S>
__global__ __launch_bounds__(kSpecWaves * 64) void k_spec_walk(MatchArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint16_t *s_cls = (uint16_t *)smem;                        // 512 B
    uint16_t *s_dn = (uint16_t *)(smem + 512);                 // u16 [n_dfa * C]
    const uint32_t dn_bytes = (a.img_bytes + 15) & ~15u;
    uint32_t *s_flag = (uint32_t *)(smem + a.region_bytes);   // region_bytes >= 512 + dn_bytes
    uint32_t *s_T = s_flag + 4;                                // [4][n_dfa]
    for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) s_cls[i] = a.cls[i];
    copy16((uint4 *)s_dn, (const uint4 *)a.img, dn_bytes / 16);
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
            const uint32_t b = (word_of(v, i >> 2) >> (8 * (i & 3))) & 255u;
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
    uint16_t *bm = a.block_maps + (size_t)blockIdx.x * a.map_stride;
    for (uint32_t q = threadIdx.x; q < n; q += blockDim.x) {
        uint32_t x = q;
        for (uint32_t w = 0; w < kSpecWaves; ++w) x = s_T[w * n + x];
        bm[q] = (uint16_t)x;
    }
    block_done(a, smem, s_T, s_flag);
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
// shapes of the global-table walk; each keeps its load ring in registers
// (no scratch): with 512 (1024) threads a shape fits in 256 (128)
// registers, two (four) waves per SIMD.
#define SFA_GLOBAL_SHAPES(X) \
    X(1, 64, 2, 256) X(2, 64, 2, 256) X(2, 64, 3, 256) X(4, 32, 2, 256) X(4, 32, 3, 256) X(4, 32, 4, 256) \
    X(8, 16, 2, 256) X(8, 16, 3, 256) X(8, 16, 4, 256) \
    X(1, 64, 2, 512) X(2, 64, 2, 512) X(2, 64, 3, 512) X(4, 32, 2, 512) X(4, 32, 3, 512) X(4, 32, 4, 512) \
    X(1, 64, 2, 1024) X(2, 64, 2, 1024) \
    X(1, 128, 2, 256) X(2, 128, 2, 256) X(4, 64, 2, 256) \
    X(1, 128, 2, 512) X(1, 128, 3, 512) X(1, 128, 4, 512) X(2, 128, 2, 512) X(2, 128, 3, 512) X(4, 64, 2, 512) \
    X(1, 128, 2, 1024)

bool global_shape_ok(uint32_t K, uint32_t G, uint32_t D, uint32_t TB) {
#define SFA_SHAPE_OK(k, g, d, tb) if (K == k && G == g && D == d && TB == tb) return true;
    SFA_GLOBAL_SHAPES(SFA_SHAPE_OK)
#undef SFA_SHAPE_OK
    return false;
}

bool lds_shape_ok(uint32_t K, uint32_t G, uint32_t D, uint32_t TB) {
#define SFA_SHAPE_OK(k, g, d, tb) if (K == k && G == g && D == d && TB == tb) return true;
    SFA_LDS_SHAPES(SFA_SHAPE_OK)
#undef SFA_SHAPE_OK
    return false;
}

struct Plan {
    uint32_t n_chunks = 0, blocks = 0, S = 0, K = 1, G = 16, D = 2, TB = kBlock, LPC = 1, groups = 1;
    uint64_t chunk_len = 0;
    // grid composition
    uint32_t stage_bytes = 0;   // LDS at offset 0 the finishing blocks may use for staging
    uint32_t map_stride = 0, super_blocks = 0, n_super = 1, groups1 = 1, final_groups = 1, stage1 = 0, stage2 = 0;
    size_t ws_maps = 0, ws_groups = 0, ws_bytes = 0;   // workspace offsets and size
};

// Groups for a composition of E elements: about sqrt(E) groups, so that the
// parallel phase (chains of E/G) and the serial phase (chains of G) balance,
// within the LDS scratch and at most 4096 (group, state) pairs.
uint32_t pick_groups(uint32_t E, uint32_t n_dfa) {
    uint32_t G = 1;
    while ((uint64_t)(G * 2) * (G * 2) <= E && (uint64_t)G * 2 * n_dfa * 4 <= kScratchLds &&
           (uint64_t)G * 2 * n_dfa <= 4096)
        G *= 2;
    return G;
}

// LDS bytes at offset 0 that a kernel no longer needs once its walk and
// block composition are over, usable by the grid composition for staging.
uint32_t spec_region(const sfa_table *t) {
    return std::max<uint32_t>(512 + ((2 * t->L.n_dfa * t->L.C + 15) & ~15u), kSpecStage);
}

uint32_t stage_bytes(const sfa_table *t, const Plan &P, bool speculative) {
    if (speculative) return spec_region(t);
    const uint32_t ids = P.K * P.TB * 4;
    if (P.S) return ((t->L.img[stride_index(P.S)].bytes + 15) & ~15u) + ids;
    const uint32_t row_bytes = t->L.C * t->L.next_w;
    return 512 + ((t->L.hot_rows * row_bytes + 15) & ~15u) + ids;
}

// Grid composition plan: one level when all block mappings fit the staging
// LDS at once, else runs of super_blocks blocks composed by the last block
// of each run, then the run mappings by the last run.  A level whose
// mappings do not fit reads them from global memory instead.  The control
// words sit in a fixed area at the start of every workspace that no other
// write touches, so workspaces are shared by calls with different plans.
void plan_grid(Plan &P, uint32_t n_dfa, bool ids) {
    const uint32_t B = P.blocks;
    if (ids) {
        // product mode: one u32 id per block, runs of up to kIdRun blocks
        P.map_stride = 0;
        P.super_blocks = std::max(kIdRun, (B + kMaxRuns - 1) / kMaxRuns);
        if (B <= P.super_blocks) P.super_blocks = B;
        P.n_super = (B + P.super_blocks - 1) / P.super_blocks;
        P.ws_maps = kWsHeader;
        P.ws_groups = P.ws_maps + align256((uint64_t)B * 4);
        P.ws_bytes = P.ws_groups + (P.n_super > 1 ? (size_t)P.n_super * 4 : 0);
        return;
    }
    P.map_stride = (n_dfa + 7) & ~7u;
    const uint32_t fit = P.stage_bytes / (P.map_stride * 2);   // mappings that fit in the staging LDS
    const uint32_t run = std::max(fit, 1u);
    if (B <= run) {
        P.super_blocks = B;
        P.n_super = 1;
        P.stage2 = B <= fit;
    } else {
        P.super_blocks = std::max(run, (B + kMaxRuns - 1) / kMaxRuns);
        P.n_super = (B + P.super_blocks - 1) / P.super_blocks;
        P.stage1 = P.super_blocks <= fit;
        P.stage2 = P.n_super <= fit;
        P.groups1 = pick_groups(P.super_blocks, n_dfa);
    }
    P.final_groups = pick_groups(P.n_super > 1 ? P.n_super : B, n_dfa);
    P.ws_maps = kWsHeader;
    P.ws_groups = P.ws_maps + align256((uint64_t)B * P.map_stride * 2);
    P.ws_bytes = P.ws_groups + (P.n_super > 1 ? (size_t)P.n_super * P.map_stride * 2 : 0);
}

sfa_status make_plan(const sfa_table *t, uint64_t n, uint32_t n_chunks, bool speculative, const sfa_plan *user,
                     Plan &P) {
    // a table without an LDS image is walked by the global-table kernel,
    // whose default blocks have 512 threads
    bool any_img = false;
    for (const Image &im : t->L.img) any_img |= im.present != 0;
    const bool global_walk = !speculative && !any_img;
    if (n_chunks == 0) {
        const uint64_t target = speculative ? 4096 : 1024;   // bytes per chunk at least
        // default: one block of lanes per CU
        const uint64_t per_cu = speculative ? kSpecWaves * 8 : global_walk ? kGlobalBlock : kBlock;
        const uint64_t max_chunks = (uint64_t)std::max(1u, t->num_cus) * per_cu;
        uint64_t p = std::max<uint64_t>(1, (n + target - 1) / target);
        P.n_chunks = (uint32_t)std::min(p, max_chunks);
    } else {
        P.n_chunks = n_chunks;
    }
    P.chunk_len = n ? (n + P.n_chunks - 1) / P.n_chunks : 0;
    if (speculative) {
        P.blocks = (uint32_t)((P.n_chunks + kSpecWaves - 1) / kSpecWaves);
    } else {
        // stride: the widest LDS image present, unless the plan names one
        uint32_t S = 0;
        for (uint32_t s : {4u, 2u, 1u})
            if (!S && t->L.img[stride_index(s)].present) S = s;
        // default: 2 pieces per lane, 128-byte steps, loads issued 3 steps
        // ahead (the deepest ring that stays in registers; it hides HBM
        // latency with one wave per SIMD)
        uint32_t K = 2, G = 128, D = 4, TB = 256, LPC = 1;
        const bool user_shape = user && (user->stride || user->pieces || user->load_bytes || user->depth ||
                                         user->block_threads || user->lanes_per_chunk);
        if (!user_shape && S == 4 && !global_walk && P.chunk_len <= kShortChunk) {
            // chunks of at most 4 KiB that split into whole 128-byte steps per
            // lane: the walk of one piece per lane is short, so two waves per
            // SIMD (512-thread blocks) beat more pieces per lane;
            // lanes_per_chunk fills one block per CU.  (Measured on ragged
            // chunk lengths it was no faster, and at times slower.)
            uint32_t lpc = 1;
            const uint64_t want = (uint64_t)std::max(1u, t->num_cus) * 512;
            while (lpc < 16 && (uint64_t)P.n_chunks * lpc < want) lpc *= 2;
            if (P.chunk_len % ((uint64_t)lpc * 128) == 0) K = 1, G = 128, D = 2, TB = 512, LPC = lpc;
        }
        if (user) {
            if (user->stride) {
                const int si = stride_index(user->stride);
                if (si < 0 || !t->L.img[si].present)
                    return sfa_fail(SFA_ERR_INVALID_ARG, "plan stride not available for this table");
                S = user->stride;
            }
            if (user->pieces) K = user->pieces;
            if (user->load_bytes) G = user->load_bytes;
            if (user->depth) D = user->depth;
            if (user->block_threads) TB = user->block_threads;
            if (user->lanes_per_chunk) LPC = user->lanes_per_chunk;
        }
        if (LPC == 0 || (LPC & (LPC - 1)) || LPC > 16)
            return sfa_fail(SFA_ERR_INVALID_ARG, "plan lanes_per_chunk must be a power of two <= 16");
        if (S == 0) {
            // global-table walk: default (4, 64, 2) with 512 threads (two
            // waves per SIMD share the staged rows and hide each other's
            // LDS latency; 64-byte steps visit each 128-byte line twice,
            // 32-byte steps four times, with lines evicted in between)
            if (!user || !user->pieces) K = 4;
            if (!user || !user->load_bytes) G = 64;
            if (!user || !user->depth) D = 2;
            if (!user || !user->block_threads) TB = kGlobalBlock;
            if (LPC != 1)
                return sfa_fail(SFA_ERR_INVALID_ARG, "the global-table walk uses one lane per chunk");
            if (!global_shape_ok(K, G, D, TB))
                return sfa_fail(SFA_ERR_INVALID_ARG, "plan (pieces, load_bytes, depth) not supported by the global walk");
        } else if (!lds_shape_ok(K, G, D, TB)) {
            return sfa_fail(SFA_ERR_INVALID_ARG, "plan (pieces, load_bytes, depth, block_threads) not supported");
        }
        if (LPC > TB) return sfa_fail(SFA_ERR_INVALID_ARG, "plan lanes_per_chunk exceeds block_threads");
        // short chunks: fewer pieces, then fewer lanes per chunk
        while (K > 1 && P.chunk_len < (uint64_t)LPC * K * G * 2) {
            K /= 2;
            if (S ? !lds_shape_ok(K, G, D, TB) : !global_shape_ok(K, G, D, TB)) {
                G = 64;
                D = 2;
            }
        }
        while (LPC > 1 && P.chunk_len < (uint64_t)LPC * K * G * 2) LPC /= 2;
        if (S ? !lds_shape_ok(K, G, D, TB) : !global_shape_ok(K, G, D, TB))
            return sfa_fail(SFA_ERR_INVALID_ARG, "no launch shape for this plan");
        // every piece of a full chunk is whole G-byte load groups when L is a
        // multiple of LPC * K * G (no byte-at-a-time tail); used when that
        // lengthens a chunk by at most an eighth, else L is a multiple of 16
        // (chunk starts stay 16-byte aligned).  Trailing chunks may end up
        // short or empty.
        const uint64_t unit = (uint64_t)LPC * K * G;
        const uint64_t q = P.chunk_len >= 8 * unit ? unit : 16;
        P.chunk_len = (P.chunk_len + q - 1) / q * q;
        P.S = S;
        P.K = K;
        P.G = G;
        P.D = D;
        P.TB = TB;
        P.LPC = LPC;
        P.blocks = (uint32_t)(((uint64_t)P.n_chunks * LPC + TB - 1) / TB);
        P.groups = pick_groups(P.K * TB, t->L.n_dfa);
    }
    P.stage_bytes = stage_bytes(t, P, speculative);
    plan_grid(P, t->L.n_dfa, !speculative && t->L.mul_bytes);
    return SFA_OK;
}

template <typename F>
hipError_t launch(F fn, uint32_t blocks, uint32_t threads, size_t lds, hipStream_t s, const MatchArgs &a) {
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <int S>
hipError_t dispatch_shape(uint32_t K, uint32_t G, uint32_t D, uint32_t TB, uint32_t blocks, size_t lds, hipStream_t s,
                          const MatchArgs &a) {
#define SFA_SHAPE_LAUNCH(k, g, d, tb) \
    if (K == k && G == g && D == d && TB == tb) return launch(k_sfa_lds<S, k, g, d, tb>, blocks, tb, lds, s, a);
    SFA_LDS_SHAPES(SFA_SHAPE_LAUNCH)
#undef SFA_SHAPE_LAUNCH
    return hipErrorInvalidValue;
}

template <typename NT>
hipError_t dispatch_global(uint32_t K, uint32_t G, uint32_t D, uint32_t TB, uint32_t blocks, size_t lds,
                           hipStream_t s, const MatchArgs &a) {
#define SFA_SHAPE_LAUNCH(k, g, d, tb) \
    if (K == k && G == g && D == d && TB == tb) return launch(k_sfa_global<k, g, d, NT, tb>, blocks, tb, lds, s, a);
    SFA_GLOBAL_SHAPES(SFA_SHAPE_LAUNCH)
#undef SFA_SHAPE_LAUNCH
    return hipErrorInvalidValue;
}

sfa_status common_checks(const sfa_table *t, const uint8_t *d_in, uint64_t n, void *d_ws, size_t ws_bytes,
                         sfa_result *d_out, const Plan &P) {
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
    a.groups1 = P.groups1;
    a.final_groups = P.final_groups;
    a.map_stride = P.map_stride;
    a.super_blocks = P.super_blocks;
    a.n_super = P.n_super;
    a.stage1 = P.stage1;
    a.stage2 = P.stage2;
    a.lanes_per_chunk = P.LPC;
    a.accept = t->d_base + t->L.off_acc;
    a.map = t->d_base + t->L.off_map;
    a.map_bytes = (uint32_t)std::min<uint64_t>(UINT32_MAX, (uint64_t)t->L.map_w * t->L.n_sfa * t->L.n_dfa);
    a.counter = (uint32_t *)d_ws;
    a.block_maps = (uint16_t *)((uint8_t *)d_ws + P.ws_maps);
    a.group_maps = (uint16_t *)((uint8_t *)d_ws + P.ws_groups);
    a.block_ids = (uint32_t *)((uint8_t *)d_ws + P.ws_maps);
    a.run_ids = (uint32_t *)((uint8_t *)d_ws + P.ws_groups);
    a.out = d_out;
    return a;
}

size_t scratch_lds(const Plan &P, uint32_t n_dfa) {
    const uint32_t G = std::max({P.groups, P.final_groups, P.n_super > 1 ? P.groups1 : 1u});
    return std::max<size_t>(G > 1 ? (size_t)G * n_dfa * 4 : 0, 64);   // >= one word per wave
}

}  // namespace

extern "C" sfa_status sfa_match_workspace_bytes(const sfa_table *t, uint64_t n, uint32_t n_chunks, size_t *out_bytes) {
    if (!t || !out_bytes) return sfa_fail(SFA_ERR_INVALID_ARG, "null argument");
    Plan a, b;
    sfa_status st = make_plan(t, n, n_chunks, true, nullptr, b);
    if (st != SFA_OK) return st;
    size_t bound = b.ws_bytes;
    if (t->L.n_sfa) {
        st = make_plan(t, n, n_chunks, false, nullptr, a);
        if (st != SFA_OK) return st;
        // any launch plan: at most 16 lanes per chunk in blocks of >= 256 lanes,
        // and at most one level-1 run mapping per block
        const uint64_t B = ((uint64_t)a.n_chunks * 16 + 255) / 256;
        const uint64_t ms = ((uint64_t)t->L.n_dfa + 7) & ~7ull;
        bound = std::max<size_t>(bound, kWsHeader + align256(B * ms * 2) + B * ms * 2);
    }
    *out_bytes = std::max(a.ws_bytes, bound);
    return SFA_OK;
}

extern "C" sfa_status sfa_match_ex(const sfa_table *t, const uint8_t *d_in, uint64_t n, uint32_t n_chunks,
                                   const sfa_plan *plan, void *d_ws, size_t ws_bytes, sfa_result *d_out,
                                   void *stream) {
    if (!t) return sfa_fail(SFA_ERR_INVALID_ARG, "null table");
    if (t->L.n_sfa == 0) return sfa_fail(SFA_ERR_NO_SFA, "table has no D-SFA; use sfa_match_speculative");
    Plan P;
    sfa_status st = make_plan(t, n, n_chunks, false, plan, P);
    if (st != SFA_OK) return st;
    st = common_checks(t, d_in, n, d_ws, ws_bytes, d_out, P);
    if (st != SFA_OK) return st;
    MatchArgs a = base_args(t, d_in, n, d_ws, d_out, P);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (t->L.mul_bytes) {
        a.mul = t->d_base + t->L.off_mul;
        a.mul_lds = (t->L.mul_bytes + 15) & ~15u;
        a.n_sfa = t->L.n_sfa;
    }
    if (P.S) {
        const Image &im = t->L.img[stride_index(P.S)];
        a.img = t->d_base + im.off;
        a.img_bytes = im.bytes;
        a.row_bytes = im.row_bytes;
        a.one_off = im.one_off;
        a.wide_mul = t->L.C * t->L.C;
        a.region_bytes = (im.bytes + 15) & ~15u;
        a.map_lds = a.map_bytes <= a.region_bytes;
        const size_t lds = a.region_bytes + a.mul_lds + (size_t)P.K * P.TB * 4 + 16 + scratch_lds(P, t->L.n_dfa);
        if (lds > t->lds_per_block) return sfa_fail(SFA_ERR_INVALID_ARG, "LDS plan exceeds the device limit");
        switch (P.S) {
            case 4: e = dispatch_shape<4>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a); break;
            case 2: e = dispatch_shape<2>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a); break;
            default: e = dispatch_shape<1>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a); break;
        }
    } else {
        a.img = t->d_base + t->L.off_next;
        a.cls = (const uint16_t *)(t->d_base + t->L.off_cls);
        a.row_bytes = t->L.C * t->L.next_w;
        a.hot_rows = t->L.hot_rows;
        const uint32_t hot_bytes = ((a.hot_rows * a.row_bytes) + 15) & ~15u;
        a.region_bytes = 512 + hot_bytes;
        a.map_lds = a.map_bytes <= a.region_bytes;
        const size_t lds = a.region_bytes + a.mul_lds + (size_t)P.K * P.TB * 4 + 16 + scratch_lds(P, t->L.n_dfa);
        if (lds > t->lds_per_block) return sfa_fail(SFA_ERR_INVALID_ARG, "LDS plan exceeds the device limit");
        if (t->L.next_w == 1) e = dispatch_global<uint8_t>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a);
        else if (t->L.next_w == 2) e = dispatch_global<uint16_t>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a);
        else e = dispatch_global<uint32_t>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a);
    }
    if (e != hipSuccess) return sfa_fail(SFA_ERR_HIP, std::string("walk launch: ") + hipGetErrorString(e));
    return SFA_OK;
}

extern "C" sfa_status sfa_match(const sfa_table *t, const uint8_t *d_in, uint64_t n, uint32_t n_chunks, void *d_ws,
                                size_t ws_bytes, sfa_result *d_out, void *stream) {
    return sfa_match_ex(t, d_in, n, n_chunks, nullptr, d_ws, ws_bytes, d_out, stream);
}

extern "C" sfa_status sfa_match_speculative(const sfa_table *t, const uint8_t *d_in, uint64_t n, uint32_t n_chunks,
                                            void *d_ws, size_t ws_bytes, sfa_result *d_out, void *stream) {
    if (!t) return sfa_fail(SFA_ERR_INVALID_ARG, "null table");
    Plan P;
    sfa_status st = make_plan(t, n, n_chunks, true, nullptr, P);
    if (st != SFA_OK) return st;
    st = common_checks(t, d_in, n, d_ws, ws_bytes, d_out, P);
    if (st != SFA_OK) return st;
    MatchArgs a = base_args(t, d_in, n, d_ws, d_out, P);
    a.row_bytes = t->L.C * 2;
    a.img_bytes = 2 * t->L.n_dfa * t->L.C;
    a.cls = (const uint16_t *)(t->d_base + t->L.off_dcls);
    a.img = t->d_base + t->L.off_dnext;
    const uint32_t nd = t->L.n_dfa;
    a.region_bytes = spec_region(t);
    a.map_lds = 0;
    const size_t lds = a.region_bytes + 16 + std::max<size_t>((size_t)kSpecWaves * nd * 4, scratch_lds(P, nd));
    if (lds > t->lds_per_block)
        return sfa_fail(SFA_ERR_INVALID_ARG, "DFA too large for the speculative kernel's LDS plan");
    const uint32_t S = (nd + 63) / 64;
    hipStream_t s = (hipStream_t)stream;
    const uint32_t threads = kSpecWaves * 64;
    hipError_t e;
    if (S <= 1) e = launch(k_spec_walk<1>, P.blocks, threads, lds, s, a);
    else if (S <= 2) e = launch(k_spec_walk<2>, P.blocks, threads, lds, s, a);
    else if (S <= 4) e = launch(k_spec_walk<4>, P.blocks, threads, lds, s, a);
    else if (S <= 8) e = launch(k_spec_walk<8>, P.blocks, threads, lds, s, a);
    else if (S <= 16) e = launch(k_spec_walk<16>, P.blocks, threads, lds, s, a);
    else return sfa_fail(SFA_ERR_INVALID_ARG, "speculative kernel supports at most 1024 DFA states");
    if (e != hipSuccess) return sfa_fail(SFA_ERR_HIP, std::string("speculative launch: ") + hipGetErrorString(e));
    return SFA_OK;
}
