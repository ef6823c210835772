// HIP runtime of the SFA matcher for gfx950: table packing and loading, the
// walk kernel (Algorithm 5, Section 5.2), the speculative kernel
// (Algorithm 3, Section 3) and the ordered composition of chunk mappings
// (reverse composition, Section 2.1; Lemma 1 and Theorem 2, Section 4.3).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "walk.h"
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

using namespace sfa_rt;

namespace sfa_rt {

hipError_t prepare_kernel(const void *fn) {
    static std::mutex mu;
    static std::set<std::pair<const void *, int>> ready;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    if (ready.count({fn, dev})) return hipSuccess;
    hipFuncAttributes attr;
    e = hipFuncGetAttributes(&attr, fn);
    if (e != hipSuccess) return e;
    if (attr.sharedSizeBytes != 0) return hipErrorInvalidKernelFile;   // dynamic LDS would not start at 0
    int max_lds = 0;
    e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    if (e != hipSuccess) return e;
    ready.insert({fn, dev});
    return hipSuccess;
}

}  // namespace sfa_rt



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
            if (d->sfa_next[i] >= d->n_sfa && d->sfa_next[i] != SFA_UNBUILT)
                return sfa_fail(SFA_ERR_INVALID_ARG, "sfa_next out of range");
        const uint64_t nm = (uint64_t)d->n_sfa * d->n_dfa;
        for (uint64_t i = 0; i < nm; ++i)
            if (d->sfa_map[i] >= d->n_dfa) return sfa_fail(SFA_ERR_INVALID_ARG, "sfa_map out of range");
        for (uint32_t q = 0; q < d->n_dfa; ++q)
            if (d->sfa_map[q] != q) return sfa_fail(SFA_ERR_INVALID_ARG, "D-SFA state 0 is not the identity");
    }
    return SFA_OK;
}

// True when some transition of d's D-SFA is unbuilt (an on-the-fly D-SFA).
bool is_partial(const sfa_table_desc *d) {
    const uint64_t ns = (uint64_t)d->n_sfa * d->n_classes;
    for (uint64_t i = 0; i < ns; ++i)
        if (d->sfa_next[i] == SFA_UNBUILT) return true;
    return false;
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
    if (m == 0 || (uint64_t)m * C * n > (1u << 24) || is_partial(d)) return false;
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

// Share of the profiling walk's visits beyond the hot rows above which the
// global walk uses vector re-walks (C3's keyword D-SFA: 3e-5; r500: most).
constexpr double kVectorShare = 0.002;

// LDS bytes the walk kernel needs besides the image: piece states + scratch.
constexpr uint32_t kWalkExtraLds = kMaxIds * 4 + 16 + kScratchLds;

Layout plan(const sfa_table_desc *d, const sfa_load_options *o, uint32_t lds_limit) {
    Layout L;
    L.n_dfa = d->n_dfa;
    L.n_sfa = d->n_sfa;
    L.C = d->n_classes;
    L.q0 = d->q0;
    L.partial = d->n_sfa && is_partial(d) ? 1 : 0;
    // a partial D-SFA keeps the largest id of the entry width for unbuilt
    // transitions
    const uint64_t ids = (uint64_t)d->n_sfa + L.partial;
    L.next_w = ids <= 256 ? 1 : ids <= 65536 ? 2 : 4;
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
    const bool allow_lds = d->n_sfa && !L.partial && !(o && o->force_global);
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
    const bool any_img = L.img[0].present || L.img[1].present || L.img[2].present;
    if (d->n_sfa && !any_img && L.C <= kGlobalMaxClasses) {
        // global-table walk: a hot image of as many leading rows as the LDS
        // (or the caller's budget for the rows) holds, plus the cold row (and
        // for a partial D-SFA the parking row after it).  After the walk the
        // piece ids and the composition scratch reuse the image's region, so
        // only the product table and the flag word are kept apart.  Entries
        // are row indices in u16.
        const uint64_t rb = 2ull * L.C;
        const uint64_t extra_rows = 1 + L.partial;
        const uint64_t keep = ((L.mul_bytes + 15) & ~15u) + 16 + 256 + extra_rows * rb;
        const uint64_t room = lds_limit > keep ? lds_limit - keep : 0;
        const uint64_t hb = std::min<uint64_t>((o && o->lds_budget) ? o->lds_budget : room, room);
        const uint64_t h = std::min<uint64_t>({(uint64_t)d->n_sfa, hb / rb, 65536 - extra_rows});
        L.hot_rows = (uint32_t)h;
        L.off_himg = off;
        L.himg_bytes = (uint32_t)(256 + (h + extra_rows) * rb);
        off = align256(off + L.himg_bytes);
    }
    L.total = off;
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
                if (w == SFA_UNBUILT) continue;
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
                for (uint32_t cc = 0; cc < C; ++cc) {
                    const uint32_t w = d->sfa_next[(uint64_t)comp[i] * C + cc];
                    if (w == SFA_UNBUILT || on[w] != 2) { closed = false; break; }
                }
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
std::vector<uint32_t> visit_order(const sfa_table_desc *d, const sfa_load_options *o, uint32_t H,
                                  double *cold_share) {
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
                if (s == SFA_UNBUILT) s = 0;   // unbuilt: the walker starts over
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
                if (s == SFA_UNBUILT) s = 0;
                ++count[s];
            }
        }
    }
    // closed sets rank above every visited state (a count no walk reaches)
    const uint64_t top = ~0ull;
    const std::vector<uint32_t> traps = trap_states(d);
    std::vector<uint8_t> is_trap(m, 0);
    for (size_t i = 0; i < traps.size(); ++i) {
        count[traps[i]] = top - i;
        is_trap[traps[i]] = 1;
    }
    std::vector<uint32_t> ids(m);
    for (uint32_t i = 0; i < m; ++i) ids[i] = i;
    std::stable_sort(ids.begin() + 1, ids.end(), [&](uint32_t a, uint32_t b) { return count[a] > count[b]; });
    std::vector<uint32_t> perm(m);   // old id -> new id
    for (uint32_t i = 0; i < m; ++i) perm[ids[i]] = i;
    // share of the profiling walk's visits that land beyond the first H rows
    double all = 0, cold = 0;
    for (uint32_t i = 0; i < m; ++i) {
        if (is_trap[i]) continue;
        all += (double)count[i];
        if (perm[i] >= H) cold += (double)count[i];
    }
    if (cold_share) *cold_share = all > 0 ? cold / all : 0.0;
    return perm;
}

template <typename T>
void put(std::vector<uint8_t> &img, uint64_t off, uint64_t i, T v) {
    std::memcpy(&img[off + i * sizeof(T)], &v, sizeof(T));
}

void pack(const sfa_table_desc *d0, const sfa_load_options *o, Layout &L, std::vector<uint8_t> &img) {
    img.assign(L.total, 0);
    const uint32_t C = L.C;
    // renumbered copies of the D-SFA arrays (new id = perm[old id])
    sfa_table_desc dd = *d0;
    std::vector<uint32_t> rnext, rmap;
    if (L.renumbered) {
        double cold_share = 0;
        const std::vector<uint32_t> perm = visit_order(d0, o, L.hot_rows, &cold_share);
        // a walk that often leaves the hot rows re-walks its cold words with
        // vector loads (many pieces of a wave at once) rather than one lane
        // at a time
        L.vector_redo = L.himg_bytes && L.hot_rows < d0->n_sfa && cold_share > kVectorShare ? 1 : 0;
        const uint32_t m = d0->n_sfa, n = d0->n_dfa;
        rnext.resize((uint64_t)m * C);
        rmap.resize((uint64_t)m * n);
        for (uint32_t s = 0; s < m; ++s) {
            const uint32_t t = perm[s];
            for (uint32_t c = 0; c < C; ++c) {
                const uint32_t u = d0->sfa_next[(uint64_t)s * C + c];
                rnext[(uint64_t)t * C + c] = u == SFA_UNBUILT ? u : perm[u];
            }
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
        uint32_t v = d->sfa_next[i];   // SFA_UNBUILT becomes the largest id of the width
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
    if (L.himg_bytes) {
        // hot image of the global-table walk: doubled class indices (the
        // column byte offsets), then rows 0..H-1 and the cold row H, entries
        // u (u < H) or H; a partial D-SFA adds the parking row H + 1, whose
        // entries are H + 1, and its unbuilt entries in rows < H are H (the
        // scalar walk through the global table finds them unbuilt there)
        const uint32_t H = L.hot_rows, last = H + L.partial;
        for (int b = 0; b < 256; ++b) img[L.off_himg + b] = (uint8_t)(2 * d->byte_class[b]);
        const uint64_t rows = L.off_himg + 256;
        for (uint32_t r = 0; r <= last; ++r)
            for (uint32_t c = 0; c < C; ++c) {
                const uint32_t u = r < H ? d->sfa_next[(uint64_t)r * C + c] : r;
                put<uint16_t>(img, rows, (uint64_t)r * C + c, (uint16_t)(r < H ? std::min(u, H) : u));
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
    out->partial = t->L.partial;
    out->vector_redo = t->L.vector_redo;
    return SFA_OK;
}

extern "C" sfa_status sfa_free_table(sfa_table *t) {
    delete t;
    return SFA_OK;
}

namespace {

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


bool special_shape(uint32_t K, uint32_t G, uint32_t D, uint32_t TB) {
#define SFA_SHAPE_OK(k, g, d, tb) if (K == k && G == g && D == d && TB == tb) return true;
    SFA_SPECIAL_SHAPES(SFA_SHAPE_OK)
#undef SFA_SHAPE_OK
    return false;
}

// A partial D-SFA has kernels for the special shapes only; a table with
// vector re-walks uses them for those shapes and the plain kernel otherwise.
bool global_shape_ok(uint32_t K, uint32_t G, uint32_t D, uint32_t TB, bool partial) {
    if (partial) return special_shape(K, G, D, TB);
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
    size_t ws_park = 0;         // partial D-SFA: park records (one per piece), after the rest
    uint32_t group_lds = 0;     // global walk: block-composition groups in the free LDS region
};

// Groups for a composition of E elements: about sqrt(E) groups, so that the
// parallel phase (chains of E/G) and the serial phase (chains of G) balance,
// within `scratch` bytes of LDS and at most `max_pairs` (group, state) pairs.
uint32_t pick_groups(uint32_t E, uint32_t n_dfa, uint64_t scratch = kScratchLds, uint64_t max_pairs = 4096) {
    uint32_t G = 1;
    while ((uint64_t)(G * 2) * (G * 2) <= E && (uint64_t)G * 2 * n_dfa * 4 <= scratch &&
           (uint64_t)G * 2 * n_dfa <= max_pairs)
        G *= 2;
    return G;
}

// LDS bytes at offset 0 that a kernel no longer needs once its walk and
// block composition are over, usable by the grid composition for staging.
uint32_t spec_region(const sfa_table *t) {
    return std::max<uint32_t>(512 + ((2 * t->L.n_dfa * t->L.C + 15) & ~15u), kSpecStage);
}

// LDS of the global-table walk: the hot image's region [0, region), whose
// end takes the piece ids and the composition scratch once the walk is over,
// leaving [0, free) for staging.
struct GlobalLds {
    uint32_t region, free;
};
GlobalLds global_lds(const sfa_table *t, const Plan &P) {
    const uint32_t tail = P.K * P.TB * 4 + kScratchLds;
    const uint32_t region = std::max(((t->L.himg_bytes + 15) & ~15u), tail);
    return {region, region - tail};
}

uint32_t stage_bytes(const sfa_table *t, const Plan &P, bool speculative) {
    if (speculative) return spec_region(t);
    const uint32_t ids = P.K * P.TB * 4;
    if (P.S) return ((t->L.img[stride_index(P.S)].bytes + 15) & ~15u) + ids;
    return global_lds(t, P).free;
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
    // Global-table walk: the default shape is (2, 128, 1) in 1024-thread
    // blocks ("wide") when the input fills one such block per CU with chunks
    // of at least 1 KiB; else, and for complete D-SFAs with vector re-walks,
    // (4, 128, 1) in 512-thread blocks.  Measured on keyword text (ms, wide
    // against 512): 4 GiB 1.61 / 1.73, 1 GiB 0.534 / 0.616, 256 MiB 0.181 /
    // 0.215; 64 MiB 0.194 / 0.147 (half as many blocks as CUs).  On-the-fly
    // D-SFA of 60 keywords, 1 GiB: 8.9 / 13.1 ms; r500's complete D-SFA with
    // vector re-walks, 1 GiB: 1.42 / 1.35 ms.
    const uint64_t cus = std::max(1u, t->num_cus);
    const bool wide = global_walk && !(t->L.vector_redo && !t->L.partial) && n >= cus * kGlobalBlock * 1024;
    if (n_chunks == 0) {
        const uint64_t target = speculative ? 4096 : 1024;   // bytes per chunk at least
        // default: one block of lanes per CU
        // (the global-table walk: several blocks per CU, run one after
        // another, which balances the CUs' end times better.  Wide: four,
        // two or one, the most that keep chunks of at least 2 KiB; measured
        // on 4 GiB of keyword text, blocks per CU 2: 1.695 ms, 3: 1.708, 4:
        // 1.61-1.69, 4.5: 1.78, 5: 1.75; on 1 GiB 1: 0.54, 2: 0.534, 4:
        // 0.651.  512-thread blocks: blocks per CU 1: 1.99 ms, 2: 1.98, 3:
        // 1.88, 4: 1.79, 5: 1.73, 6: 1.76, 8: 1.89 on 4 GiB; five only when
        // its chunks still hold at least 8 whole 512-byte steps of four
        // pieces (the chunk length then rounds to whole steps); else four,
        // which splits power-of-two inputs into whole steps: 1 GiB r500 with
        // five, pieces ending in single bytes, ran at half the rate)
        const uint64_t p = std::max<uint64_t>(1, (n + target - 1) / target);
        uint64_t per_cu = speculative ? kSpecWaves * 8 : global_walk ? 5 * kGlobalSpecialBlock : kLdsBlock;
        if (wide) {
            uint64_t b = 4;
            while (b > 1 && n / (cus * kGlobalBlock * b) < 2048) b /= 2;
            per_cu = b * kGlobalBlock;
        } else if (global_walk && (n + cus * per_cu - 1) / (cus * per_cu) < 8 * 512) {
            per_cu = 4 * kGlobalSpecialBlock;
        }
        P.n_chunks = (uint32_t)std::min(p, cus * per_cu);
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
        // default: 2 pieces per lane, 128-byte steps, loads issued 2 steps
        // ahead, 512-thread blocks: two waves per SIMD share the one staged
        // table and hide each other's LDS latency (4 GiB (a|b)*a(a|b){4}:
        // 0.85 ms against 0.97 ms with (2, 128, 4, 256), one wave per SIMD
        // with a 4-deep ring)
        uint32_t K = 2, G = 128, D = 3, TB = kLdsBlock, LPC = 1;
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
            // a plan that names a shape but not its block size: the block
            // size that supports it
            if (S && !user->block_threads && !lds_shape_ok(K, G, D, TB))
                for (uint32_t tb : {256u, 512u, 1024u})
                    if (lds_shape_ok(K, G, D, tb)) {
                        TB = tb;
                        break;
                    }
        }
        if (LPC == 0 || (LPC & (LPC - 1)) || LPC > 16)
            return sfa_fail(SFA_ERR_INVALID_ARG, "plan lanes_per_chunk must be a power of two <= 16");
        if (S == 0) {
            // global-table walk: default (2, 128, 1) with 1024 threads when
            // wide: four waves per SIMD, two pieces each, share the staged
            // rows and hide each other's LDS latency (4 GiB keyword text:
            // 1.61 ms against 1.73 ms with (4, 128, 1) in 512-thread blocks,
            // two waves of four pieces); else (4, 128, 1) with 512 threads.
            // The rolling ring requests every 128-byte line whole (64-byte
            // steps read a line in two visits, between which it leaves the
            // L2: 1.94x the input bytes fetched, against 1.03x).
            if (!user || !user->pieces) K = wide ? 2 : 4;
            if (!user || !user->load_bytes) G = 128;
            if (!user || !user->depth) D = 1;
            if (!user || !user->block_threads) {
                TB = wide ? kGlobalBlock : kGlobalSpecialBlock;
                // a plan that names a shape but not its block size: the block
                // size that supports it
                if (!global_shape_ok(K, G, D, TB, t->L.partial))
                    for (uint32_t tb : {512u, 256u, 1024u})
                        if (global_shape_ok(K, G, D, tb, t->L.partial)) {
                            TB = tb;
                            break;
                        }
            }
            if (LPC != 1)
                return sfa_fail(SFA_ERR_INVALID_ARG, "the global-table walk uses one lane per chunk");
            if (!global_shape_ok(K, G, D, TB, t->L.partial))
                return sfa_fail(SFA_ERR_INVALID_ARG, "plan (pieces, load_bytes, depth) not supported by the global walk");
        } else if (!lds_shape_ok(K, G, D, TB)) {
            return sfa_fail(SFA_ERR_INVALID_ARG, "plan (pieces, load_bytes, depth, block_threads) not supported");
        }
        if (LPC > TB) return sfa_fail(SFA_ERR_INVALID_ARG, "plan lanes_per_chunk exceeds block_threads");
        // short chunks: fewer pieces, then fewer lanes per chunk
        while (K > 1 && P.chunk_len < (uint64_t)LPC * K * G * 2) {
            K /= 2;
            if (S ? !lds_shape_ok(K, G, D, TB) : !global_shape_ok(K, G, D, TB, t->L.partial)) {
                G = 64;
                D = 2;
            }
        }
        while (LPC > 1 && P.chunk_len < (uint64_t)LPC * K * G * 2) LPC /= 2;
        if (S ? !lds_shape_ok(K, G, D, TB) : !global_shape_ok(K, G, D, TB, t->L.partial))
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
        if (S == 0 && !t->L.mul_bytes) {
            // global walk whose mapping rows stay in global memory: the
            // block composition's groups go to the LDS the hot image frees,
            // so there can be more of them, with shorter chains of global
            // reads (C3: 16 groups of 128 pieces -> 32 of 64; measured 1.86 ->
            // 1.78 ms; 64 groups of 32, 24 chains per thread: no faster)
            const GlobalLds g = global_lds(t, P);
            if ((uint64_t)t->L.map_w * t->L.n_sfa * t->L.n_dfa > g.free) {
                P.group_lds = 1;
                P.groups = pick_groups(P.K * TB, t->L.n_dfa, g.free, (uint64_t)TB * kGroupPairsPerThread);
            }
        }
    }
    P.stage_bytes = stage_bytes(t, P, speculative);
    plan_grid(P, t->L.n_dfa, !speculative && t->L.mul_bytes);
    if (!speculative && t->L.partial) {
        P.ws_park = align256(P.ws_bytes);
        P.ws_bytes = P.ws_park + (size_t)P.blocks * P.K * P.TB * sizeof(ParkRec);
    }
    return SFA_OK;
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
        // partial D-SFA (global-table walk, one lane per chunk): park records
        // for blocks of up to 1024 lanes and 4 pieces per lane
        if (t->L.partial)
            bound = align256(bound) + (((uint64_t)a.n_chunks + 1024) / 256 + 1) * 256 * 4 * sizeof(ParkRec);
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
        if (!t->L.himg_bytes)
            return sfa_fail(SFA_ERR_NO_SFA, "the global-table walk takes at most 128 byte classes; "
                                            "use sfa_match_speculative");
        a.img = t->d_base + t->L.off_himg;
        a.img_bytes = t->L.himg_bytes;
        a.gtab = t->d_base + t->L.off_next;
        if (t->L.partial) {
            a.partial = 1;
            a.park = (ParkRec *)((uint8_t *)d_ws + P.ws_park);
            a.dnext = (const uint16_t *)(t->d_base + t->L.off_dnext);
            a.cls = (const uint16_t *)(t->d_base + t->L.off_dcls);
        }
        a.n_classes = t->L.C;
        a.hot_rows = t->L.hot_rows;
        a.cold = t->L.hot_rows;
        const GlobalLds g = global_lds(t, P);
        a.region_bytes = g.free;
        a.mul_off = g.region;
        a.group_lds = P.group_lds;
        a.map_lds = a.map_bytes <= a.region_bytes;
        const size_t lds = (size_t)g.region + a.mul_lds + 16;
        if (lds > t->lds_per_block) return sfa_fail(SFA_ERR_INVALID_ARG, "LDS plan exceeds the device limit");
        const bool vec = t->L.vector_redo && special_shape(P.K, P.G, P.D, P.TB);
        if (t->L.partial) {
            if (t->L.next_w == 1)
                e = vec ? dispatch_special<uint8_t, true, true>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a)
                        : dispatch_special<uint8_t, true, false>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a);
            else if (t->L.next_w == 2)
                e = vec ? dispatch_special<uint16_t, true, true>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a)
                        : dispatch_special<uint16_t, true, false>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a);
            else
                e = vec ? dispatch_special<uint32_t, true, true>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a)
                        : dispatch_special<uint32_t, true, false>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a);
        } else if (vec) {
            if (t->L.next_w == 1) e = dispatch_special<uint8_t, false, true>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a);
            else if (t->L.next_w == 2) e = dispatch_special<uint16_t, false, true>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a);
            else e = dispatch_special<uint32_t, false, true>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a);
        } else if (t->L.next_w == 1) {
            e = dispatch_global<uint8_t>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a);
        } else if (t->L.next_w == 2) {
            e = dispatch_global<uint16_t>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a);
        } else {
            e = dispatch_global<uint32_t>(P.K, P.G, P.D, P.TB, P.blocks, lds, s, a);
        }
    }
    if (e != hipSuccess) return sfa_fail(SFA_ERR_HIP, std::string("walk launch: ") + hipGetErrorString(e));
    return SFA_OK;
}

extern "C" sfa_status sfa_match(const sfa_table *t, const uint8_t *d_in, uint64_t n, uint32_t n_chunks, void *d_ws,
                                size_t ws_bytes, sfa_result *d_out, void *stream) {
    return sfa_match_ex(t, d_in, n, n_chunks, nullptr, d_ws, ws_bytes, d_out, stream);
}

// ---------------------------------------------------------------------------
// sfa_match_noalloc: sfa_match with the library's own workspace.  The
// workspace is a file-scope device array (one copy per device, held until
// the process ends); its address on a device is taken once, with that device
// current, and the host never passes the array's name to a kernel.
// ---------------------------------------------------------------------------
namespace {

static __device__ __align__(256) uint8_t scratch[SFA_NOALLOC_WORKSPACE_BYTES];

__global__ void k_zero_words(uint32_t *p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

std::mutex g_scratch_mu;
std::map<int, uint8_t *> g_scratch;   // device -> address of scratch on that device

// Address of the device's scratch array; on the first call for a device the
// control words (the part that must start at zero) are cleared on `stream`
// with a fill kernel.
sfa_status device_scratch(int dev, hipStream_t stream, uint8_t **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) {
        *out = it->second;
        return SFA_OK;
    }
    void *ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || ((uintptr_t)ptr & 255)) return sfa_fail(SFA_ERR_HIP, "scratch symbol address is not 256-byte aligned");
    hipLaunchKernelGGL(k_zero_words, dim3(4), dim3(256), 0, stream, (uint32_t *)ptr, (uint32_t)(kWsHeader / 4));
    HIP_TRY(hipGetLastError());
    g_scratch[dev] = (uint8_t *)ptr;
    *out = (uint8_t *)ptr;
    return SFA_OK;
}

}  // namespace

extern "C" sfa_status sfa_match_noalloc(const sfa_table *t, const uint8_t *d_in, uint64_t n, uint32_t n_chunks,
                                        sfa_result *d_out, void *stream) {
    if (!t) return sfa_fail(SFA_ERR_INVALID_ARG, "null table");
    if (t->L.n_sfa == 0) return sfa_fail(SFA_ERR_NO_SFA, "table has no D-SFA; use sfa_match_speculative");
    Plan P;
    sfa_status st = make_plan(t, n, n_chunks, false, nullptr, P);
    if (st != SFA_OK) return st;
    if (P.ws_bytes > SFA_NOALLOC_WORKSPACE_BYTES)
        return sfa_fail(SFA_ERR_INVALID_ARG, "this call needs " + std::to_string(P.ws_bytes) +
                                                 " workspace bytes, more than sfa_match_noalloc holds (" +
                                                 std::to_string((unsigned long long)SFA_NOALLOC_WORKSPACE_BYTES) +
                                                 "); use sfa_match with a caller workspace");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    uint8_t *ws = nullptr;
    st = device_scratch(dev, (hipStream_t)stream, &ws);
    if (st != SFA_OK) return st;
    return sfa_match_ex(t, d_in, n, n_chunks, nullptr, ws, SFA_NOALLOC_WORKSPACE_BYTES, d_out, stream);
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
