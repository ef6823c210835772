// Host compiler: regex -> position (Glushkov) NFA -> DFA (subset construction,
// Algorithm 1, Section 2.3) -> Hopcroft minimisation -> canonical numbering ->
// byte classes -> D-SFA (correspondence construction, Algorithm 4, with the
// deterministic simplification of Section 5.1).
//
// The regex syntax is the one documented in sfa.h.

#include <algorithm>
#include <bitset>
#include <chrono>
#include <cstring>
#include <deque>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace {

constexpr int kMaxRepeat = 1000;
constexpr uint32_t kMaxPositions = 1u << 20;
constexpr uint32_t kMaxDfa = 65535;

using ByteSet = std::bitset<256>;

struct ParseErr {
    std::string msg;
};

// ---------------------------------------------------------------------------
// Parser -> AST
// ---------------------------------------------------------------------------
enum class K { Eps, Set, Cat, Alt, Star, Rep };

struct Node {
    K kind;
    ByteSet set;
    std::vector<int> kids;
    int lo = 0, hi = -1;  // Rep bounds; hi = -1 means unbounded
};

ByteSet range_set(int a, int b) {
    ByteSet s;
    for (int i = a; i <= b; ++i) s.set(i);
    return s;
}

ByteSet class_escape(char c, bool &ok) {
    ok = true;
    ByteSet digit = range_set('0', '9');
    ByteSet word = range_set('a', 'z') | range_set('A', 'Z') | digit;
    word.set('_');
    ByteSet space;
    for (char ch : std::string(" \t\n\r\f\v")) space.set((unsigned char)ch);
    switch (c) {
        case 'd': return digit;
        case 'D': return ~digit;
        case 'w': return word;
        case 'W': return ~word;
        case 's': return space;
        case 'S': return ~space;
        default: ok = false; return ByteSet();
    }
}

class Parser {
public:
    Parser(const char *s, size_t n) : s_(s), n_(n) {}

    int parse() {
        int r = alt();
        if (i_ != n_) throw ParseErr{"unbalanced ) at " + std::to_string(i_)};
        return r;
    }
    std::vector<Node> nodes;

private:
    const char *s_;
    size_t n_;
    size_t i_ = 0;

    int add(Node nd) {
        nodes.push_back(std::move(nd));
        return (int)nodes.size() - 1;
    }
    int peek() const { return i_ < n_ ? (unsigned char)s_[i_] : -1; }
    int take() {
        if (i_ >= n_) throw ParseErr{"unexpected end of pattern"};
        return (unsigned char)s_[i_++];
    }
    static bool is_digit(int c) { return c >= '0' && c <= '9'; }
    static bool is_alnum(int c) {
        return is_digit(c) || (c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z');
    }
    static int hexval(int c) {
        if (is_digit(c)) return c - '0';
        if (c >= 'a' && c <= 'f') return c - 'a' + 10;
        if (c >= 'A' && c <= 'F') return c - 'A' + 10;
        return -1;
    }

    // After a backslash.  Returns true with `byte` set for a single byte,
    // false with `set` set for a class escape.
    bool escape(int &byte, ByteSet &set) {
        int c = take();
        bool ok;
        set = class_escape((char)c, ok);
        if (ok) return false;
        switch (c) {
            case 'n': byte = 10; return true;
            case 't': byte = 9; return true;
            case 'r': byte = 13; return true;
            case 'f': byte = 12; return true;
            case 'v': byte = 11; return true;
            case '0': byte = 0; return true;
            case 'x': {
                if (i_ + 2 > n_) throw ParseErr{"bad \\x escape"};
                int h = hexval((unsigned char)s_[i_]), l = hexval((unsigned char)s_[i_ + 1]);
                if (h < 0 || l < 0) throw ParseErr{"bad \\x escape"};
                i_ += 2;
                byte = h * 16 + l;
                return true;
            }
            default: break;
        }
        if (is_alnum(c)) throw ParseErr{std::string("unknown escape \\") + (char)c};
        if (c > 127) throw ParseErr{"non-ASCII pattern character"};
        byte = c;
        return true;
    }

    // One item inside [...]: single byte (true) or class escape (false).
    bool bracket_item(int &byte, ByteSet &set) {
        int c = take();
        if (c == '\\') return escape(byte, set);
        if (c > 127) throw ParseErr{"non-ASCII pattern character"};
        byte = c;
        return true;
    }

    ByteSet bracket() {
        bool neg = false;
        if (peek() == '^') {
            neg = true;
            ++i_;
        }
        ByteSet acc;
        bool first = true;
        for (;;) {
            int c = peek();
            if (c < 0) throw ParseErr{"unterminated ["};
            if (c == ']' && !first) {
                ++i_;
                break;
            }
            first = false;
            int lo_b = 0;
            ByteSet lo_s;
            bool lo_single = bracket_item(lo_b, lo_s);
            if (peek() == '-' && i_ + 1 < n_ && s_[i_ + 1] != ']') {
                ++i_;
                int hi_b = 0;
                ByteSet hi_s;
                bool hi_single = bracket_item(hi_b, hi_s);
                if (!lo_single || !hi_single) throw ParseErr{"class escape in a range"};
                if (hi_b < lo_b) throw ParseErr{"reversed range"};
                acc |= range_set(lo_b, hi_b);
            } else if (lo_single) {
                acc.set(lo_b);
            } else {
                acc |= lo_s;
            }
        }
        return neg ? ~acc : acc;
    }

    // Try to read {n}, {n,}, {,m}, {n,m} at i_ (which points at '{').
    bool bound(int &lo, int &hi) {
        size_t j = i_ + 1;
        auto digits = [&](size_t k) {
            while (k < n_ && is_digit((unsigned char)s_[k])) ++k;
            return k;
        };
        auto to_int = [&](size_t a, size_t b) {
            long v = 0;
            for (size_t k = a; k < b; ++k) {
                v = v * 10 + (s_[k] - '0');
                if (v > 100000000L) v = 100000000L;
            }
            return (int)v;
        };
        size_t e1 = digits(j);
        if (e1 < n_ && s_[e1] == '}') {
            if (e1 == j) return false;
            lo = hi = to_int(j, e1);
            i_ = e1 + 1;
            return true;
        }
        if (e1 < n_ && s_[e1] == ',') {
            size_t e2 = digits(e1 + 1);
            if (e2 < n_ && s_[e2] == '}') {
                if (e1 == j && e2 == e1 + 1) return false;
                lo = (e1 == j) ? 0 : to_int(j, e1);
                hi = (e2 == e1 + 1) ? -1 : to_int(e1 + 1, e2);
                i_ = e2 + 1;
                return true;
            }
        }
        return false;
    }

    int alt() {
        std::vector<int> br{concat()};
        while (peek() == '|') {
            ++i_;
            br.push_back(concat());
        }
        if (br.size() == 1) return br[0];
        Node nd{K::Alt};
        nd.kids = br;
        return add(nd);
    }

    int concat() {
        std::vector<int> items;
        while (peek() >= 0 && peek() != '|' && peek() != ')') items.push_back(repeat());
        if (items.empty()) return add(Node{K::Eps});
        if (items.size() == 1) return items[0];
        Node nd{K::Cat};
        nd.kids = items;
        return add(nd);
    }

    int repeat() {
        int node = atom();
        bool quantified = false;
        for (;;) {
            int c = peek();
            int lo, hi;
            if (c == '*' || c == '+' || c == '?') {
                lo = (c == '+') ? 1 : 0;
                hi = (c == '?') ? 1 : -1;
                ++i_;
            } else if (c == '{') {
                if (!bound(lo, hi)) break;
            } else {
                break;
            }
            if (quantified) throw ParseErr{"multiple repeat at " + std::to_string(i_)};
            quantified = true;
            if (hi >= 0 && hi < lo) throw ParseErr{"bad repeat bounds"};
            if (lo > kMaxRepeat || hi > kMaxRepeat) throw ParseErr{"repeat bound too large"};
            if (lo == 0 && hi < 0) {
                Node nd{K::Star};
                nd.kids = {node};
                node = add(nd);
            } else {
                Node nd{K::Rep};
                nd.kids = {node};
                nd.lo = lo;
                nd.hi = hi;
                node = add(nd);
            }
        }
        return node;
    }

    int atom() {
        int c = take();
        if (c == '(') {
            int r = alt();
            if (peek() != ')') throw ParseErr{"missing )"};
            ++i_;
            return r;
        }
        if (c == '*' || c == '+' || c == '?')
            throw ParseErr{"nothing to repeat at " + std::to_string(i_ - 1)};
        if (c == '{') {
            --i_;
            int lo, hi;
            if (bound(lo, hi)) throw ParseErr{"nothing to repeat at " + std::to_string(i_)};
            ++i_;
            Node nd{K::Set};
            nd.set.set('{');
            return add(nd);
        }
        if (c == ')') throw ParseErr{"unbalanced )"};
        Node nd{K::Set};
        if (c == '.') {
            nd.set.set();
        } else if (c == '[') {
            nd.set = bracket();
        } else if (c == '\\') {
            int b = 0;
            ByteSet s;
            if (escape(b, s))
                nd.set.set(b);
            else
                nd.set = s;
        } else {
            if (c > 127) throw ParseErr{"non-ASCII pattern character"};
            nd.set.set(c);
        }
        return add(nd);
    }
};

// ---------------------------------------------------------------------------
// Position automaton: positions 1..P are the byte-set leaves of the AST with
// bounded repeats unrolled; position 0 is the initial state.
// ---------------------------------------------------------------------------
struct Frag {
    bool nullable;
    std::vector<uint32_t> first, last;
};

class Glushkov {
public:
    explicit Glushkov(const std::vector<Node> &nodes) : nodes_(nodes) {
        sets.emplace_back();  // position 0
        follow.emplace_back();
    }
    std::vector<ByteSet> sets;                   // byte set of each position
    std::vector<std::vector<uint32_t>> follow;   // follow[p]

    Frag build(int id) {
        const Node &nd = nodes_[id];
        switch (nd.kind) {
            case K::Eps: return Frag{true, {}, {}};
            case K::Set: {
                if (sets.size() >= kMaxPositions) throw ParseErr{"pattern too large"};
                uint32_t p = (uint32_t)sets.size();
                sets.push_back(nd.set);
                follow.emplace_back();
                return Frag{false, {p}, {p}};
            }
            case K::Cat: {
                Frag acc{true, {}, {}};
                for (int k : nd.kids) acc = cat(std::move(acc), build(k));
                return acc;
            }
            case K::Alt: {
                Frag acc{false, {}, {}};
                for (int k : nd.kids) {
                    Frag f = build(k);
                    acc.nullable = acc.nullable || f.nullable;
                    acc.first.insert(acc.first.end(), f.first.begin(), f.first.end());
                    acc.last.insert(acc.last.end(), f.last.begin(), f.last.end());
                }
                return acc;
            }
            case K::Star: return star(build(nd.kids[0]));
            case K::Rep: {
                Frag acc{true, {}, {}};
                for (int r = 0; r < nd.lo; ++r) acc = cat(std::move(acc), build(nd.kids[0]));
                if (nd.hi < 0) {
                    acc = cat(std::move(acc), star(build(nd.kids[0])));
                } else {
                    for (int r = nd.lo; r < nd.hi; ++r) {
                        Frag opt = build(nd.kids[0]);
                        opt.nullable = true;
                        acc = cat(std::move(acc), std::move(opt));
                    }
                }
                return acc;
            }
        }
        return Frag{true, {}, {}};
    }

private:
    const std::vector<Node> &nodes_;

    void link(const std::vector<uint32_t> &from, const std::vector<uint32_t> &to) {
        for (uint32_t p : from) follow[p].insert(follow[p].end(), to.begin(), to.end());
    }
    Frag cat(Frag a, Frag b) {
        link(a.last, b.first);
        Frag r;
        r.nullable = a.nullable && b.nullable;
        r.first = a.first;
        if (a.nullable) r.first.insert(r.first.end(), b.first.begin(), b.first.end());
        r.last = b.last;
        if (b.nullable) r.last.insert(r.last.end(), a.last.begin(), a.last.end());
        return r;
    }
    Frag star(Frag a) {
        link(a.last, a.first);
        a.nullable = true;
        return a;
    }
};

// ---------------------------------------------------------------------------
// DFA over a byte partition.
// ---------------------------------------------------------------------------
struct RawDfa {
    uint32_t n = 0, k = 0, q0 = 0;
    std::vector<uint32_t> delta;  // [n*k]
    std::vector<uint8_t> accept;
};

// Partition bytes by their membership pattern over the position sets.
std::vector<uint32_t> nfa_byte_classes(const std::vector<ByteSet> &sets, uint32_t &k) {
    std::vector<uint32_t> cls(256, 0);
    k = 1;
    for (size_t p = 1; p < sets.size(); ++p) {
        // split every class by membership in sets[p]
        std::vector<int> in_id(k, -1), out_id(k, -1);
        uint32_t nk = 0;
        std::vector<uint32_t> next(256);
        for (int b = 0; b < 256; ++b) {
            int &slot = sets[p].test(b) ? in_id[cls[b]] : out_id[cls[b]];
            if (slot < 0) slot = (int)nk++;
            next[b] = (uint32_t)slot;
        }
        cls.swap(next);
        k = nk;
    }
    return cls;
}

struct VecHash {
    size_t operator()(const std::vector<uint64_t> &v) const {
        uint64_t h = 1469598103934665603ull;
        for (uint64_t w : v) {
            h ^= w + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
            h *= 1099511628211ull;
        }
        return (size_t)h;
    }
};

RawDfa subset_construction(const Glushkov &g, const Frag &root, const std::vector<uint32_t> &cls,
                           uint32_t k, uint32_t dfa_cap, std::vector<std::vector<uint64_t>> *sets_out = nullptr) {
    const uint32_t P = (uint32_t)g.sets.size();  // incl. position 0
    const uint32_t W = (P + 63) / 64;
    // class masks over positions
    std::vector<uint32_t> rep(k, 256);
    for (int b = 255; b >= 0; --b) rep[cls[b]] = (uint32_t)b;
    std::vector<std::vector<uint64_t>> cmask(k, std::vector<uint64_t>(W, 0));
    for (uint32_t c = 0; c < k; ++c)
        for (uint32_t p = 1; p < P; ++p)
            if (g.sets[p].test(rep[c])) cmask[c][p >> 6] |= 1ull << (p & 63);
    std::vector<uint64_t> lastmask(W, 0);
    for (uint32_t p : root.last) lastmask[p >> 6] |= 1ull << (p & 63);

    // follow(0) = first(root)
    std::vector<std::vector<uint32_t>> follow = g.follow;
    follow[0] = root.first;

    RawDfa d;
    d.k = k;
    std::unordered_map<std::vector<uint64_t>, uint32_t, VecHash> index;
    std::vector<std::vector<uint64_t>> states;
    std::vector<uint64_t> start(W, 0);
    start[0] = 1;  // {0}
    index.emplace(start, 0);
    states.push_back(start);
    std::vector<uint64_t> fol(W), nxt(W);
    for (size_t i = 0; i < states.size(); ++i) {  // FIFO worklist
        std::fill(fol.begin(), fol.end(), 0);
        const std::vector<uint64_t> S = states[i];
        bool acc = false;
        for (uint32_t w = 0; w < W; ++w) {
            uint64_t bits = S[w];
            if (bits & lastmask[w]) acc = true;
            while (bits) {
                uint32_t p = w * 64 + (uint32_t)__builtin_ctzll(bits);
                bits &= bits - 1;
                for (uint32_t q : follow[p]) fol[q >> 6] |= 1ull << (q & 63);
            }
        }
        if ((S[0] & 1) && root.nullable) acc = true;
        d.accept.push_back(acc ? 1 : 0);
        for (uint32_t c = 0; c < k; ++c) {
            for (uint32_t w = 0; w < W; ++w) nxt[w] = fol[w] & cmask[c][w];
            auto it = index.find(nxt);
            uint32_t id;
            if (it == index.end()) {
                if (states.size() >= dfa_cap)
                    throw sfa_status(SFA_ERR_DFA_TOO_LARGE);
                id = (uint32_t)states.size();
                index.emplace(nxt, id);
                states.push_back(nxt);
            } else {
                id = it->second;
            }
            d.delta.push_back(id);
        }
    }
    d.n = (uint32_t)states.size();
    if (sets_out) sets_out->swap(states);
    return d;
}

// Hopcroft's partition refinement.  Returns block id per state.
std::vector<uint32_t> hopcroft(const RawDfa &d, uint32_t &nblocks) {
    const uint32_t n = d.n, k = d.k;
    // inverse transitions in CSR form per symbol
    std::vector<uint32_t> pstart((size_t)k * (n + 1), 0), plist((size_t)k * n);
    for (uint32_t c = 0; c < k; ++c) {
        uint32_t *st = &pstart[(size_t)c * (n + 1)];
        for (uint32_t q = 0; q < n; ++q) st[d.delta[(size_t)q * k + c] + 1]++;
        for (uint32_t t = 0; t < n; ++t) st[t + 1] += st[t];
        std::vector<uint32_t> fill(st, st + n);
        for (uint32_t q = 0; q < n; ++q) {
            uint32_t t = d.delta[(size_t)q * k + c];
            plist[(size_t)c * n + fill[t]++] = q;
        }
    }
    std::vector<uint32_t> elems(n), loc(n), blk(n);
    std::vector<uint32_t> first, end, mid;
    // initial partition: accepting first, then rejecting (empty parts dropped)
    uint32_t pos = 0;
    for (int want = 1; want >= 0; --want) {
        uint32_t b0 = pos;
        for (uint32_t q = 0; q < n; ++q)
            if ((int)d.accept[q] == want) {
                elems[pos] = q;
                loc[q] = pos++;
            }
        if (pos > b0) {
            uint32_t id = (uint32_t)first.size();
            for (uint32_t i = b0; i < pos; ++i) blk[elems[i]] = id;
            first.push_back(b0);
            end.push_back(pos);
            mid.push_back(b0);
        }
    }
    std::vector<uint8_t> inw;  // [block * k + c]
    std::vector<std::pair<uint32_t, uint32_t>> work;
    inw.assign(first.size() * k, 0);
    {
        uint32_t smaller = 0;
        if (first.size() == 2 && end[1] - first[1] < end[0] - first[0]) smaller = 1;
        for (uint32_t c = 0; c < k; ++c) {
            work.emplace_back(smaller, c);
            inw[(size_t)smaller * k + c] = 1;
        }
    }
    std::vector<uint32_t> X, touched;
    while (!work.empty()) {
        auto [A, c] = work.back();
        work.pop_back();
        inw[(size_t)A * k + c] = 0;
        X.clear();
        const uint32_t *st = &pstart[(size_t)c * (n + 1)];
        const uint32_t *pl = &plist[(size_t)c * n];
        for (uint32_t i = first[A]; i < end[A]; ++i) {
            uint32_t t = elems[i];
            for (uint32_t j = st[t]; j < st[t + 1]; ++j) X.push_back(pl[j]);
        }
        touched.clear();
        for (uint32_t q : X) {
            uint32_t B = blk[q];
            if (mid[B] == first[B]) touched.push_back(B);
            uint32_t a = loc[q], b = mid[B]++;
            uint32_t other = elems[b];
            std::swap(elems[a], elems[b]);
            loc[other] = a;
            loc[q] = b;
        }
        for (uint32_t B : touched) {
            if (mid[B] == end[B]) {
                mid[B] = first[B];
                continue;
            }
            uint32_t N = (uint32_t)first.size();
            first.push_back(first[B]);
            end.push_back(mid[B]);
            mid.push_back(first[B]);
            first[B] = mid[B];
            mid[B] = first[B];
            for (uint32_t i = first[N]; i < end[N]; ++i) blk[elems[i]] = N;
            inw.resize(first.size() * k, 0);
            uint32_t szB = end[B] - first[B], szN = end[N] - first[N];
            for (uint32_t cc = 0; cc < k; ++cc) {
                if (inw[(size_t)B * k + cc]) {
                    work.emplace_back(N, cc);
                    inw[(size_t)N * k + cc] = 1;
                } else {
                    uint32_t S = szN <= szB ? N : B;
                    work.emplace_back(S, cc);
                    inw[(size_t)S * k + cc] = 1;
                }
            }
        }
    }
    nblocks = (uint32_t)first.size();
    return blk;
}

struct Timer {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double seconds() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

// Hash table of mapping rows (open addressing over row ids).
class RowTable {
public:
    RowTable(const std::vector<uint16_t> &rows, uint32_t width) : rows_(rows), w_(width) {
        slots_.assign(1024, UINT32_MAX);
    }
    // Returns id of `row` if present, else UINT32_MAX with `slot` set.
    uint32_t find(const uint16_t *row, uint64_t h, size_t &slot) const {
        size_t mask = slots_.size() - 1;
        size_t i = (size_t)h & mask;
        for (;;) {
            uint32_t id = slots_[i];
            if (id == UINT32_MAX) {
                slot = i;
                return UINT32_MAX;
            }
            if (std::memcmp(&rows_[(size_t)id * w_], row, w_ * sizeof(uint16_t)) == 0) return id;
            i = (i + 1) & mask;
        }
    }
    void insert_at(size_t slot, uint32_t id, uint32_t count) {
        slots_[slot] = id;
        if ((size_t)count * 2 > slots_.size()) rehash();
    }
    static uint64_t hash(const uint16_t *row, uint32_t w) {
        uint64_t h = 0x243f6a8885a308d3ull;
        for (uint32_t i = 0; i < w; ++i) {
            h ^= row[i];
            h *= 0x9e3779b97f4a7c15ull;
            h ^= h >> 29;
        }
        return h;
    }

private:
    void rehash() {
        std::vector<uint32_t> old;
        old.swap(slots_);
        slots_.assign(old.size() * 2, UINT32_MAX);
        size_t mask = slots_.size() - 1;
        for (uint32_t id : old) {
            if (id == UINT32_MAX) continue;
            size_t i = (size_t)hash(&rows_[(size_t)id * w_], w_) & mask;
            while (slots_[i] != UINT32_MAX) i = (i + 1) & mask;
            slots_[i] = id;
        }
    }
    const std::vector<uint16_t> &rows_;
    uint32_t w_;
    std::vector<uint32_t> slots_;
};

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" sfa_status sfa_compile(const char *pattern, size_t pattern_len, uint32_t sfa_cap,
                                  uint32_t dfa_cap, sfa_compiled **out) {
    if (!out || (!pattern && pattern_len)) return sfa_fail(SFA_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (dfa_cap == 0 || dfa_cap > kMaxDfa) dfa_cap = kMaxDfa;
    sfa_compiled *c = new (std::nothrow) sfa_compiled();
    if (!c) return sfa_fail(SFA_ERR_HOST_ALLOC, "out of host memory");
    try {
        Timer t_dfa;
        Parser parser(pattern ? pattern : "", pattern_len);
        int root_id = parser.parse();
        Glushkov g(parser.nodes);
        Frag root = g.build(root_id);
        c->n_positions = (uint32_t)g.sets.size() - 1;
        uint32_t k = 0;
        std::vector<uint32_t> ncls = nfa_byte_classes(g.sets, k);
        RawDfa raw = subset_construction(g, root, ncls, k, dfa_cap);
        uint32_t nb = 0;
        std::vector<uint32_t> blk = hopcroft(raw, nb);
        // minimal DFA over NFA byte classes
        std::vector<uint32_t> mdelta((size_t)nb * k);
        std::vector<uint8_t> macc(nb);
        for (uint32_t q = 0; q < raw.n; ++q) {
            for (uint32_t a = 0; a < k; ++a) mdelta[(size_t)blk[q] * k + a] = blk[raw.delta[(size_t)q * k + a]];
            macc[blk[q]] = raw.accept[q];
        }
        // canonical numbering: breadth first from q0, bytes 0..255 ascending
        std::vector<uint32_t> newid(nb, UINT32_MAX), order;
        uint32_t s0 = blk[raw.q0];
        newid[s0] = 0;
        order.push_back(s0);
        for (size_t i = 0; i < order.size(); ++i) {
            uint32_t q = order[i];
            for (int b = 0; b < 256; ++b) {
                uint32_t t = mdelta[(size_t)q * k + ncls[b]];
                if (newid[t] == UINT32_MAX) {
                    newid[t] = (uint32_t)order.size();
                    order.push_back(t);
                }
            }
        }
        const uint32_t n = (uint32_t)order.size();
        // final byte classes: bytes with identical columns of the minimal DFA,
        // numbered by smallest member byte
        std::vector<std::vector<uint32_t>> col_of_nclass(k, std::vector<uint32_t>(n));
        for (uint32_t a = 0; a < k; ++a)
            for (uint32_t i = 0; i < n; ++i) col_of_nclass[a][i] = newid[mdelta[(size_t)order[i] * k + a]];
        std::vector<int> fcls_of_ncls(k, -1);
        std::vector<uint32_t> fcls_rep;
        uint32_t C = 0;
        for (int b = 0; b < 256; ++b) {
            uint32_t a = ncls[b];
            if (fcls_of_ncls[a] < 0) {
                int found = -1;
                for (uint32_t f = 0; f < C; ++f)
                    if (col_of_nclass[ncls[fcls_rep[f]]] == col_of_nclass[a]) {
                        found = (int)f;
                        break;
                    }
                if (found < 0) {
                    found = (int)C++;
                    fcls_rep.push_back((uint32_t)b);
                }
                fcls_of_ncls[a] = found;
            }
            c->byte_class[b] = (uint8_t)fcls_of_ncls[a];
        }
        c->n_dfa = n;
        c->n_classes = C;
        c->q0 = 0;
        c->dfa_next.resize((size_t)n * C);
        c->dfa_accept.resize(n);
        for (uint32_t i = 0; i < n; ++i) {
            c->dfa_accept[i] = macc[order[i]];
            for (uint32_t f = 0; f < C; ++f)
                c->dfa_next[(size_t)i * C + f] = col_of_nclass[ncls[fcls_rep[f]]][i];
        }
        c->dfa_seconds = t_dfa.seconds();

        // D-SFA: f_next(q) = delta(f(q), c), worklist first in first out
        Timer t_sfa;
        if (sfa_cap > 0) {
            std::vector<std::vector<uint16_t>> cols(C, std::vector<uint16_t>(n));
            for (uint32_t f = 0; f < C; ++f)
                for (uint32_t q = 0; q < n; ++q) cols[f][q] = (uint16_t)c->dfa_next[(size_t)q * C + f];
            std::vector<uint16_t> rows;
            rows.reserve((size_t)n * 64);
            for (uint32_t q = 0; q < n; ++q) rows.push_back((uint16_t)q);
            RowTable tab(rows, n);
            size_t slot;
            tab.find(rows.data(), RowTable::hash(rows.data(), n), slot);
            tab.insert_at(slot, 0, 1);
            std::vector<uint32_t> snext;
            std::vector<uint16_t> tmp(n);
            uint32_t m = 1;
            bool over = false;
            for (uint32_t s = 0; s < m && !over; ++s) {
                for (uint32_t f = 0; f < C; ++f) {
                    const uint16_t *row = &rows[(size_t)s * n];
                    const uint16_t *col = cols[f].data();
                    for (uint32_t q = 0; q < n; ++q) tmp[q] = col[row[q]];
                    uint64_t h = RowTable::hash(tmp.data(), n);
                    uint32_t id = tab.find(tmp.data(), h, slot);
                    if (id == UINT32_MAX) {
                        if (m >= sfa_cap) {
                            over = true;
                            break;
                        }
                        id = m++;
                        rows.insert(rows.end(), tmp.begin(), tmp.end());
                        tab.insert_at(slot, id, m);
                    }
                    snext.push_back(id);
                }
            }
            if (over) {
                c->over_cap = 1;
                c->n_sfa = 0;
            } else {
                c->n_sfa = m;
                c->sfa_next.swap(snext);
                c->sfa_map.assign(rows.begin(), rows.end());
            }
        }
        c->sfa_seconds = t_sfa.seconds();
    } catch (const ParseErr &e) {
        delete c;
        return sfa_fail(SFA_ERR_PARSE, e.msg);
    } catch (sfa_status st) {
        delete c;
        return sfa_fail(st, "DFA exceeds " + std::to_string(dfa_cap) + " states");
    } catch (const std::bad_alloc &) {
        delete c;
        return sfa_fail(SFA_ERR_HOST_ALLOC, "out of host memory");
    }
    *out = c;
    return SFA_OK;
}

// N-SFA (Definition 3 on the position automaton, Algorithm 4 with
// correspondences): states are mappings f: Q -> P(Q) stored as P rows of W
// words, delta_s(f, c)(q) = U_{p in f(q)} delta(p, c); FIFO worklist,
// classes ascending, identity = state 0.  For the tables, each state f is
// also given by its action on the reachable subsets S of the subset
// automaton, f^(S) = U_{q in S} f(q): with f = f_w, f^(S) = delta_D(S, w)
// is again reachable, (f . g)^ = g^ o f^, and S_fin = f_fin^(I).  The
// subset automaton plays the DFA's part, so every matcher applies.
extern "C" sfa_status sfa_compile_nsfa(const char *pattern, size_t pattern_len, uint32_t nsfa_cap,
                                       uint32_t dfa_cap, sfa_compiled **out) {
    if (!out || (!pattern && pattern_len)) return sfa_fail(SFA_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (dfa_cap == 0 || dfa_cap > kMaxDfa) dfa_cap = kMaxDfa;
    sfa_compiled *c = new (std::nothrow) sfa_compiled();
    if (!c) return sfa_fail(SFA_ERR_HOST_ALLOC, "out of host memory");
    try {
        Timer t_dfa;
        Parser parser(pattern ? pattern : "", pattern_len);
        int root_id = parser.parse();
        Glushkov g(parser.nodes);
        Frag root = g.build(root_id);
        const uint32_t P = (uint32_t)g.sets.size(), W = (P + 63) / 64;
        c->n_positions = P - 1;
        uint32_t k = 0;
        std::vector<uint32_t> ncls = nfa_byte_classes(g.sets, k);
        std::vector<std::vector<uint64_t>> subsets;
        RawDfa raw = subset_construction(g, root, ncls, k, dfa_cap, &subsets);
        if (k > 256) throw sfa_status(SFA_ERR_INVALID_ARG);
        c->nsfa = 1;
        c->n_nfa = P;
        c->words = W;
        c->n_dfa = raw.n;
        c->n_classes = k;
        c->q0 = 0;
        for (int b = 0; b < 256; ++b) c->byte_class[b] = (uint8_t)ncls[b];
        c->dfa_next = raw.delta;
        c->dfa_accept = raw.accept;
        c->nfa_sets.resize((size_t)raw.n * W);
        for (uint32_t d = 0; d < raw.n; ++d) std::copy(subsets[d].begin(), subsets[d].end(), &c->nfa_sets[(size_t)d * W]);
        c->nfa_final.assign(W, 0);
        for (uint32_t p : root.last) c->nfa_final[p >> 6] |= 1ull << (p & 63);
        if (root.nullable) c->nfa_final[0] |= 1;
        c->dfa_seconds = t_dfa.seconds();

        Timer t_sfa;
        if (nsfa_cap > 0) {
            // delta(p, c) as W-word sets
            std::vector<uint32_t> rep(k, 256);
            for (int b = 255; b >= 0; --b) rep[ncls[b]] = (uint32_t)b;
            std::vector<uint64_t> dq((size_t)P * k * W, 0);
            for (uint32_t p = 0; p < P; ++p) {
                const std::vector<uint32_t> &succ = p == 0 ? root.first : g.follow[p];
                for (uint32_t a = 0; a < k; ++a)
                    for (uint32_t t : succ)
                        if (g.sets[t].test(rep[a])) dq[((size_t)p * k + a) * W + (t >> 6)] |= 1ull << (t & 63);
            }
            const size_t FW = (size_t)P * W;   // words of one correspondence
            std::vector<uint64_t> maps(FW, 0);
            for (uint32_t q = 0; q < P; ++q) maps[(size_t)q * W + (q >> 6)] = 1ull << (q & 63);
            std::unordered_map<std::vector<uint64_t>, uint32_t, VecHash> index;
            index.emplace(std::vector<uint64_t>(maps.begin(), maps.end()), 0);
            std::vector<uint32_t> snext;
            std::vector<uint64_t> tmp(FW);
            uint32_t m = 1;
            bool over = false;
            for (uint32_t s = 0; s < m && !over; ++s) {
                for (uint32_t a = 0; a < k; ++a) {
                    std::fill(tmp.begin(), tmp.end(), 0);
                    const uint64_t *f = &maps[(size_t)s * FW];
                    for (uint32_t q = 0; q < P; ++q)
                        for (uint32_t w = 0; w < W; ++w) {
                            uint64_t bits = f[(size_t)q * W + w];
                            while (bits) {
                                const uint32_t p = w * 64 + (uint32_t)__builtin_ctzll(bits);
                                bits &= bits - 1;
                                const uint64_t *row = &dq[((size_t)p * k + a) * W];
                                for (uint32_t x = 0; x < W; ++x) tmp[(size_t)q * W + x] |= row[x];
                            }
                        }
                    auto it = index.find(tmp);
                    uint32_t id;
                    if (it == index.end()) {
                        if (m >= nsfa_cap) {
                            over = true;
                            break;
                        }
                        id = m++;
                        index.emplace(tmp, id);
                        maps.insert(maps.end(), tmp.begin(), tmp.end());
                    } else {
                        id = it->second;
                    }
                    snext.push_back(id);
                }
            }
            if (over) {
                c->over_cap = 1;
                c->n_sfa = 0;
            } else {
                // action of every state on the reachable subsets
                std::unordered_map<std::vector<uint64_t>, uint32_t, VecHash> sub_index;
                for (uint32_t d = 0; d < raw.n; ++d) sub_index.emplace(subsets[d], d);
                c->sfa_map.resize((size_t)m * raw.n);
                std::vector<uint64_t> img(W);
                for (uint32_t s = 0; s < m; ++s) {
                    const uint64_t *f = &maps[(size_t)s * FW];
                    for (uint32_t d = 0; d < raw.n; ++d) {
                        std::fill(img.begin(), img.end(), 0);
                        for (uint32_t w = 0; w < W; ++w) {
                            uint64_t bits = subsets[d][w];
                            while (bits) {
                                const uint32_t q = w * 64 + (uint32_t)__builtin_ctzll(bits);
                                bits &= bits - 1;
                                for (uint32_t x = 0; x < W; ++x) img[x] |= f[(size_t)q * W + x];
                            }
                        }
                        auto it = sub_index.find(img);
                        if (it == sub_index.end()) throw sfa_status(SFA_ERR_INVALID_ARG);   // cannot happen
                        c->sfa_map[(size_t)s * raw.n + d] = it->second;
                    }
                }
                c->n_sfa = m;
                c->sfa_next.swap(snext);
            }
        }
        c->sfa_seconds = t_sfa.seconds();
    } catch (const ParseErr &e) {
        delete c;
        return sfa_fail(SFA_ERR_PARSE, e.msg);
    } catch (sfa_status st) {
        delete c;
        return sfa_fail(st, st == SFA_ERR_DFA_TOO_LARGE ? "subset automaton exceeds " + std::to_string(dfa_cap) + " states"
                                                        : "N-SFA construction failed");
    } catch (const std::bad_alloc &) {
        delete c;
        return sfa_fail(SFA_ERR_HOST_ALLOC, "out of host memory");
    }
    *out = c;
    return SFA_OK;
}

// On-the-fly D-SFA: runs over the sample from the identity, constructing a
// transition the first time a run takes it (the correspondence construction
// of Algorithm 4 driven by the text instead of a worklist).
extern "C" sfa_status sfa_compiled_build_lazy(sfa_compiled *c, const uint8_t *sample, uint64_t sample_bytes,
                                              uint32_t start_every, uint32_t walk_bytes, uint32_t max_states) {
    if (!c || (sample_bytes && !sample)) return sfa_fail(SFA_ERR_INVALID_ARG, "null argument");
    if (c->nsfa) return sfa_fail(SFA_ERR_INVALID_ARG, "on-the-fly construction takes a D-SFA compilation");
    if (c->n_sfa && !c->lazy) return sfa_fail(SFA_ERR_INVALID_ARG, "the compilation already has a complete D-SFA");
    if (start_every == 0 || walk_bytes == 0 || max_states == 0 || max_states > 16777214u)
        return sfa_fail(SFA_ERR_INVALID_ARG, "start_every, walk_bytes and max_states must be positive "
                                             "(max_states at most 16777214)");
    try {
        Timer t_sfa;
        const uint32_t n = c->n_dfa, C = c->n_classes;
        std::vector<std::vector<uint16_t>> cols(C, std::vector<uint16_t>(n));
        for (uint32_t f = 0; f < C; ++f)
            for (uint32_t q = 0; q < n; ++q) cols[f][q] = (uint16_t)c->dfa_next[(size_t)q * C + f];
        std::vector<uint16_t> rows;
        for (uint32_t q = 0; q < n; ++q) rows.push_back((uint16_t)q);
        RowTable tab(rows, n);
        size_t slot;
        tab.find(rows.data(), RowTable::hash(rows.data(), n), slot);
        tab.insert_at(slot, 0, 1);
        std::vector<uint32_t> snext(C, SFA_UNBUILT);
        std::vector<uint16_t> tmp(n);
        uint32_t m = 1;
        for (uint64_t s0 = 0; s0 < sample_bytes; s0 += start_every) {
            const uint64_t s1 = std::min<uint64_t>(sample_bytes, s0 + walk_bytes);
            uint32_t f = 0;
            for (uint64_t i = s0; i < s1; ++i) {
                const uint32_t k = c->byte_class[sample[i]];
                uint32_t t = snext[(size_t)f * C + k];
                if (t == SFA_UNBUILT) {
                    const uint16_t *row = &rows[(size_t)f * n];
                    const uint16_t *col = cols[k].data();
                    for (uint32_t q = 0; q < n; ++q) tmp[q] = col[row[q]];
                    t = tab.find(tmp.data(), RowTable::hash(tmp.data(), n), slot);
                    if (t == UINT32_MAX) {
                        if (m >= max_states) break;   // no room: this run ends here
                        t = m++;
                        rows.insert(rows.end(), tmp.begin(), tmp.end());
                        snext.insert(snext.end(), C, SFA_UNBUILT);
                        tab.insert_at(slot, t, m);
                    }
                    snext[(size_t)f * C + k] = t;
                }
                f = t;
            }
        }
        // close the transitions among the states built: an edge no run took
        // is filled in when its target mapping is one of them (no new
        // state), so a walk leaves the built set only for a mapping no run
        // reached
        for (uint32_t f = 0; f < m; ++f)
            for (uint32_t k = 0; k < C; ++k) {
                if (snext[(size_t)f * C + k] != SFA_UNBUILT) continue;
                const uint16_t *row = &rows[(size_t)f * n];
                const uint16_t *col = cols[k].data();
                for (uint32_t q = 0; q < n; ++q) tmp[q] = col[row[q]];
                const uint32_t t = tab.find(tmp.data(), RowTable::hash(tmp.data(), n), slot);
                if (t != UINT32_MAX) snext[(size_t)f * C + k] = t;
            }
        c->n_sfa = m;
        c->lazy = 1;
        c->sfa_next.swap(snext);
        c->sfa_map.assign(rows.begin(), rows.end());
        c->sfa_seconds = t_sfa.seconds();
    } catch (const std::bad_alloc &) {
        return sfa_fail(SFA_ERR_HOST_ALLOC, "out of host memory");
    }
    return SFA_OK;
}

extern "C" sfa_status sfa_compiled_nsfa_sets(const sfa_compiled *c, sfa_nsfa_sets *out) {
    if (!c || !out) return sfa_fail(SFA_ERR_INVALID_ARG, "null argument");
    if (!c->nsfa) return sfa_fail(SFA_ERR_INVALID_ARG, "not an N-SFA compilation");
    out->n_nfa = c->n_nfa;
    out->words = c->words;
    out->sets = c->nfa_sets.data();
    out->final_set = c->nfa_final.data();
    return SFA_OK;
}

extern "C" sfa_status sfa_compiled_info(const sfa_compiled *c, sfa_compile_info *out) {
    if (!c || !out) return sfa_fail(SFA_ERR_INVALID_ARG, "null argument");
    out->n_dfa = c->n_dfa;
    out->n_sfa = c->n_sfa;
    out->n_classes = c->n_classes;
    out->q0 = c->q0;
    out->n_positions = c->n_positions;
    out->sfa_over_cap = c->over_cap;
    out->dfa_seconds = c->dfa_seconds;
    out->sfa_seconds = c->sfa_seconds;
    out->sfa_lazy = c->lazy;
    out->reserved = 0;
    return SFA_OK;
}

extern "C" sfa_status sfa_compiled_desc(const sfa_compiled *c, sfa_table_desc *out) {
    if (!c || !out) return sfa_fail(SFA_ERR_INVALID_ARG, "null argument");
    out->abi_version = SFA_ABI_VERSION;
    out->n_dfa = c->n_dfa;
    out->n_sfa = c->n_sfa;
    out->n_classes = c->n_classes;
    out->q0 = c->q0;
    out->byte_class = c->byte_class;
    out->dfa_next = c->dfa_next.data();
    out->dfa_accept = c->dfa_accept.data();
    out->sfa_next = c->n_sfa ? c->sfa_next.data() : nullptr;
    out->sfa_map = c->n_sfa ? c->sfa_map.data() : nullptr;
    return SFA_OK;
}

extern "C" void sfa_compiled_free(sfa_compiled *c) { delete c; }
