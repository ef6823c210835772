/*
 * sfa.h -- C ABI of the MI355X (gfx950) simultaneous-finite-automaton matcher.
 *
 * Method: Sin'ya, Matsuzaki, Sassa, "Simultaneous Finite Automata: An
 * Efficient Data-Parallel Model for Regular Expression Matching" (ICPP 2013).
 *
 *   - A D-SFA state is a transformation f: Q -> Q of the DFA's states
 *     (Definition 3, Section 4.1, with singleton images).
 *   - Reading a byte is one table lookup f <- delta_s[f, sigma], starting from
 *     the identity f_I (Algorithm 5, Section 5.2).
 *   - Chunk results compose by reverse composition (f . g)(q) = g(f(q))
 *     (Section 2.1), which is associative, so the input may be split anywhere
 *     (Lemma 1 and Theorem 2, Section 4.3).
 *   - The answer is f_fin(q0) and whether it is an accepting DFA state.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *   - Every call returns sfa_status; SFA_OK is 0.  No call aborts the process,
 *     throws across the ABI or prints.  sfa_last_error() returns a message for
 *     the calling thread's last failure.
 *   - "d_" pointers are device pointers (HIP device memory on the current
 *     device); all other pointers are host pointers.
 *   - stream is a hipStream_t passed as void* (NULL = the default stream).
 *     Device work is enqueued on it asynchronously; results are valid once
 *     the stream has been synchronised.
 *   - The caller owns all device memory: inputs, outputs, workspaces and the
 *     table buffer.  The library never allocates device memory.  Library
 *     handles (sfa_compiled, sfa_table) are host objects.
 *   - Sizes and offsets are 64-bit: an input may exceed 4 GiB.
 *   - States are reported in the canonical numbering of the minimal complete
 *     DFA: breadth-first from the start state (id 0) following bytes 0..255 in
 *     ascending order, each state numbered when first reached.
 *   - Thread safety: distinct handles may be used from distinct threads; a
 *     loaded table may be used by many streams at once.  Calls that share one
 *     workspace must not overlap in time.
 *
 * Regex syntax (whole-input membership, Definition of L(A), Section 2.2):
 *   bytes are the alphabet; "." is any byte (newline too); [..] and [^..]
 *   with ranges; escapes \n \t \r \f \v \0 \xHH \d \D \w \W \s \S and a
 *   backslash before punctuation; ( ) | * + ? {n} {n,} {,m} {n,m} (bounds at
 *   most 1000; a "{" that does not begin a valid bound is a literal);
 *   empty alternatives are allowed; stacked quantifiers are errors.
 *   A search is written with explicit ".*" on both sides.
 */
#ifndef SFA_H
#define SFA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SFA_ABI_VERSION 2u

typedef enum sfa_status {
    SFA_OK = 0,
    SFA_ERR_INVALID_ARG = 1,       /* null pointer, bad size, out-of-range table entry */
    SFA_ERR_PARSE = 2,             /* regex syntax error (message via sfa_last_error) */
    SFA_ERR_DFA_TOO_LARGE = 3,     /* subset construction exceeded the DFA state limit */
    SFA_ERR_OVER_CAP = 4,          /* D-SFA exceeds the state cap */
    SFA_ERR_NO_DEVICE = 5,         /* no HIP device visible */
    SFA_ERR_UNSUPPORTED_ARCH = 6,  /* current device is not gfx950 */
    SFA_ERR_BUFFER_TOO_SMALL = 7,  /* device buffer or workspace smaller than required */
    SFA_ERR_HIP = 8,               /* a HIP runtime call failed (message has the HIP error) */
    SFA_ERR_NO_SFA = 9,            /* no D-SFA the walk can take: use the speculative matcher */
    SFA_ERR_HOST_ALLOC = 10        /* host memory allocation failed */
} sfa_status;

/* Result of one match: final canonical DFA state and its acceptance. */
typedef struct sfa_result {
    uint32_t state;
    uint32_t accept;               /* 1 if state is accepting, else 0 */
} sfa_result;

const char *sfa_status_string(sfa_status s);
const char *sfa_last_error(void);
uint32_t    sfa_abi_version(void);

/* ------------------------------------------------------------------------
 * Host compiler: regex -> minimal canonical DFA -> byte classes -> D-SFA.
 *
 *   Position (Glushkov) NFA, subset construction (Algorithm 1, Section 2.3)
 *   over byte classes, Hopcroft minimisation, canonical renumbering, then the
 *   correspondence construction with the deterministic simplification
 *   (Algorithm 4, Section 5.1): worklist first-in first-out, classes in
 *   ascending order, the identity mapping is D-SFA state 0.
 *
 *   sfa_cap: maximum number of D-SFA states (identity included).  If the
 *   construction exceeds it, or sfa_cap is 0, sfa_compile still succeeds with
 *   the DFA only (info.n_sfa == 0); such a table is matched with
 *   sfa_match_speculative.  dfa_cap bounds the subset construction
 *   (SFA_ERR_DFA_TOO_LARGE beyond it; 0 = 65535, the maximum).
 * ---------------------------------------------------------------------- */
typedef struct sfa_compiled sfa_compiled;

typedef struct sfa_compile_info {
    uint32_t n_dfa;        /* states of the minimal complete DFA (sink included) */
    uint32_t n_sfa;        /* D-SFA states, identity included; 0 if not built */
    uint32_t n_classes;    /* byte classes (coarsest partition with equal DFA columns) */
    uint32_t q0;           /* start state: always 0 in the canonical numbering */
    uint32_t n_positions;  /* positions of the Glushkov NFA */
    uint32_t sfa_over_cap; /* 1 if the D-SFA construction stopped at the cap */
    double   dfa_seconds;  /* host time of parse + NFA + DFA + minimisation */
    double   sfa_seconds;  /* host time of the D-SFA construction */
    uint32_t sfa_lazy;     /* 1: the D-SFA was built on the fly (sfa_compiled_build_lazy) */
    uint32_t reserved;
} sfa_compile_info;

sfa_status sfa_compile(const char *pattern, size_t pattern_len, uint32_t sfa_cap,
                       uint32_t dfa_cap, sfa_compiled **out);
sfa_status sfa_compiled_info(const sfa_compiled *c, sfa_compile_info *out);
void       sfa_compiled_free(sfa_compiled *c);

/* On-the-fly D-SFA (Section 5.1, the remark that on-the-fly construction
 * carries over from the subset construction to the correspondence
 * construction): for a D-SFA compilation without a D-SFA (over its cap, or
 * sfa_cap 0), build only the states that walks over sample reach.  The
 * sample is walked in runs of walk_bytes starting every start_every bytes,
 * each from the identity, the way the matchers start every piece; a
 * transition a run takes for the first time is constructed then (state
 * f' = f followed by the DFA transition, looked up among the states built so
 * far), and at max_states states (identity included) construction stops
 * and a run that needs a new state ends there.  Then every transition no run
 * took is filled in when its target mapping is among the states built;
 * the others stay unbuilt: SFA_UNBUILT in the descriptor's sfa_next.  The partial D-SFA
 * replaces the compilation's empty one (info.n_sfa = states built,
 * info.sfa_lazy = 1) and is loaded like a complete one (sfa_load_table).
 * The matchers walk it with the global-table walk: a piece that reaches an
 * unbuilt transition stops at its last built state f and position p, and its
 * mapping is f followed, for every start state, by the DFA over the rest of
 * the piece from p (Algorithm 3 for that piece); it composes like any other.
 *   Limits: max_states in [1, 16777214]; start_every, walk_bytes >= 1.
 *   SFA_ERR_INVALID_ARG for an N-SFA compilation or one that already has a
 *   complete D-SFA; calling it again rebuilds from the new sample. */
#define SFA_UNBUILT 0xFFFFFFFFu
sfa_status sfa_compiled_build_lazy(sfa_compiled *c, const uint8_t *sample, uint64_t sample_bytes,
                                   uint32_t start_every, uint32_t walk_bytes, uint32_t max_states);

/* N-SFA compilation: the SFA of Definition 3 built from the regex's position
 * automaton (Glushkov; state 0 initial, states 1.. the byte-set leaves in
 * left-to-right order with bounded repeats written out), by Algorithm 4
 * over correspondences f: Q -> P(Q) (Section 5.1); nsfa_cap bounds its
 * states (0: do not build it; over the cap n_sfa is 0 and sfa_over_cap 1).
 *   The compiled object has the same shape as a D-SFA compilation, so it is
 *   loaded with sfa_compiled_desc / sfa_load_table and matched with every
 *   entry point: its "DFA" is the subset automaton of the NFA (the sets of
 *   NFA states reachable from I, numbered in breadth-first order over the
 *   NFA's byte classes), sfa_next is the N-SFA transition table and
 *   sfa_map[f][S] is the subset U_{q in S} f(q), which is again reachable.
 *   A match result's state is then the index of S_fin = U_{q in I} f_fin(q)
 *   (Algorithm 5), and sfa_compiled_nsfa_sets gives the NFA states of every
 *   index; accept = [S_fin meets F].
 *   sfa_compile_info.n_dfa counts the subsets, n_sfa the N-SFA states. */
sfa_status sfa_compile_nsfa(const char *pattern, size_t pattern_len, uint32_t nsfa_cap,
                            uint32_t dfa_cap, sfa_compiled **out);

typedef struct sfa_nsfa_sets {
    uint32_t n_nfa;             /* states of the position automaton */
    uint32_t words;             /* 64-bit words per state set: ceil(n_nfa / 64) */
    const uint64_t *sets;       /* [n_dfa * words]: bit q of set d = NFA state q is in subset d */
    const uint64_t *final_set;  /* [words]: F */
} sfa_nsfa_sets;

/* The subsets of an N-SFA compilation (pointers into c; valid while c
 * lives).  SFA_ERR_INVALID_ARG for a D-SFA compilation. */
sfa_status sfa_compiled_nsfa_sets(const sfa_compiled *c, sfa_nsfa_sets *out);

/* Host arrays describing a DFA and (optionally) its D-SFA.
 *   byte_class[256]             class id (< n_classes) of each byte value
 *   dfa_next[n_dfa*n_classes]   delta(q, c) at [q*n_classes + c]
 *   dfa_accept[n_dfa]           0/1
 *   sfa_next[n_sfa*n_classes]   delta_s(f, c); state 0 must be the identity;
 *                               SFA_UNBUILT marks a transition of a partial
 *                               (on-the-fly) D-SFA that was not constructed
 *   sfa_map[n_sfa*n_dfa]        f(q) at [f*n_dfa + q]
 * n_sfa == 0 means no D-SFA (sfa_next, sfa_map may be NULL).
 * Limits: n_dfa <= 65535, n_sfa <= 16777215, 1 <= n_classes <= 256, q0 < n_dfa. */
typedef struct sfa_table_desc {
    uint32_t abi_version;
    uint32_t n_dfa, n_sfa, n_classes, q0;
    const uint8_t  *byte_class;
    const uint32_t *dfa_next;
    const uint8_t  *dfa_accept;
    const uint32_t *sfa_next;
    const uint32_t *sfa_map;
} sfa_table_desc;

/* Descriptor whose arrays point into c; valid while c lives. */
sfa_status sfa_compiled_desc(const sfa_compiled *c, sfa_table_desc *out);

/* ------------------------------------------------------------------------
 * Device tables.
 *
 *   sfa_table_device_bytes: size of the device buffer sfa_load_table needs.
 *   sfa_load_table: validates every entry (out-of-range values and a state 0
 *     that is not the identity give SFA_ERR_INVALID_ARG), packs the arrays
 *     into the layout the kernels read (narrowest entry width; the walk table
 *     is copied into LDS at kernel start when it fits the LDS budget, else it
 *     is read from global memory through L2) and enqueues one host-to-device
 *     copy into d_buf on stream.  The packed host image is owned by the
 *     handle, so desc's arrays may be freed on return.  d_buf must stay
 *     allocated, and unmodified, while the handle is used.
 *   opts may be NULL (defaults).  force_global = 1 keeps the walk table in
 *   global memory even when it would fit LDS.  A D-SFA whose walk table does
 *   not fit is walked with its most visited rows staged in LDS (as many as
 *   fill the LDS, or as lds_budget bytes of rows hold; u16 row indices, so
 *   at most 65,535 rows) and the rest read from global memory; to choose
 *   those rows the loader renumbers the D-SFA states by visit count in a
 *   profiling walk over profile_sample (host bytes like the input) or,
 *   without a sample, over uniformly random byte classes.  Renumbering
 *   changes only internal ids: results are DFA states and never depend on
 *   it.  That global-table walk takes at most 128 byte classes; sfa_match
 *   returns SFA_ERR_NO_SFA for a larger table that does not fit LDS (the
 *   speculative matcher handles it).  A partial D-SFA (some SFA_UNBUILT
 *   transitions) is always walked that way, without the product table: an
 *   unbuilt transition reads as a reserved id in the global table and as a
 *   parking row in the hot image, and the piece finishes as described at
 *   sfa_compiled_build_lazy (the workspace then also holds one 16-byte record
 *   per piece).  Every device offset of the loader and
 *   the kernels is 64-bit: walk tables of 4 GiB or more are valid.
 *   Product table: the D-SFA states are closed under reverse composition
 *   (f_u . f_v = f_uv, Lemma 1 in Section 4.3; they form the monoid of
 *   Section 7.1), so for a D-SFA of at most 128
 *   states the loader tabulates mul[a][b] = the id of f_a . f_b and the
 *   matchers compose chunk results as state ids (one table lookup per
 *   composition) instead of as mappings (n_dfa lookups).  It is built only
 *   when every state is reachable from the identity and the mapping rows
 *   agree with the transitions (sfa_map[sfa_next[s][c]] equals sfa_map[s]
 *   followed by the DFA transition on class c); no_product = 1 skips it.
 *   sfa_free_table frees the host handle only; the caller frees d_buf after
 *   work that uses it has finished.
 * ---------------------------------------------------------------------- */
typedef struct sfa_table sfa_table;

typedef struct sfa_load_options {
    uint32_t force_global;   /* 0: LDS when it fits; 1: walk tables read from global memory */
    uint32_t lds_budget;     /* bytes of LDS the walk table (or its hot rows) may take; 0 = default */
    uint32_t renumber;       /* 0: renumber states by visit count when the table is walked from
                                global memory; 1: always; 2: never */
    uint32_t no_product;     /* 1: do not build the product table (compositions use the mappings) */
    const uint8_t *profile_sample;  /* host bytes for the profiling walk, or NULL */
    uint64_t profile_bytes;
} sfa_load_options;

typedef struct sfa_table_info {
    uint32_t n_dfa, n_sfa, n_classes, q0;
    uint32_t next_bytes;     /* width of a walk-table entry: 1, 2 or 4 */
    uint32_t map_bytes;      /* width of a mapping entry: 1, 2 or 4 */
    uint32_t table_in_lds;   /* 1 if the walk table is staged into LDS */
    uint32_t hot_rows;       /* global-table walk: D-SFA rows staged in LDS (0 = none) */
    uint32_t strides;        /* bit s set: stride-s LDS walk tables are present (s = 1, 2, 4) */
    uint32_t product_table;  /* 1: compositions reduce D-SFA ids through the product table */
    uint64_t device_bytes;   /* bytes used in d_buf */
    uint32_t partial;        /* 1: some D-SFA transitions are unbuilt (on-the-fly D-SFA) */
    uint32_t vector_redo;    /* 1: the profiling walk spent more than 0.2 % of its visits beyond the
                                hot rows, so the global-table walk re-walks the words of many cold
                                pieces of a wave at once with vector loads */
} sfa_table_info;

sfa_status sfa_table_device_bytes(const sfa_table_desc *desc, const sfa_load_options *opts,
                                  size_t *out_bytes);
sfa_status sfa_load_table(const sfa_table_desc *desc, const sfa_load_options *opts,
                          void *d_buf, size_t d_bytes, void *stream, sfa_table **out);
sfa_status sfa_table_get_info(const sfa_table *t, sfa_table_info *out);
sfa_status sfa_free_table(sfa_table *t);

/* ------------------------------------------------------------------------
 * Single-stream matching (Algorithm 5, Section 5.2).
 *
 *   d_in[0..n) is split into n_chunks consecutive chunks; chunk c's D-SFA
 *   state is computed from f_I and the chunk results are composed in text
 *   order; the result is f_fin(q0).  The speculative matcher cuts chunks
 *   [c*L, min((c+1)*L, n)) with L = ceil(n / n_chunks).  The SFA walk
 *   rounds L up (to a multiple of the bytes one lane loads per step when
 *   that lengthens a chunk by at most an eighth, else to a multiple of 16)
 *   and moves every boundary after the first back by d_in's misalignment,
 *   so full chunks start 16-byte aligned and hold whole load steps; the
 *   last chunks may be short or empty.  Any split gives the same result
 *   (Theorem 2).  One lane owns one chunk (or lanes_per_chunk lanes share
 *   it) and may walk it as several interleaved pieces; n_chunks = 0 lets
 *   the library choose.  n_chunks > n is legal (empty chunks are the
 *   identity); n = 0 gives (q0, accept(q0)).  Any alignment of d_in is
 *   accepted.
 *
 *   Workspace: sfa_match_workspace_bytes() bytes of device memory (enough
 *   for sfa_match, sfa_match_speculative and sfa_match_ex with any plan at
 *   the same n and n_chunks), which must be zero-filled before its first
 *   use; each call leaves its control words zero again, so a workspace is
 *   reused without clearing.  It holds the per-block mappings of the grid
 *   composition.  Calls sharing a workspace must not overlap.  d_out
 *   receives one sfa_result.
 * ---------------------------------------------------------------------- */
sfa_status sfa_match_workspace_bytes(const sfa_table *t, uint64_t n, uint32_t n_chunks,
                                     size_t *out_bytes);
sfa_status sfa_match(const sfa_table *t, const uint8_t *d_in, uint64_t n, uint32_t n_chunks,
                     void *d_ws, size_t ws_bytes, sfa_result *d_out, void *stream);

/* Launch plan of the walk (every field 0 = library choice).  None of them
 * changes the result (any division of the input is valid, Theorem 2).
 *   stride      bytes consumed per transition-table lookup: 1, 2 or 4.  With
 *               2 or 4 the table is the D-SFA transition over 2- or 4-byte
 *               words, delta_s applied 2 or 4 times, indexed through a
 *               65,536-entry table of byte-pair classes; available when the
 *               table fits the LDS budget (sfa_table_info.strides).
 *   pieces      K: interleaved pieces each chunk is walked as (1, 2, 3, 4, 8).
 *   load_bytes  G: bytes of one piece loaded per step (16, 32, 64, 128).
 *   depth       D: load steps in flight per piece (loads for step j + D - 1
 *               are issued before step j is walked; 1 = the rolling ring of
 *               the global-table walk described below).
 *   block_threads    TB: threads per block (256, 512, 1024).
 *   lanes_per_chunk  consecutive lanes that share a chunk (power of two
 *               <= 16); the chunk is cut into lanes_per_chunk * K pieces.
 * Supported (K, G, D, TB) for tables in LDS: TB=256: (1,64,2) (1,128,2)
 * (1,128,4) (2,64,2) (2,64,4) (2,128,2) (2,128,3) (2,128,4) (3,128,3)
 * (4,64,2) (8,32,2); TB=512: (1,64,2) (1,128,2) (1,128,3) (1,128,4) (2,64,2)
 * (2,64,4) (2,128,2) (2,128,3) (4,32,2) (4,64,2); TB=1024: (1,32,2) (1,64,2) (1,128,2) (2,32,2) (2,64,2).  The
 * default is (2,128,3,512); for a stride-4 table whose chunks are at most
 * 4 KiB it is (1,128,2,512) with lanes_per_chunk raised until the lanes fill
 * one 512-thread block per CU, when ceil(n / n_chunks) is a multiple of
 * 128 * lanes_per_chunk.  Tables in global memory use lanes_per_chunk=1
 * with TB=256: (1,64,2) (2,64,2) (4,32,2) (4,64,2) (1,128,2) (2,128,2)
 * (4,128,2); TB=512: (1,64,2) (2,64,2) (4,32,2) (4,64,2) (1,128,2) (2,128,2)
 * (2,128,3) and the rolling rings (2,128,1) (3,128,1) (4,128,1); TB=1024:
 * (1,64,2) (2,64,2) (1,128,2) and the rolling ring (2,128,1); default
 * (2,128,1,1024) when n is at least 1 KiB x 1024 lanes x the CU count,
 * else (4,128,1,512).  A partial D-SFA, and a table with vector re-walks
 * (sfa_table_info.vector_redo), have kernels for (4,128,1,512),
 * (2,128,1,512), (1,64,2,512) and (2,128,1,1024) only (vector re-walks:
 * other shapes walk without them); a complete D-SFA with vector re-walks
 * defaults to (4,128,1,512) at every size.  A plan that names a
 * shape but not block_threads gets a block size that supports the shape.
 * depth = 1 is a rolling ring of three half-line slots per piece: every
 * 128-byte line is requested whole, with 1.5 lines of registers per piece.
 * With n_chunks = 0 the default chunk count is one block of lanes per CU
 * (for the global-table walk: with 1024-thread blocks four, two or one per
 * CU, the most that keep chunks of at least 2 KiB; with 512-thread blocks
 * five when the chunks still hold at least 4 KiB, else four), with chunks
 * of at least 1 KiB.
 * Other values give SFA_ERR_INVALID_ARG.  Short chunks lower K first. */
typedef struct sfa_plan {
    uint32_t stride;
    uint32_t pieces;
    uint32_t load_bytes;
    uint32_t depth;
    uint32_t block_threads;
    uint32_t lanes_per_chunk;
} sfa_plan;

sfa_status sfa_match_ex(const sfa_table *t, const uint8_t *d_in, uint64_t n, uint32_t n_chunks,
                        const sfa_plan *plan, void *d_ws, size_t ws_bytes, sfa_result *d_out,
                        void *stream);

/* sfa_match without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same walk and result as sfa_match with
 * the default launch plan; d_in and d_out as there.  The workspace is the
 * library's own: a device array of SFA_NOALLOC_WORKSPACE_BYTES (4 MiB) per
 * GPU, held until the process ends; the first call on a device takes its
 * address and clears its control words with a fill kernel on `stream`.  The
 * call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine).  A call whose plan needs a larger workspace (see
 * sfa_match_workspace_bytes; e.g. millions of chunks over a large DFA)
 * returns SFA_ERR_INVALID_ARG before any device work.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (on different
 * streams, or from several threads) race and may return wrong results;
 * serialise them, or use sfa_match with a workspace per stream. */
#define SFA_NOALLOC_WORKSPACE_BYTES (4u << 20)
sfa_status sfa_match_noalloc(const sfa_table *t, const uint8_t *d_in, uint64_t n, uint32_t n_chunks,
                             sfa_result *d_out, void *stream);

/* Speculative parallel DFA (Algorithm 3, Section 3): per chunk, every DFA
 * state is simulated as a possible start (|Q| lookups per byte), giving the
 * chunk's mapping T_i; the mappings are composed as in sfa_match.  Works for
 * every table, with or without a D-SFA part; same arguments, same result. */
sfa_status sfa_match_speculative(const sfa_table *t, const uint8_t *d_in, uint64_t n,
                                 uint32_t n_chunks, void *d_ws, size_t ws_bytes,
                                 sfa_result *d_out, void *stream);

/* ------------------------------------------------------------------------
 * Batched matching: many (document, table) jobs in one kernel launch.
 *
 *   Documents are byte ranges of one device buffer, doc d = [doc_off[d],
 *   doc_off[d+1]).  A job (doc, table) is matched exactly as sfa_match would
 *   (whole-document membership, Algorithm 5 with the document cut into pieces
 *   of piece_bytes; any division is valid, Theorem 2); its result goes to
 *   d_out[job index].  Every table must have a D-SFA whose stride-1 walk table
 *   is at most 64 KiB (sfa_table_info.strides bit 1).
 *
 *   sfa_batch_create   host planning (pieces, work units, work items, the
 *                      jobs spanning items); doc_off and jobs are host arrays,
 *                      copied into the plan.  tables must stay loaded while
 *                      the plan is used.
 *   sfa_batch_workspace_bytes / sfa_batch_upload
 *                      the caller provides a device workspace (256-byte
 *                      aligned) and uploads the plan's descriptors into it once
 *                      (async on stream), together with the LDS contents (the
 *                      tables' class columns interleaved, then their stride-1
 *                      rows) when the tables are staged in LDS (taken from the
 *                      tables' packed host images when the batch is created).
 *   sfa_match_batch    enqueues one kernel launch (no allocation, no host
 *                      synchronisation, no memset), so a stream capture of it
 *                      can be replayed as a graph as long as the workspace and
 *                      table buffers stay in place.  The document bytes may
 *                      change between calls.  Launches of one plan that share
 *                      a workspace must not overlap (the arrival counters live
 *                      in it).
 *   sfa_batch_free     frees the host plan.
 * ---------------------------------------------------------------------- */
typedef struct sfa_batch sfa_batch;

typedef struct sfa_batch_options {
    uint32_t piece_bytes;     /* bytes per piece, multiple of 16 (0 = 4096) */
    uint32_t reserved;        /* must be 0 */
    uint32_t units_per_lane;  /* pieces walked together by one lane: 1, 2 or 4 (0 = 2) */
    uint32_t force_global;    /* 1: read walk tables from global memory instead of LDS */
} sfa_batch_options;

typedef struct sfa_batch_info {
    uint32_t n_jobs;
    uint32_t n_docs;          /* documents referenced by at least one job */
    uint64_t n_units;         /* (piece, job) work units */
    uint64_t n_item_map_entries; /* (job, work item, start state) entries of jobs spanning work items */
    uint32_t piece_bytes, units_per_lane, tables_in_lds, reserved;
    uint64_t workspace_bytes;
} sfa_batch_info;

sfa_status sfa_batch_create(const sfa_table *const *tables, uint32_t n_tables,
                            const uint64_t *doc_off /* host [n_docs + 1] */, uint32_t n_docs,
                            const uint32_t *jobs /* host [2 * n_jobs]: doc, table */, uint32_t n_jobs,
                            const sfa_batch_options *opts, sfa_batch **out);
sfa_status sfa_batch_get_info(const sfa_batch *b, sfa_batch_info *out);
sfa_status sfa_batch_workspace_bytes(const sfa_batch *b, size_t *out_bytes);
sfa_status sfa_batch_upload(const sfa_batch *b, void *d_ws, size_t ws_bytes, void *stream);
sfa_status sfa_match_batch(const sfa_batch *b, const uint8_t *d_data, void *d_ws, size_t ws_bytes,
                           sfa_result *d_out /* [n_jobs] */, void *stream);
void       sfa_batch_free(sfa_batch *b);

/* ------------------------------------------------------------------------
 * Streaming-read reference (measurement aid, not a matching step).
 *
 *   Reads d_in[0..n) once with wave-coalesced 16-byte loads and XORs every
 *   32-bit word (and the n % 16 tail bytes) into *d_out, so the HBM read
 *   rate of a read-only kernel can be measured on the same buffer and in
 *   the same run as the matcher: the matcher reads each input byte once
 *   (its roofline is this read), and this kernel is that read with nothing
 *   else.  d_in must be 16-byte aligned; d_out is device memory, and its
 *   value is the XOR of its old contents and the input words (callers
 *   clear it first if they want the checksum).  Asynchronous on stream.
 *   SFA_ERR_INVALID_ARG for a null or misaligned pointer.
 * ---------------------------------------------------------------------- */
sfa_status sfa_stream_read(const uint8_t *d_in, uint64_t n, uint32_t *d_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SFA_H */
