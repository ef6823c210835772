/* Parallel SFA computation (Algorithm 5, Section 5.2) on host threads --
 * CPU oracle.
 *
 * Test infrastructure only: the product library never links this file.  It
 * is the paper's own CPU design, written out plainly: one chunk per thread,
 * a D-SFA transition table of 256 columns per state (4-byte entries, the
 * 1 KB-per-state layout the paper describes in Section 6.2), and the
 * sequential reduction of the chunk mappings.
 *
 * nxt   : [m * 256] D-SFA transition over bytes, nxt[s * 256 + b]; state 0
 *         is the identity f_I
 * maps  : [m * n] the mapping of each D-SFA state, maps[s * n + q] = f_s(q)
 * q0    : DFA start state
 * w, len: input bytes, every byte read once
 * p     : chunks = threads; chunk i is [i * L, min((i + 1) * L, len)),
 *         L = ceil(len / p) (empty chunks are f_I)
 * chunk_states (optional, [p]): the D-SFA state each chunk ends in
 * Returns f_fin(q0), f_fin = f_1 . f_2 . ... . f_p (reverse composition:
 * f_1 is applied first), i.e. the DFA state after the whole input.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

struct chunk_job {
    const uint32_t *nxt;
    const uint8_t *w;
    uint64_t lo, hi;
    uint32_t state;
};

static void *walk_chunk(void *arg)
{
    struct chunk_job *j = (struct chunk_job *)arg;
    uint32_t s = 0; /* f_I */
    for (uint64_t i = j->lo; i < j->hi; ++i)
        s = j->nxt[(size_t)s * 256u + j->w[i]];
    j->state = s;
    return NULL;
}

uint32_t oracle_sfa_parallel(const uint32_t *nxt, const uint32_t *maps, uint32_t n, uint32_t q0,
                             const uint8_t *w, uint64_t len, uint32_t p, uint32_t *chunk_states)
{
    if (p == 0)
        p = 1;
    struct chunk_job *jobs = calloc(p, sizeof(*jobs));
    pthread_t *tid = calloc(p, sizeof(*tid));
    char *created = calloc(p, 1);
    uint32_t *f = malloc(sizeof(uint32_t) * n), *g = malloc(sizeof(uint32_t) * n);
    if (!jobs || !tid || !created || !f || !g) {
        free(jobs); free(tid); free(created); free(f); free(g);
        return UINT32_MAX;
    }
    const uint64_t L = len ? (len + p - 1) / p : 0;
    for (uint32_t i = 0; i < p; ++i) {
        uint64_t lo = (uint64_t)i * L, hi = lo + L;
        jobs[i].nxt = nxt;
        jobs[i].w = w;
        jobs[i].lo = lo < len ? lo : len;
        jobs[i].hi = hi < len ? hi : len;
        created[i] = pthread_create(&tid[i], NULL, walk_chunk, &jobs[i]) == 0;
        if (!created[i])
            walk_chunk(&jobs[i]); /* no thread: walk it here */
    }
    for (uint32_t i = 0; i < p; ++i)
        if (created[i])
            pthread_join(tid[i], NULL);
    /* sequential reduction of the mappings, in text order */
    for (uint32_t q = 0; q < n; ++q)
        f[q] = q;
    for (uint32_t i = 0; i < p; ++i) {
        const uint32_t *fi = maps + (size_t)jobs[i].state * n;
        for (uint32_t q = 0; q < n; ++q)
            g[q] = fi[f[q]];          /* (f . f_i)(q) = f_i(f(q)) */
        uint32_t *t = f; f = g; g = t;
        if (chunk_states)
            chunk_states[i] = jobs[i].state;
    }
    const uint32_t r = f[q0];
    free(jobs); free(tid); free(created); free(f); free(g);
    return r;
}
