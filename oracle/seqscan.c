/* Sequential DFA computation (Algorithm 2, Section 2.3) -- CPU oracle.
 *
 * Test infrastructure only: the product library never links this file.
 *
 * delta : [n_states * 256] next-state table, delta[q * 256 + b]
 * q     : start state
 * w, n  : input bytes; every byte is read exactly once, with no early exit
 *         at an absorbing state (the experiments of Section 6.2 read every
 *         character once).
 * Returns the state reached after the last byte.
 */
#include <stdint.h>
#include <stddef.h>

uint32_t oracle_seqscan(const uint32_t *delta, uint32_t q, const uint8_t *w, uint64_t n)
{
    for (uint64_t i = 0; i < n; ++i)
        q = delta[(size_t)q * 256u + w[i]];
    return q;
}
