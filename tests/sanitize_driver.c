/* Host driver for the oracle under AddressSanitizer and UBSan
 * (tests/test_sanitize_cpu.py): reads "L k seed sample flags snap_step
 * seq_cap" lines from stdin, runs rsao_run (with a sequence buffer of seq_cap
 * entries when seq_cap > 0, and a 64-bin cluster-size histogram after deposit
 * snap_step when snap_step > 0) and rsao_contacts_at_jamming, and prints one
 * line per descriptor. */
#include <inttypes.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/rsa_oracle.h"

int main(void)
{
    unsigned L, k, sample, flags;
    unsigned long long seed, seq_cap;
    long long snap;
    while (scanf("%u %u %llu %u %u %lld %llu", &L, &k, &seed, &sample, &flags, &snap, &seq_cap) == 7) {
        rsao_desc_t d = {L, k, seed, sample, flags};
        rsao_result_t r;
        uint64_t hist[64] = {0};
        uint32_t *seq = seq_cap ? (uint32_t *)malloc(seq_cap * sizeof(uint32_t)) : NULL;
        int rc = rsao_run(&d, &r, seq, seq_cap, snap, snap > 0 ? hist : NULL, 64);
        uint64_t seq_sum = 0;
        if (seq && rc == RSAO_OK)
            for (int64_t t = 0; t < r.n_jam; ++t) seq_sum += seq[t];
        free(seq);
        uint64_t c3[3] = {0, 0, 0};
        int rc2 = rsao_contacts_at_jamming(&d, c3);
        uint64_t hsum = 0;
        for (int i = 0; i < 64; ++i) hsum += hist[i] * (uint64_t)i;
        printf("%d %" PRId64 " %" PRId64 " %" PRId64 " %" PRId64 " %" PRIu64 " %" PRIu64
               " %d %d %" PRIu64 " %" PRIu64 " %d %" PRIu64 " %" PRIu64 " %" PRIu64 " %" PRIu64 "\n",
               rc, r.n_jam, r.n_wrap_x, r.n_wrap_y, r.n_wrap_any, r.occ_hash, r.seq_hash,
               r.n_clusters_jam, r.n_nonwrapping_jam, r.alg_bytes, r.wchg_words, rc2, c3[0], c3[1],
               c3[2], hsum + seq_sum);
    }
    return 0;
}
