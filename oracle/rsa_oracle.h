/*
 * rsa_oracle.h -- serial CPU oracle for random sequential adsorption (RSA) of
 * linear k-mers on an L x L torus, run to jamming, with first-wrap tracking.
 *
 * TEST INFRASTRUCTURE.  This library exists only to check the GPU library.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load or call it.  It shares no code, header, table or helper
 * with the GPU library, and the GPU library never calls it.
 *
 * Paper: Slutskii, Barash, Tarasevich, "Percolation and jamming of random
 * sequential adsorption samples of large linear k-mers on a square lattice"
 * (arXiv:1810.06800).  What one sample computes:
 *   - Sec. II.A: k-mers on an L x L square lattice with periodic boundaries,
 *     deposited by isotropic RSA until jamming.
 *   - Sec. II.B: rejection-free deposition: the next k-mer is drawn among the
 *     placements where it still fits ("viable sites", one set per
 *     orientation); jamming is the moment that set is empty.
 *   - Sec. II.C: union-find cluster labelling, relabelling the smaller cluster.
 *   - Sec. II.D: a root per cluster and per-member displacements from it
 *     (Machta's method); a wrap can only appear when the new k-mer joins two
 *     parts of one cluster.
 *   - Sec. II.E: cluster id and displacements stored per k-mer, not per site.
 *   - Appendix A: every cluster of a jammed torus wraps; percolation precedes
 *     jamming.  Both are checked at the end of every run.
 *
 * Sampling convention (the paper's RNG library cannot be reproduced, so both
 * sides define the draw canonically): a placement is p = (o, y, x) with
 * o = 0 (horizontal, covers (y, x+i)) or 1 (vertical, covers (y+i, x)),
 * i = 0..k-1, all mod L, and canonical index P = o*L*L + y*L + x.  Step t
 * draws (r0..r3) = Philox4x32-10(key = (seed mod 2^32, seed >> 32),
 * counter = (t, sample, 0, 0)) [Salmon et al., SC'11], forms
 * u = r0 + 2^32*r1 and picks rank = floor(u * A_t / 2^64) among the A_t
 * available placements in canonical order.
 */
#ifndef RSA_ORACLE_H
#define RSA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Flag: vertical placements start unavailable, so the lattice is L
 * independent rings of length L (one-dimensional RSA).  Test mode. */
#define RSAO_FLAG_H_ONLY 1u
/* Flag accepted for interface symmetry with the GPU library: the oracle
 * always takes the cluster census at jamming. */
#define RSAO_FLAG_TRACK_CLUSTERS 2u
/* Flag accepted for parity with the GPU descriptors (contact census wanted);
 * the census itself comes from rsao_contacts_at_jamming. */
#define RSAO_FLAG_CONTACTS 4u

/* One independent run (Sec. II.A).  1 <= k <= L <= 32768. */
typedef struct {
    uint32_t L, k;
    uint64_t seed;
    uint32_t sample, flags;
} rsao_desc_t;

/* Result of one run.  Counts are 1-based deposit numbers; -1 means "never".
 *   n_jam        number of k-mers at jamming (p_j = n_jam*k/L^2)
 *   n_wrap_x/y   deposit after which some cluster first wraps in x / y
 *   n_wrap_any   min of the defined wrap counts (p_c = n_wrap_any*k/L^2)
 *   occ_hash     sum over occupied sites s of mix64((s << 32) | id(s))
 *   seq_hash     sum over steps t of mix64((t << 32) | P_t)
 *   n_clusters_jam, n_nonwrapping_jam   cluster census at jamming
 *   status       0, or a negative RSAO_E* code when an invariant failed
 *   alg_bytes    algorithmic-byte model of the run (see rsao_run)
 *   wchg_words   availability words whose value changed, summed over steps
 */
typedef struct {
    int64_t n_jam, n_wrap_x, n_wrap_y, n_wrap_any;
    uint64_t occ_hash, seq_hash;
    int32_t n_clusters_jam, n_nonwrapping_jam;
    int32_t status, pad_;
    uint64_t alg_bytes, wchg_words;
} rsao_result_t;

enum {
    RSAO_OK = 0,
    RSAO_EINVAL = -1,        /* bad descriptor                                */
    RSAO_ENOMEM = -2,        /* allocation failed                             */
    RSAO_ESCAN = -10,        /* a k-mer still fits after jamming              */
    RSAO_ECOUNT = -11,       /* availability bits or counts disagree at end   */
    RSAO_ENOWRAP = -12,      /* a cluster at jamming does not wrap (App. A)   */
    RSAO_EORDER = -13,       /* n_wrap_any undefined or after n_jam (App. A)  */
    RSAO_ECAPACITY = -14     /* caller's sequence buffer too small            */
};

/* Run one sample to jamming.
 *   d        descriptor (read only)
 *   r        result (written)
 *   seq      optional (may be NULL): receives P_t for t = 0..n_jam-1
 *   seq_cap  capacity of seq in entries
 *   snap_step   if > 0, cluster sizes in sites are histogrammed right after
 *               deposit number snap_step (1-based); snap_hist[s] counts the
 *               clusters of exactly s sites, for s < snap_cap.  May be 0/NULL.
 * Returns r->status. */
int rsao_run(const rsao_desc_t *d, rsao_result_t *r, uint32_t *seq, uint64_t seq_cap,
             int64_t snap_step, uint64_t *snap_hist, uint64_t snap_cap);

/* Run n samples one after another (no threads) into r[0..n-1]. */
int rsao_run_many(const rsao_desc_t *d, rsao_result_t *r, uint32_t n);

/* Building blocks, exported so that tests can pin them one by one. */
void     rsao_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint64_t rsao_mix64(uint64_t z);
uint32_t rsao_rank(uint64_t u, uint32_t a);

/* Contacts at jamming (Eq. 12): n_x, n_y = nearest-neighbour site pairs in
 * different k-mers that are both horizontal / both vertical, n_xy = pairs of
 * perpendicular k-mers.  Runs sample d to jamming first. */
int rsao_contacts_at_jamming(const rsao_desc_t *d, uint64_t out3[3]);

#ifdef __cplusplus
}
#endif
#endif
