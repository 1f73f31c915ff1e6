/*
 * axsynth — seeded synthetic inputs shaped like the paper's corpora.
 *
 * This module only produces input bytes and request traces. It holds none of
 * the codec's arithmetic, so both the oracle (test side) and the product side
 * may use it.  Every random draw comes from SplitMix64 (Steele, Lea & Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014), with
 * u = (x >> 11) * 2^-53.
 *
 * Stand-ins (the paper's corpora are not available here):
 *   axs_dna  — chromosome-like DNA (order-3 Markov bases, planted copies,
 *              tandem repeats, lowercase runs, N runs): stands in for chr1 and
 *              the Pizza&Chili dna corpus (Setup; Table 2).
 *   axs_text — English-like text (Zipf vocabulary, re-emitted sentences):
 *              stands in for enwik / Pizza&Chili english (Table 2).
 *   axs_protein, axs_reads — protein-like sequences and FASTQ-like reads,
 *              the second workload family (Table 2's proteins; the genome
 *              vs reads depth tails).
 */
#ifndef AXSYNTH_H
#define AXSYNTH_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Fill out[0..n) with synthetic DNA for `seed`. Returns 0, or -1 on OOM. */
int axs_dna(uint8_t* out, uint64_t n, uint64_t seed);

/* Fill out[0..n) with synthetic English-like text for `seed`. 0 / -1 on OOM. */
int axs_text(uint8_t* out, uint64_t n, uint64_t seed);

/* Fill out[0..n) with protein-like sequences (one per line; 20-letter
 * alphabet; homologs, duplicates and low-complexity segments): stands in for
 * the Pizza&Chili proteins corpus (Table 2).  0 / -1 on OOM. */
int axs_protein(uint8_t* out, uint64_t n, uint64_t seed);

/* Fill out[0..n) with FASTQ-like 100-base reads of a synthetic genome (about
 * twelvefold coverage, 0.5 % substitutions, Markov quality lines): stands in
 * for the sequencing-read set of the depth-tail comparison.  0 / -1. */
int axs_reads(uint8_t* out, uint64_t n, uint64_t seed);

/* Batch plan: for archive i in [0,count): size in bytes and kind (0 = DNA,
 * 1 = text). Sizes are Lognormal(ln 1 MiB, 1.2) clipped to [64 KiB, 64 MiB];
 * kind is DNA with probability 0.6. Archive i's content seed is 1000 + i. */
void axs_batch_plan(uint32_t count, uint64_t seed, uint64_t* sizes, uint8_t* kinds);

/* Open-loop request trace over an archive of n bytes: Poisson arrivals at
 * `rate` requests/s (arrival_ns, monotone), request lengths (fixed `len_min`
 * when len_max == len_min, else log-uniform over [len_min, len_max]), and
 * start offsets: with probability 0.8 Zipf-local (a hot centre chosen by
 * Zipf(1.1) among 1024 uniformly placed centres, then a signed Zipf(1.1)
 * block distance of at most 4096 blocks of `block` bytes, plus a uniform byte
 * offset), else uniform over [0, n - len]. */
void axs_trace(uint64_t count, uint64_t seed, uint64_t n, uint32_t block, double rate,
               uint64_t len_min, uint64_t len_max,
               uint64_t* arrival_ns, uint64_t* off, uint64_t* len);

/* Raw generator access for tests of the generator itself. */
uint64_t axs_splitmix64(uint64_t* state);

#ifdef __cplusplus
}
#endif
#endif
