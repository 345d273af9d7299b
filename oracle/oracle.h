/*
 * CPU oracle for enhanced normalized min-sum (NMS) decoding of short BCH codes
 * (Li & Yu, "Effective Application of Normalized Min-Sum Decoding for Short
 * BCH Codes", arXiv 2412.20828).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It is plain, slow, obviously-correct C: dense 0/1
 * byte matrices, FP64 arithmetic, explicit loops in the order the paper states.
 *
 * Conventions shared by every function:
 *   - a binary vector of length N is N bytes, each 0 or 1; bit i is the
 *     coefficient of x^i (column i of a parity-check matrix);
 *   - matrices are row-major, rows x N bytes;
 *   - return value 0 = success, negative = bad argument / failure.
 */
#ifndef BCH_ORACLE_H
#define BCH_ORACLE_H

#include <stdint.h>

#define ORC_MAXN 128

/* ---- code algebra (Section II system model; BCH codes of Section IV) ---- */
int orc_gf_tables(int m, uint32_t prim, int *exp_tab, int *log_tab);
int orc_bch_generator(int m, uint32_t prim, int t, uint8_t *g, int *deg);
int orc_bch_matrices(int m, uint32_t prim, int t, int *N, int *K,
                     uint8_t *g, uint8_t *h, uint8_t *G, uint8_t *Hstd);

/* ---- parity-check-matrix optimisation (Section III-A, steps 1-6) ---- */
int64_t orc_count_4cycles(const uint8_t *H, int M, int N);
int orc_rank(const uint8_t *H, int M, int N);
int orc_rref(uint8_t *H, int M, int N);
int orc_min_density(const uint8_t *Hr, int Mr, int N, int with_shifts,
                    uint8_t *out, int cap);
int orc_build_hopt(const uint8_t *Hstd, int M, int N, int beta,
                   int target_rows, int Q, uint64_t seed, int sa_steps_per_row, double sa_lambda,
                   uint8_t *Ho, int cap, int *Mr1_out, uint64_t *seed_used);

/* ---- automorphisms (Section III-B) ---- */
int orc_branch_maps(int N, int n_branches, int d_o, int16_t *maps);
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
int orc_draw_offsets(int N, uint64_t seed, uint64_t key_hi, int64_t frame_base, int64_t F, uint8_t *d_o);

/* ---- decoders ---- */
enum { ORC_R1 = 1, ORC_R2 = 2, ORC_R3 = 3 };
int orc_nms_literal(const uint8_t *H, int M, int N, const int16_t *maps, int B,
                    const double *L, double alpha, int max_iter, int mode,
                    const uint8_t *Hsyn, int Msyn, uint8_t *c_hat, int *iters,
                    int *converged, double *y_trace);
int orc_nms_fast(const uint8_t *H, int M, int N, const int16_t *maps, int B,
                 const double *L, double alpha, int max_iter, int mode,
                 const uint8_t *Hsyn, int Msyn, uint8_t *c_hat, int *iters,
                 int *converged, double *y_trace);
int orc_nms_fixed(const uint8_t *H, int M, int N, const int16_t *maps, int B,
                  const int8_t *q, int max_iter, int mode, const uint8_t *Hsyn,
                  int Msyn, uint8_t *c_hat, int *iters, int *converged,
                  int32_t *y_trace);
int orc_osd(const uint8_t *G, int K, int N, const double *L, int order,
            uint8_t *c_hat);
int orc_ml_bruteforce(const uint8_t *G, int K, int N, const double *L,
                      uint8_t *c_hat);

/* ---- weight enumeration of a code given its generator rows ---- */
int orc_weight_distribution(const uint8_t *G, int K, int N, uint64_t *A);
int64_t orc_words_of_weight(const uint8_t *G, int K, int N, int w,
                            uint8_t *out, int64_t cap);

/* ---- SplitMix64, exposed so the tests can pin it ---- */
uint64_t orc_splitmix64_next(uint64_t *state);

#endif
