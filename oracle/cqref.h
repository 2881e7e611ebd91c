/* CPU oracle for exact weighted k-means colour quantization.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, single-threaded,
 * obviously-correct statement of what the GPU path computes.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never calls it and shares no code with it.
 *
 * Method: M. E. Celebi, "Improving the Performance of K-Means for Color
 * Quantization" (Weighted Sort-Means, Section 2.2 and Algo. 2).  All pointers
 * are host pointers; all buffers are owned by the caller.
 */
#ifndef CQREF_H
#define CQREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { CQREF_OK = 0, CQREF_EINVAL = 1, CQREF_ECAPACITY = 2, CQREF_ENOMEM = 5 };
enum { CQREF_INIT_FORGY = 0, CQREF_INIT_MAXMIN = 1, CQREF_INIT_KMEANSPP = 2, CQREF_INIT_USER = 3,
       CQREF_INIT_VAR = 4, CQREF_INIT_SFF = 5, CQREF_INIT_WU = 6,
       CQREF_INIT_LBG = 7, CQREF_INIT_DEN = 8 };

typedef struct {
    int32_t iters;      /* Lloyd iterations run                                  */
    int32_t converged;  /* 1 if stopped by the relative-SSE test or SSE == 0    */
    int32_t k_used;     /* min(K, N')                                           */
    int32_t prune;      /* 1 if sort-means pruning was on                       */
    int64_t n_unique;   /* N'                                                   */
    int64_t ndc_total;  /* distance calculations summed over colours and iters  */
    int64_t near_ties;  /* colour-iterations whose two best evaluated distances */
                        /* differ by at most 1e-5 relative                      */
    double sse_final;   /* SSE after the last centre update                     */
    double mse_float;   /* sse_final / number of pixels                         */
    double mse_img;     /* filled by cqref_quantize: MSE of the mapped image    */
} cqref_stats;

/* SFF subset size: max(K, ceil(2 K ln K)), at most n. */
int64_t cqref_sff_subset(int32_t K, int64_t n);

/* splitmix64 (Steele, Lea & Flood 2014): next output for state *s. */
uint64_t cqref_splitmix64_next(uint64_t* s);
/* Uniform integer in [0, T) by rejection on splitmix64 outputs (T >= 1). */
uint64_t cqref_uniform_below(uint64_t* s, uint64_t T);

/* Data reduction of Section 2.2 item 1 (unique colours) and item 2 (weights):
 * key = R<<16 | G<<8 | B, emitted in ascending key order with pixel counts.
 * subsample != 0 first applies the 2:1 subsampling of item 1 (the pixels at
 * even row and even column). */
int cqref_histogram(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride, int32_t subsample,
                    uint32_t* keys, uint32_t* counts, int64_t capacity, int64_t* n_unique);

/* Initialization schemes of Section 2.3 (FGY, MMX, KPP, VAR, SFF, LBG, DEN) and Wu's
 * greedy orthogonal bipartitioning (WU, the initializer of WSM-WU in Section
 * 3.3) on the unique colours. */
int cqref_init(const uint32_t* keys, const uint32_t* counts, int64_t n, int32_t K,
               int32_t scheme, uint64_t seed, double* centers, int32_t* k_used);

/* DEN's centres per cell (quota[512], cell (r >> 5) * 64 + (g >> 5) * 8 +
 * (b >> 5)) for K <= n unique colours.  For tests. */
int cqref_den_quotas(const uint32_t* keys, int64_t n, int32_t K, int32_t* quota);

/* The boxes of WU's partition for K (boxes[6 k .. 6 k + 5] = lo_r, lo_g,
 * lo_b, hi_r, hi_g, hi_b over the 32 levels value >> 3, inclusive), in box
 * index order; *n_boxes receives their number (at most K).  For tests. */
int cqref_wu_boxes(const uint32_t* keys, const uint32_t* counts, int64_t n, int32_t K, int32_t* boxes,
                   int32_t* n_boxes);

/* Weighted Lloyd iteration (Algo. 1 with the weights of Section 2.2) with
 * optional sort-means pruning (Algo. 2), relative-SSE stopping (Section 3.3). */
int cqref_kmeans(const uint32_t* keys, const uint32_t* counts, int64_t n, int32_t K,
                 double* centers, int32_t max_iters, double tol, int32_t prune,
                 uint8_t* assign, uint8_t* palette, double* sse_trace, cqref_stats* stats);

/* Pixel mapping to the nearest palette entry (integer distance, lowest index on
 * ties); returns the integer squared-error sum of the MSE of Section 3.1. */
int cqref_map(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride,
              const uint8_t* palette, int32_t K, uint8_t* out_idx, uint8_t* out_rgb,
              uint64_t* sq_err_sum);

/* Whole quantizer: histogram -> init -> k-means -> map. */
int cqref_quantize(const uint8_t* img, int32_t H, int32_t W, int64_t row_stride, int32_t subsample,
                   int32_t K, int32_t scheme, uint64_t seed, int32_t max_iters, double tol, int32_t prune,
                   uint8_t* palette, uint8_t* out_idx, uint8_t* out_rgb, cqref_stats* stats);

#ifdef __cplusplus
}
#endif
#endif
