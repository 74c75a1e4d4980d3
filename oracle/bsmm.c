/*
 * Block-sparse matrix product for the CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * C = A B for square block-CSR matrices of b x b row-major FP64 blocks: the
 * product of Sec. 4 of the paper (a block of C is the sum over the inner
 * block index k of A_ik B_kj, zero blocks skipped).  Output block (i, j)
 * accumulates the block products in ascending k; each block product is the
 * plain triple loop.  Truncation (Sec. 5) is left to the caller, which gets
 * every block's Frobenius norm.  Rows of C are independent and are spread
 * over OpenMP threads; nothing else is reordered.
 *
 * Two calls: bsmm_pattern() counts the blocks of every output row (the
 * caller sizes the output from the counts), bsmm_values() writes the column
 * indices (ascending within a row), the values and the norms.
 *
 * This file shares nothing with the HIP library; only the oracle's Python
 * side loads it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* counts[i] = number of distinct j with A_ik, B_kj both present */
int bsmm_pattern(int64_t nb, const int64_t* arp, const int32_t* acol, const int64_t* brp, const int32_t* bcol,
                 int64_t* counts) {
  int failed = 0;
#pragma omp parallel
  {
    unsigned char* mark = (unsigned char*)calloc((size_t)nb, 1);
    if (!mark) {
#pragma omp atomic write
      failed = 1;
    } else {
#pragma omp for schedule(dynamic, 4)
      for (int64_t i = 0; i < nb; ++i) {
        int64_t c = 0;
        for (int64_t e = arp[i]; e < arp[i + 1]; ++e) {
          const int32_t k = acol[e];
          for (int64_t f = brp[k]; f < brp[k + 1]; ++f) {
            const int32_t j = bcol[f];
            if (!mark[j]) {
              mark[j] = 1;
              ++c;
            }
          }
        }
        counts[i] = c;
        /* clear the marks of this row */
        for (int64_t e = arp[i]; e < arp[i + 1]; ++e) {
          const int32_t k = acol[e];
          for (int64_t f = brp[k]; f < brp[k + 1]; ++f) mark[bcol[f]] = 0;
        }
      }
      free(mark);
    }
  }
  return failed ? -1 : 0;
}

/* acc += a b for b x b row-major blocks */
static void block_fma(int b, const double* a, const double* bb, double* acc) {
  for (int r = 0; r < b; ++r) {
    double* cr = acc + (size_t)r * b;
    for (int k = 0; k < b; ++k) {
      const double x = a[(size_t)r * b + k];
      const double* br = bb + (size_t)k * b;
      for (int c = 0; c < b; ++c) cr[c] += x * br[c];
    }
  }
}

/* crp: row pointers of C (exclusive prefix sums of bsmm_pattern's counts) */
int bsmm_values(int64_t nb, int32_t b, const int64_t* arp, const int32_t* acol, const double* avals,
                const int64_t* brp, const int32_t* bcol, const double* bvals, const int64_t* crp, int32_t* ccol,
                double* cvals, double* cnorm) {
  const size_t bb = (size_t)b * b;
  int failed = 0;
#pragma omp parallel
  {
    int32_t* slot = (int32_t*)malloc(sizeof(int32_t) * (size_t)nb);
    unsigned char* mark = (unsigned char*)calloc((size_t)nb, 1);
    if (!slot || !mark) {
#pragma omp atomic write
      failed = 1;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int64_t i = 0; i < nb; ++i) {
        /* the row's columns, ascending: mark them, then walk 0..nb-1 */
        for (int64_t e = arp[i]; e < arp[i + 1]; ++e) {
          const int32_t k = acol[e];
          for (int64_t f = brp[k]; f < brp[k + 1]; ++f) mark[bcol[f]] = 1;
        }
        int64_t o = crp[i];
        for (int64_t j = 0; j < nb; ++j)
          if (mark[j]) {
            slot[j] = (int32_t)(o - crp[i]);
            ccol[o++] = (int32_t)j;
            mark[j] = 0;
          }
        double* row = cvals + (size_t)crp[i] * bb;
        memset(row, 0, sizeof(double) * bb * (size_t)(crp[i + 1] - crp[i]));
        /* ascending k: acol is sorted within the row */
        for (int64_t e = arp[i]; e < arp[i + 1]; ++e) {
          const int32_t k = acol[e];
          const double* a = avals + (size_t)e * bb;
          for (int64_t f = brp[k]; f < brp[k + 1]; ++f)
            block_fma(b, a, bvals + (size_t)f * bb, row + (size_t)slot[bcol[f]] * bb);
        }
        for (int64_t o2 = crp[i]; o2 < crp[i + 1]; ++o2) {
          const double* v = cvals + (size_t)o2 * bb;
          double s = 0.0;
          for (size_t t = 0; t < bb; ++t) s += v[t] * v[t];
          cnorm[o2] = sqrt(s);
        }
      }
    }
    free(slot);
    free(mark);
  }
  return failed ? -1 : 0;
}
