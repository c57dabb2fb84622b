/* Test helper: counts the (a, b) pairs for which the reciprocal-and-correct
 * form of the width-32 uniform differs from the IEEE quotient a / b.
 * Form: y = RN(1/b); q0 = RN(a y); r = fma(-q0, b, a); q = fma(r, y, q0).
 * Built with -ffp-contract=off so that only the explicit fma calls fuse. */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

static inline double form(double a, double b, double y) {
  double q0 = a * y;
  double r = fma(-q0, b, a);
  return fma(r, y, q0);
}

static inline uint64_t sm64(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Width-64 form: a = RN(c+1), b = RN(n+1) are doubles; one correction makes
 * the quotient faithful, the second rounds it correctly. */
static inline double form2(double a, double b, double y) {
  double q0 = a * y;
  double q1 = fma(fma(-q0, b, a), y, q0);
  return fma(fma(-q1, b, a), y, q1);
}

typedef struct {
  uint64_t seed, count, mode, mismatches, checked;
} job_t;

/* mode 0: random b = n + 1 with n in [2^31, 2^32), random a in [1, b-1].
 * mode 1: near-midpoint a: for random b and a random binade, a = floor or
 *         ceil of (midpoint * b). */
static void *worker(void *arg) {
  job_t *j = (job_t *)arg;
  uint64_t s = j->seed, bad = 0, done = 0;
  for (uint64_t i = 0; i < j->count; i++) {
    if (j->mode >= 2) {
      /* width 64: n in [2^62, 2^63), c in [0, n) */
      uint64_t n = ((uint64_t)1 << 62) + (sm64(&s) & (((uint64_t)1 << 62) - 1));
      double bd = (double)(n + 1), y = 1.0 / bd;
      if (j->mode == 4) {
        /* hardest cases: a/b within ~2^-107 (relative) of a rounding midpoint.
         * B = odd 53-bit significand of b; for odd d, L = d B^{-1} mod 2^54 is
         * odd, and if L has 54 bits then A = (L B - d) / 2^54 is an integer
         * significand with A/B = L/2^54 - d/(2^54 B). */
        uint64_t B = ((uint64_t)1 << 52) | (sm64(&s) & (((uint64_t)1 << 52) - 1)) | 1;
        uint64_t inv = B; /* B^{-1} mod 2^64 by Newton */
        for (int it = 0; it < 6; it++) inv *= 2 - B * inv;
        const uint64_t mask54 = ((uint64_t)1 << 54) - 1;
        for (int64_t d = -7; d <= 7; d += 2) {
          uint64_t L = ((uint64_t)d * inv) & mask54;
          if (L < ((uint64_t)1 << 53)) continue;
          unsigned __int128 LB = (unsigned __int128)L * B;
          unsigned __int128 num = LB - (unsigned __int128)(__int128)d;
          uint64_t A = (uint64_t)(num >> 54);
          if ((num & mask54) != 0 || A < ((uint64_t)1 << 52) || A >= ((uint64_t)1 << 53)) continue;
          double bd2 = ldexp((double)B, 10);             /* b in [2^62, 2^63) */
          for (int sh = 10; sh >= -30; sh -= 8) {        /* a/b in (2^-41, 1) */
            double ad = ldexp((double)A, sh);
            if (ad > bd2 || ad < 1.0) continue;
            double yy = 1.0 / bd2;
            bad += form2(ad, bd2, yy) != ad / bd2;
            done++;
          }
        }
        continue;
      }
      if (j->mode == 2) {
        uint64_t cc = sm64(&s) % n;
        double ad = (double)(cc + 1);
        bad += form2(ad, bd, y) != ad / bd;
        done++;
      } else {
        /* near-midpoint: a/b close to (2M+1) 2^(-k-53); a = the doubles around mid*b */
        int k = 1 + (int)(sm64(&s) % 40);
        uint64_t M = ((uint64_t)1 << 52) | (sm64(&s) & (((uint64_t)1 << 52) - 1));
        long double mid = ldexpl((long double)(2 * M + 1), -k - 53);
        double t = (double)(mid * (long double)bd);
        double ad = t;
        for (int u = 0; u < 3; u++) {
          if (ad >= 1.0 && ad <= bd) {
            bad += form2(ad, bd, y) != ad / bd;
            done++;
          }
          ad = nextafter(ad, 0.0);
        }
        ad = nextafter(t, 1e300);
        if (ad >= 1.0 && ad <= bd) {
          bad += form2(ad, bd, y) != ad / bd;
          done++;
        }
      }
      continue;
    }
    uint64_t b = ((uint64_t)1 << 31) + 1 + (sm64(&s) % ((uint64_t)1 << 31));
    double bd = (double)b, y = 1.0 / bd;
    if (j->mode == 0) {
      uint64_t a = 1 + sm64(&s) % (b - 1);
      double ad = (double)a;
      bad += form(ad, bd, y) != ad / bd;
      done++;
    } else {
      int k = 1 + (int)(sm64(&s) % 32);       /* a/b in [2^-k, 2^-k+1) */
      uint64_t M = ((uint64_t)1 << 52) | (sm64(&s) & (((uint64_t)1 << 52) - 1));
      /* midpoint (2M+1) 2^(-k-53); a ~ midpoint * b */
      long double mid = ldexpl((long double)(2 * M + 1), -k - 53);
      long double t = mid * (long double)b;
      uint64_t a0 = (uint64_t)floorl(t);
      for (uint64_t a = a0 > 0 ? a0 : 1; a <= a0 + 1; a++) {
        if (a >= b) continue;
        double ad = (double)a;
        bad += form(ad, bd, y) != ad / bd;
        done++;
      }
    }
  }
  j->mismatches = bad;
  j->checked = done;
  return NULL;
}

/* Exhaustive over all a in [1, b-1] for one b. */
typedef struct {
  uint64_t b, lo, hi, bad;
} ex_t;

static void *ex_worker(void *arg) {
  ex_t *j = (ex_t *)arg;
  double bd = (double)j->b, y = 1.0 / bd;
  uint64_t bad = 0;
  for (uint64_t a = j->lo; a < j->hi; a++) {
    double ad = (double)a;
    bad += form(ad, bd, y) != ad / bd;
  }
  j->bad = bad;
  return NULL;
}

uint64_t recip_exhaustive(uint64_t b, uint64_t a_lo, uint64_t a_hi, int nthreads) {
  pthread_t th[64];
  ex_t jobs[64];
  if (nthreads > 64) nthreads = 64;
  for (int t = 0; t < nthreads; t++) {
    jobs[t].b = b;
    jobs[t].lo = a_lo + (a_hi - a_lo) * t / nthreads;
    jobs[t].hi = a_lo + (a_hi - a_lo) * (t + 1) / nthreads;
    pthread_create(&th[t], NULL, ex_worker, &jobs[t]);
  }
  uint64_t bad = 0;
  for (int t = 0; t < nthreads; t++) {
    pthread_join(th[t], NULL);
    bad += jobs[t].bad;
  }
  return bad;
}

uint64_t recip_sampled(uint64_t seed, uint64_t per_thread, int mode, int nthreads, uint64_t *checked) {
  pthread_t th[64];
  job_t jobs[64];
  if (nthreads > 64) nthreads = 64;
  for (int t = 0; t < nthreads; t++) {
    jobs[t].seed = seed + 0x1000 * (uint64_t)t;
    jobs[t].count = per_thread;
    jobs[t].mode = (uint64_t)mode;
    pthread_create(&th[t], NULL, worker, &jobs[t]);
  }
  uint64_t bad = 0, done = 0;
  for (int t = 0; t < nthreads; t++) {
    pthread_join(th[t], NULL);
    bad += jobs[t].mismatches;
    done += jobs[t].checked;
  }
  *checked = done;
  return bad;
}
