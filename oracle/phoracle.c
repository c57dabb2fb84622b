/*
 * phoracle.c -- CPU oracle for the Pohlig-Hellman parameter-split pseudorandom
 * number generator (P. D. Beale, "A new class of scalable parallel pseudorandom
 * number generators based on Pohlig-Hellman exponentiation ciphers").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant generator with the GPU library, and it never
 * calls into it.
 *
 * Arithmetic: every integer product is formed exactly in unsigned __int128 and
 * reduced with the C '%' operator; there is no Montgomery form, no Mersenne
 * folding and no blocking.  Floating point appears in one place only, the
 * uniform R = (c+1)/(n+1) of step (9d), formed by converting both integers to
 * binary64 and dividing (IEEE round-to-nearest-even).  Build with
 * -O2 -fno-fast-math -ffp-contract=off.
 *
 * Each function names the passage of the paper it follows.  Readings of the
 * paper where it is silent or ambiguous:
 *   - A draw follows algorithm (9): advance the skip, advance the message,
 *     then encrypt.  From position k the t-th draw (t = 0, 1, ...) returns
 *     c_{k+1+t}; N draws leave the generator at position k+N.
 *   - Position 0 is the base state (m_0, s_0) = (0, 1) of Sec. IV unless a
 *     caller supplies m_0 / s_0; a start index k positions by eq. (7).
 *   - The skip-sum term of eq. (6b)/(7b) reduces each term mod p first and
 *     then sums over the integers, as the equations are printed.
 *   - 64-bit skip parameters are not printed in the paper (it points to
 *     L'Ecuyer "near 2^63"); this library uses p = 2^61 - 1 with the fixed
 *     primitive root a = 37^j mod p, j = 1425089352415399681.  Its
 *     statistical quality is parity unpinned.
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

/* ------------------------------------------------------------------------ */
/* Modular arithmetic (Sec. I: multiply-mod; repeated squaring)             */
/* ------------------------------------------------------------------------ */

/* x*y mod n, exact: one full product and one remainder. */
uint64_t pho_mulmod(uint64_t x, uint64_t y, uint64_t n) {
  return (uint64_t)(((u128)x * (u128)y) % (u128)n);
}

/* b^e mod n by right-to-left repeated squaring (Sec. I). */
uint64_t pho_powmod(uint64_t b, uint64_t e, uint64_t n) {
  if (n == 1) return 0;
  uint64_t result = 1;
  b %= n;
  while (e != 0) {
    if (e & 1) result = pho_mulmod(result, b, n);
    b = pho_mulmod(b, b, n);
    e >>= 1;
  }
  return result;
}

uint64_t pho_gcd(uint64_t x, uint64_t y) {
  while (y != 0) {
    uint64_t t = x % y;
    x = y;
    y = t;
  }
  return x;
}

/* Inverse of e modulo m by the extended Euclidean algorithm (Sec. I: the
 * decryption exponent d = e^{-1} mod (n-1)).  Returns 0 when gcd(e, m) != 1
 * or m < 2. */
uint64_t pho_inverse(uint64_t e, uint64_t m) {
  if (m < 2) return 0;
  i128 r0 = (i128)m, r1 = (i128)(e % m);
  i128 t0 = 0, t1 = 1;
  while (r1 != 0) {
    i128 q = r0 / r1;
    i128 tmp = r0 - q * r1;
    r0 = r1;
    r1 = tmp;
    tmp = t0 - q * t1;
    t0 = t1;
    t1 = tmp;
  }
  if (r0 != 1) return 0;
  if (t0 < 0) t0 += (i128)m;
  return (uint64_t)t0;
}

/* Encryption, eq. (1): c = m^e mod n. */
uint64_t pho_encrypt(uint64_t m, uint64_t e, uint64_t n) { return pho_powmod(m, e, n); }

/* Eq. (1) over an array (used by the brute-force permutation pins). */
void pho_encrypt_many(const uint64_t *m, uint64_t len, uint64_t e, uint64_t n, uint64_t *out) {
  for (uint64_t i = 0; i < len; i++) out[i] = pho_powmod(m[i], e, n);
}

/* Decryption, eq. (2): m = c^d mod n with d = e^{-1} mod (n-1). */
uint64_t pho_decrypt(uint64_t c, uint64_t e, uint64_t n) {
  uint64_t d = pho_inverse(e, n - 1);
  return pho_powmod(c, d, n);
}

/* ------------------------------------------------------------------------ */
/* Primality (Sec. IV: trial division, then Rabin-Miller)                   */
/* ------------------------------------------------------------------------ */

/* One Rabin-Miller round: returns 1 when odd n > 2 is a strong probable prime
 * to base g, i.e. with n - 1 = 2^r t (t odd), g^t = 1 or g^{2^j t} = n-1 for
 * some 0 <= j < r.  A base that is a multiple of n passes trivially. */
int pho_strong_probable_prime(uint64_t n, uint64_t g) {
  if (n < 3 || (n & 1) == 0) return n == 2;
  if (g % n == 0) return 1;
  uint64_t t = n - 1;
  int r = 0;
  while ((t & 1) == 0) {
    t >>= 1;
    r++;
  }
  uint64_t x = pho_powmod(g, t, n);
  if (x == 1 || x == n - 1) return 1;
  for (int j = 1; j < r; j++) {
    x = pho_mulmod(x, x, n);
    if (x == n - 1) return 1;
  }
  return 0;
}

static const uint64_t SMALL_PRIMES[] = {2,  3,  5,  7,  11, 13, 17, 19, 23, 29, 31, 37, 41,
                                        43, 47, 53, 59, 61, 67, 71, 73, 79, 83, 89, 97};
#define N_SMALL_PRIMES (sizeof(SMALL_PRIMES) / sizeof(SMALL_PRIMES[0]))

/* Deterministic primality below 2^64 (Sec. IV): divide by small primes first,
 * then Rabin-Miller with the five smallest prime bases below 2^32 and the
 * twelve smallest prime bases otherwise. */
int pho_is_prime(uint64_t n) {
  if (n < 2) return 0;
  for (size_t i = 0; i < N_SMALL_PRIMES; i++) {
    if (n == SMALL_PRIMES[i]) return 1;
    if (n % SMALL_PRIMES[i] == 0) return 0;
  }
  int nbases = (n < ((uint64_t)1 << 32)) ? 5 : 12;
  for (int i = 0; i < nbases; i++)
    if (!pho_strong_probable_prime(n, SMALL_PRIMES[i])) return 0;
  return 1;
}

/* Safe prime: n and (n-1)/2 both prime (Sec. I). */
int pho_is_safe_prime(uint64_t n) { return n > 4 && pho_is_prime(n) && pho_is_prime((n - 1) / 2); }

/* Primitive root test: a generates (Z/pZ)^* iff a^((p-1)/q) != 1 mod p for
 * every prime q dividing p - 1 (Sec. II: the skip multiplier must be a
 * primitive root mod p).  p - 1 is factored by plain trial division, which is
 * fast for the smooth p - 1 of the skip moduli used here. */
int pho_is_primitive_root(uint64_t a, uint64_t p) {
  if (!pho_is_prime(p) || a % p == 0) return 0;
  uint64_t m = p - 1, rest = m;
  for (uint64_t q = 2; q * q <= rest; q++) {
    if (rest % q == 0) {
      if (pho_powmod(a, m / q, p) == 1) return 0;
      while (rest % q == 0) rest /= q;
    }
  }
  if (rest > 1 && pho_powmod(a, m / rest, p) == 1) return 0;
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Instance parameters                                                      */
/* ------------------------------------------------------------------------ */

#define PHO_OK 0
#define PHO_E_INVALID (-1)
#define PHO_E_NOT_PRIME (-2)
#define PHO_E_EXPONENT (-3)
#define PHO_E_RANGE (-4)

/* Skip generators of eq. (5).  32-bit: the L'Ecuyer prime-modulus LCG the
 * paper tests with (Sec. II).  64-bit: p = 2^61 - 1 and a fixed primitive
 * root (not given by the paper; see the header comment). */
int pho_lcg_params(int width, uint64_t *p, uint64_t *a) {
  if (width == 32) {
    *p = 2147483647ULL;
    *a = 784588716ULL;
    return PHO_OK;
  }
  if (width == 64) {
    *p = 2305843009213693951ULL; /* 2^61 - 1 */
    *a = 1633150009242682173ULL; /* 37^1425089352415399681 mod p */
    return PHO_OK;
  }
  return PHO_E_INVALID;
}

/* Admissibility of (n, e) for a width (Sec. I, II, IV): n prime in the
 * width's range ([2^31, 2^32) or [2^62, 2^63)), gcd(e, n-1) = 1, e >= 3,
 * e mod (n-1) != 1 (not the identity map), and skip modulus p < n. */
int pho_check_instance(int width, uint64_t n, uint64_t e) {
  uint64_t lo, hi, p, a;
  if (width == 32) {
    lo = (uint64_t)1 << 31;
    hi = (uint64_t)1 << 32;
  } else if (width == 64) {
    lo = (uint64_t)1 << 62;
    hi = (uint64_t)1 << 63;
  } else {
    return PHO_E_INVALID;
  }
  if (n < lo || n >= hi) return PHO_E_RANGE;
  if (!pho_is_prime(n)) return PHO_E_NOT_PRIME;
  if (e < 3 || pho_gcd(e, n - 1) != 1 || e % (n - 1) == 1) return PHO_E_EXPONENT;
  pho_lcg_params(width, &p, &a);
  if (p >= n) return PHO_E_RANGE;
  return PHO_OK;
}

/* ------------------------------------------------------------------------ */
/* Skip-sum checkpoints for eq. (7b)                                        */
/* ------------------------------------------------------------------------ */

/* U(r) = sum_{j=1}^{r} (a^j mod p): the skip sum of eq. (7b) for s_0 = 1.
 * It has no closed form, so the oracle memoises it at every multiple of
 * `stride` up to max_r by plain summation; U(r) for other r continues from
 * the checkpoint below r.  Segments are summed by independent threads, each
 * starting from a^{start} mod p; the integer sum is the same in any order. */
typedef struct {
  uint64_t p, a, stride, count; /* count = number of checkpoints (index 0 is U(0) = 0) */
  u128 *U;                      /* U(i * stride) */
  uint64_t *S;                  /* a^{i * stride} mod p */
} pho_skiptab;

typedef struct {
  const pho_skiptab *tab;
  uint64_t seg_lo, seg_hi; /* segments [seg_lo, seg_hi) */
  u128 *seg_sum;
} skiptab_job;

static void *skiptab_worker(void *arg) {
  skiptab_job *job = (skiptab_job *)arg;
  const pho_skiptab *tab = job->tab;
  for (uint64_t seg = job->seg_lo; seg < job->seg_hi; seg++) {
    uint64_t s = pho_powmod(tab->a, seg * tab->stride, tab->p);
    u128 sum = 0;
    for (uint64_t j = 0; j < tab->stride; j++) {
      s = pho_mulmod(tab->a, s, tab->p);
      sum += s;
    }
    job->seg_sum[seg] = sum;
  }
  return NULL;
}

static int resolve_threads(int nthreads) {
  if (nthreads > 0) return nthreads;
  long n = sysconf(_SC_NPROCESSORS_ONLN);
  return n > 0 ? (int)n : 1;
}

pho_skiptab *pho_skiptab_new(uint64_t p, uint64_t a, uint64_t stride, uint64_t max_r, int nthreads) {
  if (stride == 0 || max_r > p - 1) return NULL;
  pho_skiptab *tab = (pho_skiptab *)calloc(1, sizeof(pho_skiptab));
  if (!tab) return NULL;
  tab->p = p;
  tab->a = a;
  tab->stride = stride;
  tab->count = max_r / stride + 1;
  tab->U = (u128 *)calloc(tab->count, sizeof(u128));
  tab->S = (uint64_t *)calloc(tab->count, sizeof(uint64_t));
  u128 *seg_sum = (u128 *)calloc(tab->count, sizeof(u128));
  if (!tab->U || !tab->S || !seg_sum) {
    free(tab->U);
    free(tab->S);
    free(seg_sum);
    free(tab);
    return NULL;
  }
  uint64_t nseg = tab->count - 1; /* segment i covers j in (i*stride, (i+1)*stride] */
  int nt = resolve_threads(nthreads);
  if ((uint64_t)nt > nseg) nt = nseg > 0 ? (int)nseg : 1;
  pthread_t *th = (pthread_t *)calloc(nt, sizeof(pthread_t));
  skiptab_job *jobs = (skiptab_job *)calloc(nt, sizeof(skiptab_job));
  for (int t = 0; t < nt; t++) {
    jobs[t].tab = tab;
    jobs[t].seg_lo = nseg * t / nt;
    jobs[t].seg_hi = nseg * (t + 1) / nt;
    jobs[t].seg_sum = seg_sum;
    pthread_create(&th[t], NULL, skiptab_worker, &jobs[t]);
  }
  for (int t = 0; t < nt; t++) pthread_join(th[t], NULL);
  free(th);
  free(jobs);
  tab->U[0] = 0;
  for (uint64_t i = 1; i < tab->count; i++) tab->U[i] = tab->U[i - 1] + seg_sum[i - 1];
  for (uint64_t i = 0; i < tab->count; i++) tab->S[i] = pho_powmod(a, i * stride, p);
  free(seg_sum);
  return tab;
}

void pho_skiptab_free(pho_skiptab *tab) {
  if (!tab) return;
  free(tab->U);
  free(tab->S);
  free(tab);
}

uint64_t pho_skiptab_max_r(const pho_skiptab *tab) { return (tab->count - 1) * tab->stride + tab->stride - 1; }

/* U(r) for 0 <= r <= p - 1 within the table's reach; returns -1 if out of reach. */
int pho_skip_prefix(const pho_skiptab *tab, uint64_t r, uint64_t *u_lo, uint64_t *u_hi) {
  if (r > tab->p - 1) return PHO_E_RANGE;
  uint64_t i = r / tab->stride;
  if (i >= tab->count) return PHO_E_RANGE;
  u128 sum = tab->U[i];
  uint64_t s = tab->S[i];
  for (uint64_t j = i * tab->stride; j < r; j++) {
    s = pho_mulmod(tab->a, s, tab->p);
    sum += s;
  }
  *u_lo = (uint64_t)sum;
  *u_hi = (uint64_t)(sum >> 64);
  return PHO_OK;
}

/* ------------------------------------------------------------------------ */
/* Message schedule and generation                                          */
/* ------------------------------------------------------------------------ */

/* State at position k by eq. (7): q = floor(k/(p-1)), r = k mod (p-1),
 *   s_k = s_0 a^r mod p,
 *   m_k = (m_0 + q p(p-1)/2 + sum_{j=1}^{r} (s_0 a^j mod p)) mod n.
 * With s_0 = 1 the sum is U(r), read from the checkpoint table (tab may be
 * NULL, then the sum is looped); other s_0 loop over the r terms. */
int pho_position(const pho_skiptab *tab, uint64_t p, uint64_t a, uint64_t n, uint64_t m0, uint64_t s0, uint64_t k,
                 uint64_t *m_out, uint64_t *s_out) {
  if (s0 == 0 || s0 >= p || m0 >= n) return PHO_E_INVALID;
  uint64_t q = k / (p - 1), r = k % (p - 1);
  u128 sum = 0;
  if (s0 == 1 && tab != NULL && tab->p == p && tab->a == a) {
    uint64_t lo, hi;
    int st = pho_skip_prefix(tab, r, &lo, &hi);
    if (st != PHO_OK) return st;
    sum = ((u128)hi << 64) | lo;
  } else {
    uint64_t term = s0;
    for (uint64_t j = 1; j <= r; j++) {
      term = pho_mulmod(a, term, p);
      sum += term;
    }
  }
  u128 full_period_sum = ((u128)p * (u128)(p - 1)) / 2; /* sum of 1..p-1 */
  u128 qterm = ((u128)(q % n) * (full_period_sum % n)) % n;
  u128 m = ((u128)m0 + qterm + sum % n) % n;
  *m_out = (uint64_t)m;
  *s_out = pho_mulmod(s0, pho_powmod(a, r, p), p);
  return PHO_OK;
}

/* Algorithm (9), `count` times, from state (*m, *s):
 *   s := a s mod p;  m := (m + s) mod n;  c := m^e mod n;  R := (c+1)/(n+1).
 * Either output array may be NULL.  The state is left after the last draw. */
void pho_generate(uint64_t p, uint64_t a, uint64_t n, uint64_t e, uint64_t *m, uint64_t *s, uint64_t count,
                  uint64_t *c_out, double *r_out) {
  uint64_t mm = *m, ss = *s;
  double denom = (double)(n + 1);
  for (uint64_t t = 0; t < count; t++) {
    ss = pho_mulmod(a, ss, p);
    mm = (uint64_t)(((u128)mm + ss) % n);
    uint64_t c = pho_powmod(mm, e, n);
    if (c_out) c_out[t] = c;
    if (r_out) r_out[t] = (double)(c + 1) / denom;
  }
  *m = mm;
  *s = ss;
}

/* Many independent instances, split over threads.  Instance i starts from
 * (m[i], s[i]) and writes count[i] draws at out_off[i]; the states are
 * updated in place. */
typedef struct {
  uint64_t lo, hi;
  const uint64_t *p, *a, *n, *e, *count, *out_off;
  uint64_t *m, *s, *c_out;
  double *r_out;
} gen_job;

static void *gen_worker(void *arg) {
  gen_job *j = (gen_job *)arg;
  for (uint64_t i = j->lo; i < j->hi; i++)
    pho_generate(j->p[i], j->a[i], j->n[i], j->e[i], &j->m[i], &j->s[i], j->count[i],
                 j->c_out ? j->c_out + j->out_off[i] : NULL, j->r_out ? j->r_out + j->out_off[i] : NULL);
  return NULL;
}

void pho_generate_many(int nthreads, uint64_t ninst, const uint64_t *p, const uint64_t *a, const uint64_t *n,
                       const uint64_t *e, uint64_t *m, uint64_t *s, const uint64_t *count, const uint64_t *out_off,
                       uint64_t *c_out, double *r_out) {
  int nt = resolve_threads(nthreads);
  if ((uint64_t)nt > ninst) nt = ninst > 0 ? (int)ninst : 1;
  pthread_t *th = (pthread_t *)calloc(nt, sizeof(pthread_t));
  gen_job *jobs = (gen_job *)calloc(nt, sizeof(gen_job));
  for (int t = 0; t < nt; t++) {
    gen_job g = {ninst * t / nt, ninst * (t + 1) / nt, p, a, n, e, count, out_off, m, s, c_out, r_out};
    jobs[t] = g;
    pthread_create(&th[t], NULL, gen_worker, &jobs[t]);
  }
  for (int t = 0; t < nt; t++) pthread_join(th[t], NULL);
  free(th);
  free(jobs);
}

/* Constant-skip schedule of Sec. II (unit skip when b = 1): the message at
 * position k is m_k = (m_0 + k b) mod n. */
uint64_t pho_cskip_message(uint64_t n, uint64_t m0, uint64_t b, uint64_t k) {
  return (uint64_t)(((u128)m0 + (u128)(k % n) * (u128)(b % n)) % n);
}

/* Draws under the constant skip, from message *m: m := (m + b) mod n,
 * c := m^e mod n, R := (c+1)/(n+1), `count` times. */
void pho_generate_cskip(uint64_t n, uint64_t e, uint64_t b, uint64_t *m, uint64_t count, uint64_t *c_out,
                        double *r_out) {
  uint64_t mm = *m;
  double denom = (double)(n + 1);
  for (uint64_t t = 0; t < count; t++) {
    mm = (uint64_t)(((u128)mm + b % n) % n);
    uint64_t c = pho_powmod(mm, e, n);
    if (c_out) c_out[t] = c;
    if (r_out) r_out[t] = (double)(c + 1) / denom;
  }
  *m = mm;
}

/* Forward jump by stepping (9a)-(9b) delta times (no encryption). */
void pho_jump_forward(uint64_t p, uint64_t a, uint64_t n, uint64_t *m, uint64_t *s, uint64_t delta) {
  uint64_t mm = *m, ss = *s;
  for (uint64_t t = 0; t < delta; t++) {
    ss = pho_mulmod(a, ss, p);
    mm = (uint64_t)(((u128)mm + ss) % n);
  }
  *m = mm;
  *s = ss;
}

/* Backward jump (Sec. II): the inverse step subtracts the current skip from
 * the message, then replaces s by a^{-1} s mod p; repeated delta times. */
void pho_jump_backward(uint64_t p, uint64_t a, uint64_t n, uint64_t *m, uint64_t *s, uint64_t delta) {
  uint64_t ainv = pho_inverse(a, p);
  uint64_t mm = *m, ss = *s;
  for (uint64_t t = 0; t < delta; t++) {
    mm = (uint64_t)(((u128)mm + n - ss % n) % n);
    ss = pho_mulmod(ainv, ss, p);
  }
  *m = mm;
  *s = ss;
}

/* ------------------------------------------------------------------------ */
/* Seeding (Sec. IV: each instance gets its own prime modulus)              */
/* ------------------------------------------------------------------------ */

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the state advances by the
 * golden-ratio increment and each output is the state passed through the
 * variant-13 finaliser. */
static uint64_t splitmix64_next(uint64_t *state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Exposed for the seeding pin test. */
void pho_splitmix64(uint64_t seed, uint64_t count, uint64_t *out) {
  uint64_t st = seed;
  for (uint64_t i = 0; i < count; i++) out[i] = splitmix64_next(&st);
}

/* Seeded instances, drawn in this order from one SplitMix64 stream:
 *   repeat: x = next(); candidate n = (lo + (x mod span)) | 1, where
 *           [lo, lo + span) is the width's range; reject n unless it is
 *           prime and not already drawn in this call; then y = next(),
 *           try e_set[(y mod e_len + t) mod e_len] for t = 0, 1, ... and
 *           keep the first admissible one; if none is, reject n;
 *   then, if k_hi > k_lo, z = next() and k = k_lo + z mod (k_hi - k_lo),
 *   else k = k_lo.
 * Distinctness is checked with a plain linear-probing set of drawn moduli. */
int pho_seed(int width, uint64_t seed, uint64_t count, const uint64_t *e_set, int e_len, uint64_t k_lo,
             uint64_t k_hi, uint64_t *n_out, uint64_t *e_out, uint64_t *k_out) {
  uint64_t lo, span;
  if (width == 32) {
    lo = (uint64_t)1 << 31;
    span = (uint64_t)1 << 31;
  } else if (width == 64) {
    lo = (uint64_t)1 << 62;
    span = (uint64_t)1 << 62;
  } else {
    return PHO_E_INVALID;
  }
  if (e_len <= 0 || k_hi < k_lo) return PHO_E_INVALID;
  int any_ok = 0;
  for (int i = 0; i < e_len; i++)
    if (e_set[i] >= 3) any_ok = 1;
  if (!any_ok) return PHO_E_EXPONENT;
  uint64_t cap = 16;
  while (cap < 2 * count + 16) cap <<= 1;
  uint64_t *set = (uint64_t *)calloc(cap, sizeof(uint64_t)); /* 0 = empty; moduli are never 0 */
  if (!set) return PHO_E_INVALID;
  uint64_t st = seed;
  for (uint64_t i = 0; i < count; i++) {
    for (;;) {
      uint64_t x = splitmix64_next(&st);
      uint64_t n = (lo + x % span) | 1;
      if (!pho_is_prime(n)) continue;
      uint64_t h = (n * 0x9E3779B97F4A7C15ULL) & (cap - 1);
      int dup = 0;
      while (set[h] != 0) {
        if (set[h] == n) {
          dup = 1;
          break;
        }
        h = (h + 1) & (cap - 1);
      }
      if (dup) continue;
      uint64_t y = splitmix64_next(&st);
      uint64_t e = 0;
      for (int t = 0; t < e_len; t++) {
        uint64_t cand = e_set[(y % (uint64_t)e_len + (uint64_t)t) % (uint64_t)e_len];
        if (pho_check_instance(width, n, cand) == PHO_OK) {
          e = cand;
          break;
        }
      }
      if (e == 0) continue;
      set[h] = n;
      n_out[i] = n;
      e_out[i] = e;
      break;
    }
    if (k_hi > k_lo) {
      uint64_t z = splitmix64_next(&st);
      k_out[i] = k_lo + z % (k_hi - k_lo);
    } else {
      k_out[i] = k_lo;
    }
  }
  free(set);
  return PHO_OK;
}

/* ------------------------------------------------------------------------ */
/* Bulk predicates used by the prime-count pins (threaded loops)            */
/* ------------------------------------------------------------------------ */

typedef struct {
  const uint64_t *v;
  uint64_t lo, hi, e;
  int mode;
  uint64_t count;
} count_job;

static void *count_worker(void *arg) {
  count_job *j = (count_job *)arg;
  uint64_t c = 0;
  for (uint64_t i = j->lo; i < j->hi; i++) {
    uint64_t n = j->v[i];
    int ok = 0;
    if (j->mode == 0) ok = pho_is_prime(n);
    else if (j->mode == 1) ok = pho_is_safe_prime(n);
    else if (j->mode == 2) ok = pho_gcd(j->e, n - 1) == 1;
    c += ok ? 1 : 0;
  }
  j->count = c;
  return NULL;
}

/* mode 0: count of prime v[i]; mode 1: count of safe primes; mode 2: count
 * with gcd(e, v[i]-1) = 1. */
uint64_t pho_count_many(int nthreads, const uint64_t *v, uint64_t len, int mode, uint64_t e) {
  int nt = resolve_threads(nthreads);
  if ((uint64_t)nt > len) nt = len > 0 ? (int)len : 1;
  pthread_t *th = (pthread_t *)calloc(nt, sizeof(pthread_t));
  count_job *jobs = (count_job *)calloc(nt, sizeof(count_job));
  for (int t = 0; t < nt; t++) {
    count_job cj = {v, len * t / nt, len * (t + 1) / nt, e, mode, 0};
    jobs[t] = cj;
    pthread_create(&th[t], NULL, count_worker, &jobs[t]);
  }
  uint64_t total = 0;
  for (int t = 0; t < nt; t++) {
    pthread_join(th[t], NULL);
    total += jobs[t].count;
  }
  free(th);
  free(jobs);
  return total;
}

/* ------------------------------------------------------------------------ */
/* Full-period local pattern (Sec. II, Figs. 3-4: the D-dimensional pattern of         */
/* consecutive ciphertexts over the whole period, in O(p L0) steps)          */
/* ------------------------------------------------------------------------ */

/* Over the full period every pair (m_k, s_k) occurs exactly once, so the
 * tuples (c_k, c_{k+1}, ..., c_{k+D-1}) whose first point lies in a window
 * are enumerated by the window's ciphertexts c and all skips s: with
 * m = c^d mod n (d = e^{-1} mod (n-1)), the following points are
 *   c_{k+1} = (m + s)^e,  c_{k+2} = (m + s + (a s mod p))^e, ...
 * (all mod n), the skip advancing by one multiplication by a mod p per point.
 * Each tuple with c in [x0, x0 + l0) and s in [s_lo, s_hi) (the full period
 * takes s = 1 .. p-1) adds one to the cell of its D-1 following points:
 * bins floor(c_j B / n) per axis, the first following point the most
 * significant digit of the cell index.  hist has B^(D-1) entries and is
 * accumulated, not cleared. */
void pho_pattern_hist(uint64_t n, uint64_t e, uint64_t p, uint64_t a, uint64_t x0, uint64_t l0, int dim,
                      uint64_t bins, uint64_t s_lo, uint64_t s_hi, uint64_t *hist) {
  uint64_t d = pho_inverse(e, n - 1);
  for (uint64_t c = x0; c < x0 + l0; c++) {
    uint64_t m = pho_powmod(c, d, n);
    for (uint64_t s = s_lo; s < s_hi; s++) {
      uint64_t sk = s;
      uint64_t mk = (uint64_t)(((u128)m + sk) % n);
      uint64_t cell = 0;
      for (int j = 1; j < dim; j++) {
        if (j > 1) {
          sk = pho_mulmod(a, sk, p);
          mk = (uint64_t)(((u128)mk + sk) % n);
        }
        uint64_t cj = pho_powmod(mk, e, n);
        uint64_t b = (uint64_t)(((u128)cj * bins) / n);
        cell = cell * bins + b;
      }
      hist[cell]++;
    }
  }
}
