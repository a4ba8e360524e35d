/*
 * ntt_oracle.c -- plain, slow, obviously-correct CPU oracle for the
 * negacyclic number-theoretic transform over a prime modulus.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may use it.  It shares no code, header, table or
 * constant generator with the GPU library: its number theory (primality,
 * quadratic non-residue, root choice), its twiddle tables and its butterflies
 * are written here again, independently, with unsigned __int128 products and
 * the % operator -- no Shoup, Montgomery, Barrett or lazy reduction.
 *
 * What it follows (Chameleon, arXiv 2410.05934):
 *   - Sec. II-D: the ring R_q = Z_q[x]/(x^N+1) and the product c = a*b in it.
 *   - Sec. II-D, Eq. (1): c = INTT^{GS,psi^-1}_{bo->no}( NTT^{CT,psi}_{no->bo}(a)
 *     (.) NTT^{CT,psi}_{no->bo}(b) ), psi a primitive 2N-th root of unity mod q.
 *   - Sec. V-A/V-B: the radix-2 baseline shape, (N/2)*log2(N) butterflies in
 *     log2(N) stages; this oracle runs exactly that shape, one stage at a time.
 *
 * Readings of points the paper leaves open (each also listed with the design
 * notes of the repository):
 *   - Which psi: the paper only asks for primitivity.  The oracle takes
 *     psi = g^((q-1)/(2N)) mod q with g the smallest quadratic non-residue
 *     mod q (Euler's criterion).  Then psi^N = g^((q-1)/2) = -1.
 *   - Forward output order is bit-reversed: out[j] = a(psi^(2*brv(j)+1)).
 *   - The inverse includes the factor N^-1, so inverse(forward(a)) == a.
 *   - Every output is canonical, in [0, q).
 *
 * Two families of functions:
 *   orc_forward / orc_inverse       -- the radix-2 CT (no->bo) and GS (bo->no)
 *                                      loops; O(N log N); used for whole arrays.
 *   orc_forward_at / orc_inverse_at /
 *   orc_negacyclic_at               -- the plain definitions, one output at a
 *                                      time in O(N); used on tiny inputs and
 *                                      for sampled outputs at full sizes.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include <unistd.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------ */
/* Plain modular arithmetic: one 128-bit product or sum, then %.             */

static uint64_t mulm(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
static uint64_t addm(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + b) % q); }
static uint64_t subm(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + q - (b % q)) % q); }

uint64_t orc_powmod(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q, b = a % q;
  while (e) {
    if (e & 1) r = mulm(r, b, q);
    b = mulm(b, b, q);
    e >>= 1;
  }
  return r;
}

/* Deterministic Miller-Rabin: the bases 2..37 decide every n < 3.3e24. */
int orc_is_prime(uint64_t n) {
  static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; ++i) {
    if (n == bases[i]) return 1;
    if (n % bases[i] == 0) return 0;
  }
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (int i = 0; i < 12; ++i) {
    uint64_t x = orc_powmod(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int witness = 1;
    for (int r = 1; r < s; ++r) {
      x = mulm(x, x, n);
      if (x == n - 1) { witness = 0; break; }
    }
    if (witness) return 0;
  }
  return 1;
}

/* Smallest g in [2, q) with g^((q-1)/2) == -1 mod q (Euler's criterion). */
uint64_t orc_smallest_qnr(uint64_t q) {
  if (q < 3) return 0;
  for (uint64_t g = 2; g < q; ++g)
    if (orc_powmod(g, (q - 1) / 2, q) == q - 1) return g;
  return 0;
}

/* psi = g^((q-1)/(2N)); returns 0 when q is not prime or 2N does not divide
 * q-1 (then no primitive 2N-th root exists). */
uint64_t orc_psi(uint32_t N, uint64_t q) {
  if (N < 1 || (N & (N - 1)) != 0) return 0;
  if (!orc_is_prime(q)) return 0;
  if ((q - 1) % (2 * (uint64_t)N) != 0) return 0;
  uint64_t g = orc_smallest_qnr(q);
  if (g == 0) return 0;
  return orc_powmod(g, (q - 1) / (2 * (uint64_t)N), q);
}

/* Inverse by Fermat's little theorem (q prime). */
uint64_t orc_invmod(uint64_t a, uint64_t q) { return orc_powmod(a, q - 2, q); }

static int log2u(uint32_t N) { int n = 0; while ((1u << n) < N) ++n; return n; }

uint32_t orc_bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

/* ------------------------------------------------------------------------ */
/* The radix-2 loops (Sec. II-D: CT no->bo with psi, GS bo->no with psi^-1). */

/* tab[k] = w^brv(k), k in [0, N). */
static void brv_powers(uint64_t* tab, uint32_t N, uint64_t w, uint64_t q) {
  int n = log2u(N);
  uint64_t p = 1 % q;
  uint64_t* pw = (uint64_t*)malloc(sizeof(uint64_t) * N);
  for (uint32_t k = 0; k < N; ++k) { pw[k] = p; p = mulm(p, w, q); }
  for (uint32_t k = 0; k < N; ++k) tab[k] = pw[orc_bitrev(k, n)];
  free(pw);
}

/* Forward: Cooley-Tukey butterflies, natural-order input, bit-reversed output.
 * Stage with m groups (m = 1, 2, ..., N/2): group i pairs a[j] with a[j+t],
 * t = N/(2m), for j in [2*i*t, 2*i*t + t), with twiddle psi^brv(m+i):
 *   (u, v) -> (u + v*w, u - v*w).                                           */
int orc_forward(uint64_t* a, uint32_t N, uint64_t q) {
  uint64_t psi = orc_psi(N, q);
  if (psi == 0) return -1;
  uint64_t* W = (uint64_t*)malloc(sizeof(uint64_t) * N);
  brv_powers(W, N, psi, q);
  uint32_t t = N;
  for (uint32_t m = 1; m < N; m <<= 1) {
    t >>= 1;
    for (uint32_t i = 0; i < m; ++i) {
      uint64_t w = W[m + i];
      uint32_t j0 = 2 * i * t;
      for (uint32_t j = j0; j < j0 + t; ++j) {
        uint64_t u = a[j];
        uint64_t v = mulm(a[j + t], w, q);
        a[j] = addm(u, v, q);
        a[j + t] = subm(u, v, q);
      }
    }
  }
  free(W);
  return 0;
}

/* Inverse: Gentleman-Sande butterflies, bit-reversed input, natural output.
 * Stages run in the opposite order (m = N/2, ..., 1), twiddle psi^-brv(m+i):
 *   (u, v) -> (u + v, (u - v)*w);  finally every value times N^-1.          */
int orc_inverse(uint64_t* a, uint32_t N, uint64_t q) {
  uint64_t psi = orc_psi(N, q);
  if (psi == 0) return -1;
  uint64_t* W = (uint64_t*)malloc(sizeof(uint64_t) * N);
  brv_powers(W, N, orc_invmod(psi, q), q);
  uint32_t t = 1;
  for (uint32_t m = N >> 1; m >= 1; m >>= 1) {
    for (uint32_t i = 0; i < m; ++i) {
      uint64_t w = W[m + i];
      uint32_t j0 = 2 * i * t;
      for (uint32_t j = j0; j < j0 + t; ++j) {
        uint64_t u = a[j];
        uint64_t v = a[j + t];
        a[j] = addm(u, v, q);
        a[j + t] = mulm(subm(u, v, q), w, q);
      }
    }
    t <<= 1;
  }
  uint64_t ninv = orc_invmod(N % q, q);
  for (uint32_t j = 0; j < N; ++j) a[j] = mulm(a[j], ninv, q);
  free(W);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Plain definitions, one output at a time.                                   */

/* out[j] = sum_i a[i] * psi^((2*brv(j)+1)*i)  -- evaluation of a(x) at the
 * odd power psi^(2*brv(j)+1), i.e. at one root of x^N + 1 (Horner).         */
uint64_t orc_forward_at(const uint64_t* a, uint32_t N, uint64_t q, uint32_t j) {
  uint64_t psi = orc_psi(N, q);
  if (psi == 0 || j >= N) return UINT64_MAX;
  uint64_t e = 2 * (uint64_t)orc_bitrev(j, log2u(N)) + 1;
  uint64_t x = orc_powmod(psi, e, q);
  uint64_t acc = 0;
  for (uint32_t i = N; i-- > 0;) acc = addm(mulm(acc, x, q), a[i] % q, q);
  return acc;
}

/* a[i] = N^-1 * sum_j ahat[j] * psi^(-(2*brv(j)+1)*i). */
uint64_t orc_inverse_at(const uint64_t* ahat, uint32_t N, uint64_t q, uint32_t i) {
  uint64_t psi = orc_psi(N, q);
  if (psi == 0 || i >= N) return UINT64_MAX;
  uint64_t psi_inv = orc_invmod(psi, q);
  int n = log2u(N);
  uint64_t acc = 0;
  for (uint32_t j = 0; j < N; ++j) {
    uint64_t e = ((2 * (uint64_t)orc_bitrev(j, n) + 1) * (uint64_t)i) % (2 * (uint64_t)N);
    acc = addm(acc, mulm(ahat[j] % q, orc_powmod(psi_inv, e, q), q), q);
  }
  return mulm(acc, orc_invmod(N % q, q), q);
}

/* c[k] of a*b mod (x^N + 1): sum_{i+j=k} a_i b_j - sum_{i+j=k+N} a_i b_j. */
uint64_t orc_negacyclic_at(const uint64_t* a, const uint64_t* b, uint32_t N, uint64_t q, uint32_t k) {
  uint64_t pos = 0, neg = 0;
  for (uint32_t i = 0; i < N; ++i) {
    if (i <= k) pos = addm(pos, mulm(a[i] % q, b[k - i] % q, q), q);
    else        neg = addm(neg, mulm(a[i] % q, b[N + k - i] % q, q), q);
  }
  return subm(pos, neg, q);
}

/* Whole negacyclic product by the definition, O(N^2). */
void orc_schoolbook(uint64_t* c, const uint64_t* a, const uint64_t* b, uint32_t N, uint64_t q) {
  for (uint32_t k = 0; k < N; ++k) c[k] = orc_negacyclic_at(a, b, N, q, k);
}

/* ------------------------------------------------------------------------ */
/* Elementwise operations on transformed operands (Eq. (1)'s (.) product).   */

void orc_pointwise_mul(uint64_t* c, const uint64_t* a, const uint64_t* b, uint64_t n, uint64_t q) {
  for (uint64_t j = 0; j < n; ++j) c[j] = mulm(a[j], b[j], q);
}

/* acc[j] = sum_r x_r[j] * k_r[j] mod q over `rows` operand/key pairs. */
void orc_mac(uint64_t* acc, const uint64_t* const* x, const uint64_t* const* k, uint32_t rows,
             uint64_t n, uint64_t q) {
  for (uint64_t j = 0; j < n; ++j) {
    uint64_t s = 0;
    for (uint32_t r = 0; r < rows; ++r) s = addm(s, mulm(x[r][j], k[r][j], q), q);
    acc[j] = s;
  }
}

/* Negacyclic product through Eq. (1): forward both, multiply, inverse. */
int orc_polymul(uint64_t* c, const uint64_t* a, const uint64_t* b, uint32_t N, uint64_t q) {
  uint64_t* fa = (uint64_t*)malloc(sizeof(uint64_t) * N);
  uint64_t* fb = (uint64_t*)malloc(sizeof(uint64_t) * N);
  memcpy(fa, a, sizeof(uint64_t) * N);
  memcpy(fb, b, sizeof(uint64_t) * N);
  int rc = orc_forward(fa, N, q);
  if (rc == 0) rc = orc_forward(fb, N, q);
  if (rc == 0) {
    orc_pointwise_mul(c, fa, fb, N, q);
    rc = orc_inverse(c, N, q);
  }
  free(fa);
  free(fb);
  return rc;
}

/* Automorphism sigma_k of R_q = Z_q[x]/(x^N+1) (Sec. III lists Automorph among
 * the CKKS operators; Sec. IV-B builds repacking on it): b(x) = a(x^k) for odd
 * k.  Written as the substitution itself: the term a_i x^i becomes a_i x^(i k);
 * the exponent is reduced mod 2N because x^(2N) = 1, and x^N = -1 turns an
 * exponent e >= N into -x^(e-N).  Every term is added into b, so nothing here
 * assumes the map is a permutation. */
void orc_automorph(uint64_t* b, const uint64_t* a, uint32_t N, uint64_t q, uint64_t k) {
  const uint64_t two_n = 2 * (uint64_t)N;
  for (uint32_t t = 0; t < N; ++t) b[t] = 0;
  for (uint32_t i = 0; i < N; ++i) {
    const uint64_t e = (uint64_t)(((u128)i * k) % two_n);
    if (e < N) b[e] = addm(b[e], a[i], q);
    else b[e - N] = subm(b[e - N], a[i], q);
  }
}

/* RNS basis conversion (BConv; Sec. III lists it among the CKKS operators around
 * the NTT).  x[L][N] holds residues of X modulo q_0..q_(L-1); the output
 * y[M][N] holds, modulo each p_j,
 *     sum_i [x_i * (Q/q_i)^-1 mod q_i] * (Q/q_i)        (Q = prod q_i),
 * which is X + alpha*Q for an integer 0 <= alpha < L (the fast conversion: no
 * correction of alpha).  Q/q_i is never formed: its residues are products of
 * the other moduli, reduced as they are multiplied. */
void orc_bconv(uint64_t* y, const uint64_t* x, uint32_t N, const uint64_t* q, uint32_t L,
               const uint64_t* p, uint32_t M) {
  for (uint32_t j = 0; j < M; ++j)
    for (uint32_t n = 0; n < N; ++n) y[(size_t)j * N + n] = 0;
  for (uint32_t i = 0; i < L; ++i) {
    uint64_t qhat_mod_qi = 1;                 /* (Q/q_i) mod q_i */
    for (uint32_t k = 0; k < L; ++k)
      if (k != i) qhat_mod_qi = mulm(qhat_mod_qi, q[k] % q[i], q[i]);
    const uint64_t qhat_inv = orc_invmod(qhat_mod_qi, q[i]);
    for (uint32_t j = 0; j < M; ++j) {
      uint64_t qhat_mod_pj = 1;               /* (Q/q_i) mod p_j */
      for (uint32_t k = 0; k < L; ++k)
        if (k != i) qhat_mod_pj = mulm(qhat_mod_pj, q[k] % p[j], p[j]);
      for (uint32_t n = 0; n < N; ++n) {
        const uint64_t t = mulm(x[(size_t)i * N + n], qhat_inv, q[i]);
        y[(size_t)j * N + n] = addm(y[(size_t)j * N + n], mulm(t % p[j], qhat_mod_pj, p[j]), p[j]);
      }
    }
  }
}

/* The last step of ModDown (Sec. III names BConv among the operators of CKKS
 * key switching; ModDown divides by the special modulus P): for one limb q,
 * y[n] = (x[n] - c[n]) * s mod q with s = P^-1 mod q and c the BConv of the
 * P-limbs into q.  Inputs in [0, q). */
void orc_sub_scale(uint64_t* y, const uint64_t* x, const uint64_t* c, uint32_t N, uint64_t q,
                   uint64_t s) {
  for (uint32_t n = 0; n < N; ++n) {
    const uint64_t d = x[n] >= c[n] ? x[n] - c[n] : x[n] + (q - c[n]);
    y[n] = mulm(d, s, q);
  }
}

/* ------------------------------------------------------------------------ */
/* Batched drivers: data[batch][L][N], moduli[L].  Independent (poly, limb)
 * rows are handed to a pool of threads; each row is transformed by the same
 * plain loop as above.  nthreads == 0 means one per online host core.       */

typedef struct {
  uint64_t* data;
  const uint64_t* moduli;
  uint32_t N, L;
  uint64_t rows;
  int op; /* 0 forward, 1 inverse */
  uint64_t next;
  int rc;
  pthread_mutex_t mu;
} batch_job;

static void* batch_worker(void* arg) {
  batch_job* jb = (batch_job*)arg;
  for (;;) {
    pthread_mutex_lock(&jb->mu);
    uint64_t r = jb->next++;
    pthread_mutex_unlock(&jb->mu);
    if (r >= jb->rows) break;
    uint64_t q = jb->moduli[r % jb->L];
    uint64_t* row = jb->data + r * (uint64_t)jb->N;
    int rc = jb->op == 0 ? orc_forward(row, jb->N, q) : orc_inverse(row, jb->N, q);
    if (rc != 0) {
      pthread_mutex_lock(&jb->mu);
      jb->rc = rc;
      pthread_mutex_unlock(&jb->mu);
    }
  }
  return NULL;
}

int orc_num_cores(void) {
  long n = sysconf(_SC_NPROCESSORS_ONLN);
  return n > 0 ? (int)n : 1;
}

static int run_batch(uint64_t* data, uint64_t batch, uint32_t L, uint32_t N, const uint64_t* moduli,
                     int op, int nthreads) {
  batch_job jb;
  jb.data = data; jb.moduli = moduli; jb.N = N; jb.L = L;
  jb.rows = batch * (uint64_t)L; jb.op = op; jb.next = 0; jb.rc = 0;
  pthread_mutex_init(&jb.mu, NULL);
  if (nthreads <= 0) nthreads = orc_num_cores();
  if ((uint64_t)nthreads > jb.rows) nthreads = (int)jb.rows;
  if (nthreads <= 1) {
    batch_worker(&jb);
  } else {
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
    for (int i = 0; i < nthreads; ++i) pthread_create(&th[i], NULL, batch_worker, &jb);
    for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
    free(th);
  }
  pthread_mutex_destroy(&jb.mu);
  return jb.rc;
}

int orc_forward_batch(uint64_t* data, uint64_t batch, uint32_t L, uint32_t N, const uint64_t* moduli, int nthreads) {
  return run_batch(data, batch, L, N, moduli, 0, nthreads);
}

int orc_inverse_batch(uint64_t* data, uint64_t batch, uint32_t L, uint32_t N, const uint64_t* moduli, int nthreads) {
  return run_batch(data, batch, L, N, moduli, 1, nthreads);
}
