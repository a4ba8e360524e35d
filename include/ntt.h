/*
 * ntt.h -- C ABI of the MI355X (gfx950) negacyclic NTT library (libntt.so).
 *
 * The operation (Chameleon, arXiv 2410.05934, Sec. II-D and Eq. (1)): for a
 * power-of-two N and a prime q = 1 (mod 2N), the ring R_q = Z_q[x]/(x^N + 1);
 * the forward transform of a(x) is the Cooley-Tukey NTT taking natural order to
 * bit-reversed order, out[j] = a(psi^(2*brv(j)+1)) mod q, with psi a primitive
 * 2N-th root of unity mod q; the inverse is the Gentleman-Sande NTT with
 * psi^-1, bit-reversed order to natural order, including the factor N^-1; the
 * product of two polynomials is INTT(NTT(a) (.) NTT(b)).
 *
 * Root choice (the paper only requires primitivity): psi = g^((q-1)/(2N)) mod q
 * with g the smallest quadratic non-residue mod q.  ntt_plan_root() returns it.
 *
 * Data layout: a batch of RNS polynomials is one contiguous device array
 * data[batch][L][N] of uint32_t (word_bits 32) or uint64_t (word_bits 64);
 * limb l of every polynomial is reduced modulo moduli[l].  Every input must be
 * canonical, in [0, moduli[l]); every output is canonical.  Out-of-range input
 * is a precondition violation: the output is then unspecified, but no call
 * faults on it.  Plans created with NTT_FLAG_VALIDATE check it (NTT_ERANGE).
 *
 * Ownership: the caller owns every data buffer (device memory, e.g. from a
 * PyTorch tensor).  A plan owns its device twiddle tables and is read-only
 * after creation, so one plan may be used from several host threads and
 * streams at once (a polymul with a column pass takes a stream-ordered
 * workspace with hipMallocAsync on the caller's stream and releases it there
 * with hipFreeAsync).  All transform calls are asynchronous on the
 * given stream (a hipStream_t passed as void*, NULL = the default stream);
 * their results are valid once the stream has reached that point.
 *
 * Errors: every call returns a status code and never aborts; a thread-local
 * message is available from ntt_last_error().  Calls on an invalid argument
 * change nothing.
 */
#ifndef NTT_MI355X_H
#define NTT_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ntt_plan_s* ntt_plan_t;

typedef enum {
  NTT_OK = 0,
  NTT_EINVAL = 1,     /* bad argument: null pointer, N not a power of two in [2, 2^16], word_bits, ... */
  NTT_ENOTPRIME = 2,  /* a modulus is not prime */
  NTT_ENOROOT = 3,    /* q != 1 (mod 2N): no primitive 2N-th root of unity */
  NTT_ERANGE = 4,     /* modulus too wide for the word: q >= 2^32 (32-bit) or q >= 2^62 (64-bit);
                         with NTT_FLAG_VALIDATE also an input word outside [0, q) */
  NTT_ENOMEM = 5,     /* device or host allocation failed */
  NTT_EDEVICE = 6,    /* HIP runtime error (no device, launch failure, ...) */
  NTT_EBUSY = 7,      /* resource in use */
  NTT_ETIMEOUT = 8    /* a bounded wait inside a persistent launch expired */
} ntt_status;

/* Plan flags.  NTT_FLAG_SPLIT(n1) forces the pass split N = 2^n1 * 2^(log2 N - n1):
 * n1 = 0 is a single on-chip pass (N <= 2^14), n1 >= 1 a column pass of n1
 * stages followed by a row pass (the row part must be 2^4 .. 2^14 words, or
 * n1 = log2 N for N < 16).  Without it each call takes the split the tuning
 * table records for its shape (see ntt_tune_split), else the default:
 * N < 16 one column pass, N <= 2^12 one row pass, else 2^12-word rows. */
#define NTT_FLAG_SPLIT(n1) ((uint32_t)(((n1) + 1) & 0x1f) << 8)
#define NTT_FLAG_SPLIT_MASK (0x1fu << 8)
/* Force the 64-bit integer (Shoup) arithmetic for every limb, even where the
 * exact fp64 arithmetic would be chosen (testing and measurement). */
#define NTT_FLAG_FORCE_INT64 (1u << 16)
/* Row passes of 2^10 .. 2^13 words with 8 values per thread (radix-8 rounds,
 * twice the threads of radix-16 rounds, one more LDS exchange).  Without it the
 * tuning table chooses per direction and shape, else: radix-4 rows (below) for
 * the 64-bit integer class (q >= 2^50) when a call has at most 256 row chunks
 * (one per compute unit); otherwise radix-8 for inverse rows, forward rows of
 * 2^10 .. 2^11 words and single-pass polymul rows, radix-16 for the rest. */
#define NTT_FLAG_ROW_RADIX8 (1u << 17)
/* Two-pass transforms with 2^12-word rows (N = 2^13 .. 2^16) run both passes in
 * one persistent launch: the one global synchronisation per transform of the
 * paper's single-kernel hybrid NTT (Sec. V-D) becomes a per-transform counter
 * that row (forward) or column (inverse) pieces wait on.  Results are
 * bit-identical to the two-launch form.  The waits are bounded (2^20 polls by
 * default, see ntt_debug_wait_limit); the order of the work list guarantees
 * that they end long before.  A call in this form waits for its stream before
 * it returns (so it cannot be captured into a graph) and returns NTT_ETIMEOUT
 * if any wait gave up; its output is then unspecified, but every kernel has
 * finished normally.  On MI355X this form is slower than the default two
 * launches (cross-XCD release/acquire per piece); it is there for callers
 * that need a single launch per call. */
#define NTT_FLAG_FUSED (1u << 18)
/* Forward and inverse row passes of 2^8 .. 2^12 words with 4 values per thread
 * (radix-4 rounds: four times the threads of radix-16 rounds and twice the LDS
 * exchanges).  It shortens each thread's chain of dependent butterflies, which
 * is what bounds a call with few transforms (the single-polynomial latency
 * regime of the paper's Tab. ntt-mix); polymul rows ignore it.  Exclusive with
 * NTT_FLAG_ROW_RADIX8. */
#define NTT_FLAG_ROW_RADIX4 (1u << 19)
/* Check every input word of every call on this plan before its kernels run:
 * a device-side scan of the inputs (data, a, b, key, ct, acc, in) for words
 * outside [0, q) of their limb.  Such a call returns NTT_ERANGE, naming the
 * first offending word (polynomial, limb, index), and launches nothing else,
 * so its outputs are untouched.  A validated call waits for its stream (the
 * scan's result is read back), so it cannot be captured into a graph.
 * Ragged batches and the request server do not validate. */
#define NTT_FLAG_VALIDATE (1u << 20)

/* Create a plan for length N and num_moduli RNS limbs (Sec. II-D; twiddles are
 * precomputed per modulus as the paper keeps them in constant memory, Sec. II-E).
 *   N           power of two, 2 <= N <= 65536
 *   moduli      host array of num_moduli (1 .. 4096) distinct-or-not primes,
 *               each q = 1 (mod 2N); q < 2^32 for word_bits 32, q < 2^62 for 64
 *   word_bits   32 or 64: the storage width of every coefficient
 *   flags       NTT_FLAG_* bits, 0 for defaults
 * On success *out receives the plan (release with ntt_plan_destroy).  Uses the
 * current HIP device. */
ntt_status ntt_plan_create(ntt_plan_t* out, uint32_t N, const uint64_t* moduli,
                           uint32_t num_moduli, uint32_t word_bits, uint32_t flags);

/* Release a plan and its device tables.  The caller must make sure no work
 * using the plan is still pending on any stream. */
ntt_status ntt_plan_destroy(ntt_plan_t plan);

/* The primitive 2N-th root psi used for limb `limb` (see root choice above). */
ntt_status ntt_plan_root(ntt_plan_t plan, uint32_t limb, uint64_t* psi);

/* The pass split in use: *log_n1 = number of column stages (0 = single pass). */
ntt_status ntt_plan_split(ntt_plan_t plan, uint32_t* log_n1);

/* The split a call over `batch` polynomials would use (tuning table or default). */
ntt_status ntt_plan_split_for(ntt_plan_t plan, uint32_t batch, uint32_t* log_n1);

/* Arithmetic class of a limb: 0 = exact fp64 for 32-bit words, 1 = exact fp64
 * for q < 2^50 - 2^10 in 64-bit words, 2 = 64-bit integer Shoup. */
ntt_status ntt_plan_limb_class(ntt_plan_t plan, uint32_t limb, uint32_t* cls);

/* Forward NTT in place on data[batch][L][N] (natural -> bit-reversed order). */
ntt_status ntt_forward(ntt_plan_t plan, void* data, uint32_t batch, void* stream);

/* Inverse NTT in place on data[batch][L][N] (bit-reversed -> natural, times N^-1). */
ntt_status ntt_inverse(ntt_plan_t plan, void* data, uint32_t batch, void* stream);

/* Eq. (1)'s elementwise product of transformed operands: out = a (.) b mod q_l,
 * all three [batch][L][N]; out may alias a or b. */
ntt_status ntt_pointwise_mul(ntt_plan_t plan, void* out, const void* a, const void* b,
                             uint32_t batch, void* stream);

/* Grouped multiply-accumulate of transformed operands against a key table (the
 * MAC of the TFHE external product, Sec. IV-A):
 *   a     [num_operands][L][N]; operand p is row r = p % rows of group g = p / rows
 *   key   [rows][cols][L][N]
 *   out   [groups][cols][L][N], groups = ceil(num_operands / rows)
 *   out[g][c] = sum over the rows r present in group g of a[g*rows + r] (.) key[r][c]
 * The last group may be partial.  out must not alias a or key; out and key
 * must each hold fewer than 2^32 words (else NTT_EINVAL). */
ntt_status ntt_mac(ntt_plan_t plan, void* out, const void* a, const void* key, uint32_t rows,
                   uint32_t cols, uint32_t num_operands, void* stream);

/* The same grouped multiply-accumulate (Sec. IV-A), sized by groups:
 *   acc[g][c] = sum over the rows r present in group g of a[g*rows + r] (.) key[r][c]
 * for g < groups; every group holds `rows` operands except the last, which holds
 * batch_tail (1 .. rows; 0 means a full last group).  So a holds
 * (groups - 1) * rows + (batch_tail ? batch_tail : rows) operands [.][L][N],
 * key [rows][cols][L][N], acc [groups][cols][L][N] (overwritten, not added to;
 * must not alias a or key).  For the TFHE shape (2048 operands, rows = 6,
 * cols = 2): groups = 342, batch_tail = 2.  Errors as ntt_mac, plus NTT_EINVAL
 * for groups or rows 0 or batch_tail > rows. */
ntt_status ntt_pointwise_mac(ntt_plan_t plan, void* acc, const void* a, const void* key,
                             uint32_t rows, uint32_t cols, uint32_t groups, uint32_t batch_tail,
                             void* stream);

/* RNS basis conversion (BConv; Sec. III lists it among the CKKS operators
 * around the NTT).  in[batch][L][N] holds residues of X modulo the source
 * moduli q_0..q_(L-1) (coefficient domain); out[batch][M][N] receives, modulo
 * each target modulus p_j,
 *     sum_i [x_i (Q/q_i)^-1 mod q_i] (Q/q_i mod p_j)      (Q = prod q_i),
 * that is X + alpha Q mod p_j for one integer 0 <= alpha < L per coefficient
 * (the fast conversion; alpha is not corrected).
 *   create: N a power of two in [2, 65536]; 1 <= L <= 64 distinct prime source
 *           moduli and 1 <= M <= 4096 target moduli >= 2, all below 2^32
 *           (word_bits 32) or 2^62 (word_bits 64); the constants go to the
 *           current device.  Errors: NTT_EINVAL, NTT_ENOTPRIME, NTT_ERANGE,
 *           NTT_ENOMEM / NTT_EDEVICE.
 *   run:    in canonical residues; out must not overlap in; batch * L * N and
 *           batch * M * N below 2^32 words (else NTT_EINVAL).  Asynchronous on
 *           `stream`. */
typedef struct ntt_bconv_s* ntt_bconv_t;
/* When every modulus is below 2^50 - 2^10, N >= 32 and L, M >= 16 the sum runs
 * on the int8 matrix cores (balanced base-256 digits, exact int32 sums; below
 * 16 moduli on either side the vector units are faster).  NTT_BCONV_NO_MFMA
 * keeps it on the vector units, NTT_BCONV_MFMA takes the matrix cores at any
 * L and M (the fp64 bound and N >= 32 still apply); the words are the same. */
#define NTT_BCONV_NO_MFMA 1u
#define NTT_BCONV_MFMA 2u
/* With at most 48 source and 48 target moduli the matrix-core form keeps each
 * wave's constant operands in registers for the whole launch (one wave per 4
 * targets beside four waves that form the digits, each workgroup walking a run
 * of 32-coefficient tiles); NTT_BCONV_NO_WS keeps the streaming form, which
 * reloads them per tile.  The words are the same. */
#define NTT_BCONV_NO_WS 4u
ntt_status ntt_bconv_create(ntt_bconv_t* out, uint32_t N, const uint64_t* src_moduli, uint32_t L,
                            const uint64_t* dst_moduli, uint32_t M, uint32_t word_bits,
                            uint32_t flags);
ntt_status ntt_bconv(ntt_bconv_t h, void* out, const void* in, uint32_t batch, void* stream);
ntt_status ntt_bconv_destroy(ntt_bconv_t h);

/* ModUp and ModDown: the basis changes of CKKS key switching built on BConv
 * (Sec. III lists BConv, ModMul and ModAdd among the operators around the NTT).
 * A key-switching basis holds L moduli q_i (Q = prod q_i) and K special moduli
 * p_k (P = prod p_k), all distinct primes.  Polynomials over Q u P are laid out
 * [batch][L + K][N] with the L limbs of Q first; coefficient domain.
 *   ntt_mod_up:   in[batch][L][N] over Q -> out[batch][L + K][N]: limbs 0..L-1
 *                 are in's residues, limb L + k is BConv_{Q->P}(x) mod p_k, i.e.
 *                 X + alpha Q with one 0 <= alpha < L per coefficient (not
 *                 corrected).  One launch: the copy is fused into the reads.
 *   ntt_mod_down: in[batch][L + K][N] over Q u P -> out[batch][L][N] over Q:
 *                 out_i = (x_i - BConv_{P->Q}(x_P)_i) * (P^-1 mod q_i) mod q_i.
 *                 For X = P Y + e with 0 <= e < P this is Y - alpha mod Q with one
 *                 0 <= alpha < K (the fast conversion's error).  One launch: the
 *                 subtraction and the scale are fused into the conversion's stores.
 *   create: N a power of two in [2, 65536]; 1 <= L, K <= 64; moduli below 2^32
 *           (word_bits 32) or 2^62 (word_bits 64); flags as ntt_bconv_create
 *           (each direction takes the matrix cores under the same rule).
 *           Constants go to the current device.  Errors: NTT_EINVAL (sizes, flags,
 *           a modulus in both sets or twice in one), NTT_ENOTPRIME, NTT_ERANGE,
 *           NTT_ENOMEM / NTT_EDEVICE.
 *   run:    device pointers; inputs canonical residues; out must not overlap in;
 *           batch * (L + K) * N below 2^32 words (else NTT_EINVAL).  Asynchronous
 *           on `stream`; the caller owns both buffers. */
typedef struct ntt_basis_ext_s* ntt_basis_ext_t;
ntt_status ntt_basis_ext_create(ntt_basis_ext_t* out, uint32_t N, const uint64_t* q_moduli,
                                uint32_t L, const uint64_t* p_moduli, uint32_t K,
                                uint32_t word_bits, uint32_t flags);
ntt_status ntt_mod_up(ntt_basis_ext_t h, void* out, const void* in, uint32_t batch, void* stream);
ntt_status ntt_mod_down(ntt_basis_ext_t h, void* out, const void* in, uint32_t batch, void* stream);
ntt_status ntt_basis_ext_destroy(ntt_basis_ext_t h);

/* Automorphism sigma_k of R_q = Z_q[x]/(x^N+1): b(x) = a(x^k) for odd k,
 * 1 <= k < 2N, on every limb of in[batch][L][N] into out[batch][L][N] (Sec. III
 * names Automorph among the CKKS operators around the NTT; Sec. IV-B builds
 * repacking on it).  Coefficient domain by default: the term a_i x^i becomes
 * a_i x^(i k mod 2N), negated when that exponent is N or more (x^N = -1).  With
 * NTT_AUTOMORPH_TRANSFORMED, in and out are in the forward transform's output
 * order and the map is a permutation of slots: slot j holds the value at
 * psi^(2 brv(j) + 1), and out slot j takes the input slot whose exponent is
 * (2 brv(j) + 1) k mod 2N.  Inputs canonical in [0, q); outputs likewise.
 * Errors (NTT_EINVAL, before any launch): null pointers, even k or k >= 2N,
 * unknown flags, out overlapping in, batch * L * N >= 2^32 words. */
#define NTT_AUTOMORPH_TRANSFORMED 1u
ntt_status ntt_automorph(ntt_plan_t plan, void* out, const void* in, uint32_t batch, uint32_t k,
                         uint32_t flags, void* stream);

/* External product of the TFHE CMux (Sec. II-B, Sec. IV-A: decomposed operands
 * are transformed, multiplied-and-accumulated against a key in the transform
 * domain, and the accumulators are inverse-transformed):
 *   out[g][c] = INTT( sum over the rows r present in group g of
 *                     NTT(a[g*rows + r]) (.) key[r][c] )
 * with the grouping of ntt_mac.  a [num_operands][L][N] in natural order (not
 * modified), key [rows][cols][L][N] in the transform domain (the order
 * ntt_forward produces), out [groups][cols][L][N] in natural order; out must
 * not alias a or key.  The same words as ntt_forward on a copy of a, ntt_mac
 * and ntt_inverse on out.  For N <= 2^12 with cols <= rows (and a workgroup of
 * rows * N/16 <= 1024 threads) one launch does everything per group and limb;
 * other shapes take the three steps through a stream-ordered workspace. */
ntt_status ntt_external_product(ntt_plan_t plan, void* out, const void* a, const void* key,
                                uint32_t rows, uint32_t cols, uint32_t num_operands,
                                void* stream);

/* External product of RLWE ciphertexts with the gadget decomposition fused in
 * (Sec. II-B: RGSW keys of (k+1) x (k+1) l RLWE rows; Sec. IV-A: Decompose, NTT
 * and MAC of a batched CMux).  Each coefficient a of component c of ciphertext g
 * is split into `levels` signed digits in base B = 2^log_base: from the
 * remainder r (initially a), a lower digit is r mod B moved to [-B/2, B/2) and
 * r becomes (r - d) / B; the top digit is the last remainder, so
 * a = sum_j d_j B^j exactly.  Digit j of component c is operand row
 * r = c * levels + j (as a residue mod q), and
 *   out[g][col] = INTT( sum_r NTT(digit row r of ct[g]) (.) key[r][col] ).
 *   ct    [num_ct][comps][L][N], natural order, not modified
 *   key   [comps * levels][cols][L][N], transform domain
 *   out   [num_ct][cols][L][N], natural order; must not alias ct or key
 * Requires q <= 2^(levels * log_base - 1) for every limb (the top digit stays in
 * [0, B/2]), levels * log_base <= 64 and 1 <= log_base <= 32; the operands, out
 * and key must each hold
 * fewer than 2^32 words (else NTT_EINVAL).  The same words as decomposing into
 * a buffer and calling ntt_external_product on it.  For N <= 2^12 with
 * cols <= comps * levels one launch per class decomposes while it loads;
 * other shapes decompose into a stream-ordered workspace first. */
ntt_status ntt_external_product_decomposed(ntt_plan_t plan, void* out, const void* ct,
                                           const void* key, uint32_t num_ct, uint32_t comps,
                                           uint32_t levels, uint32_t log_base, uint32_t cols,
                                           void* stream);

/* One batched CMux step of blind rotation (Sec. II-B: the accumulator goes
 * through n_lwe CMux gates against RGSW bootstrapping keys; Sec. IV-A: all
 * ciphertexts of one key bit in one batched gate).  For every ciphertext g,
 *   out[g] = acc[g] + ExtProd(key, X^rot[g] acc[g] - acc[g])
 * where X^r acc is the negacyclic monomial product (r taken mod 2N) and ExtProd
 * is the external product of ntt_external_product_decomposed (gadget digits of
 * each component, rows c * levels + j, columns = comps).
 *   acc   [num_ct][comps][L][N], natural order, not modified
 *   rot   device array of num_ct rotation amounts
 *   key   [comps * levels][comps][L][N], transform domain (the RGSW key)
 *   out   [num_ct][comps][L][N]; must not alias acc or key
 * Digit and size rules as ntt_external_product_decomposed.  For N <= 2^12 one
 * launch per class rotates, decomposes, transforms, multiplies-and-accumulates,
 * inverse-transforms and adds; other shapes go through a stream-ordered
 * workspace. */
ntt_status ntt_cmux(ntt_plan_t plan, void* out, const void* acc, const uint32_t* rot,
                    const void* key, uint32_t num_ct, uint32_t comps, uint32_t levels,
                    uint32_t log_base, void* stream);

/* Forward transforms of a and b in place (as ntt_forward on each) and their
 * elementwise product out = a (.) b (as ntt_pointwise_mul), from one pass over
 * the rows: the row pass that finishes both transforms also writes the product,
 * so the transformed operands are not read back.  All three [batch][L][N];
 * a, b and out distinct (else NTT_EINVAL).  The words equal those of the
 * separate calls. */
ntt_status ntt_forward_mul(ntt_plan_t plan, void* out, void* a, void* b, uint32_t batch,
                           void* stream);

/* Negacyclic product c = a * b mod (x^N + 1) per limb, through Eq. (1):
 * out, a, b are [batch][L][N] in natural order; a and b are not modified;
 * out must not alias a or b.  A two-pass product (N above the single-pass
 * length) takes a workspace of batch * L * N words from the device's default
 * memory pool, stream-ordered (hipMallocAsync / hipFreeAsync on `stream`);
 * callers that issue many products on several streams at once may prefer to
 * batch them per stream, as the request server does with its own arenas. */
ntt_status ntt_polymul(ntt_plan_t plan, void* out, const void* a, const void* b, uint32_t batch,
                       void* stream);

/* ntt_polymul for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, kernels and words, but the two-pass workspace comes from a
 * 64 MiB array that the library holds on each GPU it runs on until the process
 * ends, and the call allocates nothing (no hipMalloc / hipMallocAsync / free).
 *   - batch * L * N * (word_bits / 8) above 64 MiB for a two-pass product
 *     (N above the single-pass length) -> NTT_EINVAL; single-pass products
 *     need no workspace and take any batch ntt_polymul takes.
 *   - plans created with NTT_FLAG_VALIDATE -> NTT_EINVAL (the range check
 *     allocates a flag and waits for the stream).
 *   - every call on one GPU shares that GPU's array: calls that overlap in
 *     time on one GPU (several streams, unordered host threads) race on it and
 *     may return wrong words; order them on one stream.
 *   - the array's device address is looked up on the first call on each
 *     device (NTT_EDEVICE if that fails); that first call takes tens of
 *     milliseconds longer (the runtime loads the module's device globals), so
 *     a caller with a latency budget makes one call at set-up. */
ntt_status ntt_polymul_noalloc(ntt_plan_t plan, void* out, const void* a, const void* b,
                               uint32_t batch, void* stream);

/* ---- Ragged batches in one persistent launch ---------------------------- */

/* One job of a ragged batch under `plan` (any N >= 16, any limb count and
 * moduli), on [batch][L][N] device words of the plan's width:
 *   NTT_OP_FORWARD / NTT_OP_INVERSE  transform out in place (a, b NULL or out);
 *   NTT_OP_POLYMUL                   out = a * b mod (x^N + 1) per limb, as
 *                                    ntt_polymul (Eq. (1)); a and b are not
 *                                    modified, out must not overlap them. */
#define NTT_OP_FORWARD 0u
#define NTT_OP_INVERSE 1u
#define NTT_OP_POLYMUL 2u
typedef struct {
  ntt_plan_t plan;
  uint32_t op;     /* NTT_OP_FORWARD, NTT_OP_INVERSE or NTT_OP_POLYMUL */
  uint32_t batch;  /* polynomials in out (and in a, b) */
  void* out;       /* device words, [batch][L][N] */
  const void* a;   /* polymul operands, [batch][L][N] each */
  const void* b;
} ntt_job;

typedef struct ntt_ragged_s* ntt_ragged_t;

/* ntt_ragged_create flags. */
#define NTT_RAGGED_NO_GRAPH (1u << 0)           /* launch directly instead of replaying a hipGraph */
#define NTT_RAGGED_IN_WORKGROUP (1u << 1)       /* N >= 2^13 too in the persistent kernel (below) */
#define NTT_RAGGED_ROW_LOG(n2) (((uint32_t)(n2) & 0xfu) << 8) /* with NTT_RAGGED_IN_WORKGROUP: row length 2^n2 (11 or 12) */

/* Build a reusable ragged batch over jobs[0 .. n-1] (the paper's single kernel
 * launch for the hybrid NTT, Sec. V-D, applied to a mixed batch).  Jobs of
 * N <= 2^12 form a work list -- up to 16 limb-rows of one small N and kind per
 * item; a product item transforms a and b, multiplies and inverse-transforms
 * in registers/LDS -- built on the host, sorted largest first, uploaded once
 * and run by one persistent launch per word width.  Jobs of N >= 2^13 are
 * grouped by (N, arithmetic class, kind): every limb-row of a group goes into
 * one row table, and one column launch plus one row launch cover a transform
 * group (a product group: one column launch over both operands, the fused
 * product rows, one inverse column launch), as the batched calls do for one
 * plan.  With NTT_RAGGED_IN_WORKGROUP they go into the persistent kernel too
 * instead (one workgroup per limb-row, the intermediates kept with its CU).
 * Products with a column pass use a workspace of batch * L * N words per job,
 * allocated here and owned by the handle.  The plans and buffers named by the
 * jobs must stay valid for the life of the handle. */
ntt_status ntt_ragged_create(ntt_ragged_t* out, const ntt_job* jobs, uint32_t n, uint32_t flags);

/* Run the batch on `stream`: reset the work counter and launch the persistent
 * kernel(s) and the grouped launches.  Unless NTT_RAGGED_NO_GRAPH was given, the
 * first run captures these launches into a hipGraph and every run replays it.
 * Runs of one handle must not overlap in time (they share the work counter). */
ntt_status ntt_ragged_run(ntt_ragged_t r, void* stream);

/* Work items of a batch (persistent-kernel items plus the limb-rows of the
 * grouped launches) and persistent workgroups. */
ntt_status ntt_ragged_info(ntt_ragged_t r, uint32_t* items, uint32_t* workgroups);

ntt_status ntt_ragged_destroy(ntt_ragged_t r);

/* One-shot form: create, run without a graph, wait for `stream`, destroy. */
ntt_status ntt_batch_ragged(const ntt_job* jobs, uint32_t n, void* stream);

/* ---- Serving: continuous batching of requests ----------------------------- */

/* A request: one operation on `batch` polynomials of N coefficients over the
 * given moduli ([batch][L][N] words).  a, b (polymul only) and out are either
 * device pointers to resident operands (NTT_REQ_DEVICE) or host pointers
 * (preferably pinned) that the server copies in and out (NTT_REQ_HOST).  The
 * buffers must stay valid until the request completes. */
#define NTT_REQ_POLYMUL 0u
#define NTT_REQ_FORWARD 1u
#define NTT_REQ_INVERSE 2u
#define NTT_REQ_DEVICE 0u
#define NTT_REQ_HOST 1u
typedef struct {
  uint32_t op;            /* NTT_REQ_POLYMUL / FORWARD / INVERSE */
  uint32_t N;
  uint32_t word_bits;     /* 32 or 64 */
  uint32_t num_moduli;
  const uint64_t* moduli; /* copied at submit */
  uint32_t batch;
  uint32_t memory;        /* NTT_REQ_DEVICE or NTT_REQ_HOST */
  const void* a;
  const void* b;          /* polymul only */
  void* out;              /* may equal a for FORWARD/INVERSE */
} ntt_request;

/* Completion record of a request (times in seconds on the host's monotonic clock). */
typedef struct {
  uint64_t id;
  int32_t status;         /* NTT_OK, or the error that ended the request */
  uint32_t batched_with;  /* requests that shared its launch (1 = alone) */
  double t_submit, t_admit, t_launch, t_done;
  uint64_t bytes;         /* device bytes it held while in flight */
  uint64_t launch_id;     /* the launch it was part of (1, 2, ...) */
} ntt_request_info;

typedef struct {
  uint64_t submitted, completed, rejected;
  uint64_t launches;            /* batched launches issued */
  uint64_t max_inflight_bytes;  /* high-water mark, never above the budget */
  uint64_t max_inflight_requests;
  uint64_t budget_bytes;
  uint64_t plans_cached;
  uint64_t arena_bytes;         /* staging arenas held now (never above the budget) */
  uint64_t max_arena_bytes;     /* high-water mark of arena_bytes */
  uint64_t merged_launches;     /* launches whose requests had different moduli */
  uint64_t direct_launches;     /* batched two-pass polymul launches that read and wrote the
                                   requests' buffers in place (no gather or scatter copies) */
} ntt_server_counters;

typedef struct ntt_server_s* ntt_server_t;

/* Server flags. */
#define NTT_SERVER_SERIAL (1u << 0)   /* one request at a time, FIFO, no batching: the baseline */
#define NTT_SERVER_DRY_RUN (1u << 1)  /* no device work: a batch "completes" after a modelled
                                         time; admission/batching logic testable without a GPU */
#define NTT_SERVER_MERGE_MODULI (1u << 2) /* also batch requests whose moduli differ but share
                                           one arithmetic class (one launch over their limbs) */

/* Create a server: a host thread that admits requests while their device bytes
 * fit in budget_bytes (HBM admission), groups admitted requests into one launch
 * (continuous batching: requests that arrive while others run join the next
 * launch), and keeps up to n_streams launches in flight on separate streams.
 * Requests share a launch when op, N, word width, memory kind and moduli match;
 * with NTT_SERVER_MERGE_MODULI also when only the moduli differ and all of
 * them fall in one arithmetic class (at most 4096 limb-rows per such launch).
 * A submit checks each distinct modulus once per server.  Plans and their twiddle
 * tables stay resident for the server's life.  max_batch caps the polynomials
 * per launch (0 = 4096); a launch also takes at most 64 requests.  A batched
 * polymul of device-resident requests whose transforms take two passes reads
 * and writes the requests' buffers in place (row-address tables); other
 * batched operands are staged in a per-stream device arena.  Arenas (also
 * holding intermediates and workspaces) grow on demand and are reused in
 * stream order; together they stay within budget_bytes (another stream's arena
 * is released, after its stream has drained, when growing one would pass it). */
ntt_status ntt_server_create(ntt_server_t* out, uint64_t budget_bytes, uint32_t n_streams,
                             uint32_t max_batch, uint32_t flags);

/* Queue a request; *id identifies it.  A request holds, while in flight, its
 * operand bytes times 4 (polymul: inputs, output, workspace) or 2 (transforms)
 * plus 128 bytes per limb-row and 1 KiB (staged constants, row tables,
 * alignment).  A request larger than the budget is rejected here with NTT_ENOMEM, one of batch * L * N >= 2^32 words with
 * NTT_EINVAL.  A launch gathers requests only while their words stay below
 * 2^32 (the library's per-call limit), so a request that succeeds alone also
 * succeeds in any mix; its result is the same word for word. */
ntt_status ntt_server_submit(ntt_server_t s, const ntt_request* r, uint64_t* id);

/* Wait for request `id` (timeout_ms < 0: forever); fills *info and forgets the
 * request.  NTT_ETIMEOUT if it did not complete in time. */
ntt_status ntt_server_wait(ntt_server_t s, uint64_t id, ntt_request_info* info, int32_t timeout_ms);

/* Submit reqs[i] at arrival_s[i] seconds after the call starts (a load
 * generator that runs at native speed; arrival_s must be non-decreasing).
 * Returns once every request is submitted; ids[i] receives each id (0 for
 * requests not submitted after an error). */
ntt_status ntt_server_replay(ntt_server_t s, const ntt_request* reqs, const double* arrival_s,
                             uint32_t n, uint64_t* ids);

ntt_status ntt_server_counters_get(ntt_server_t s, ntt_server_counters* c);

/* Stop accepting, finish everything queued, join the thread, free everything. */
ntt_status ntt_server_destroy(ntt_server_t s);

/* ---- Autotuner ------------------------------------------------------------ */

/* Time every admissible pass split for (N, moduli, word_bits) on `batch`
 * polynomials of scratch data (forward + inverse, HIP events on an internal
 * stream, the fastest of three timed groups per configuration), record the
 * fastest in the library's tuning table and return it.
 * Later calls with a similar number of limb-rows (same power-of-two bucket of
 * batch * L) and no forced split use it.  The paper's switch trigger (chunks
 * closest to the SM count, Sec. V-D) is for one polynomial; a batch changes the
 * concurrency, so the split is measured per (N, class, rows).  Each split is
 * timed with 16, 8 and 4 values per row-pass thread (where built) and the
 * fastest is kept per direction; at the chosen split, column passes of 256, 128
 * and 64 columns (threads) per workgroup are timed and the fastest kept;
 * polymul rows at the chosen split are timed with 16 and 8 values per thread
 * when a second scratch buffer of the same size can be allocated. */
ntt_status ntt_tune_split(uint32_t N, const uint64_t* moduli, uint32_t num_moduli,
                          uint32_t word_bits, uint32_t batch, uint32_t* best_n1, float* best_us);

/* Time row lengths 2^11 and 2^12 for the in-workgroup split of ragged batches
 * (NTT_RAGGED_IN_WORKGROUP) with this N (>= 2^13) and record the faster;
 * returns log2 of the row length. */
ntt_status ntt_tune_ragged(uint32_t N, const uint64_t* moduli, uint32_t num_moduli,
                           uint32_t batch, uint32_t* best_row_log, float* best_us);

/* Save / load / clear the tuning table (a small JSON file).  At first use the
 * library loads the file named by the environment variable NTT_TUNE_FILE, if set. */
ntt_status ntt_tune_save(const char* path);
ntt_status ntt_tune_load(const char* path);
ntt_status ntt_tune_clear(void);

/* Per-kernel timing of this library's own launches (tracing).  While enabled,
 * every kernel launch is bracketed by two HIP events recorded on the stream the
 * kernel is launched on.  ntt_stats_collect() waits for the recorded events and
 * fills out[0 .. min(cap, count)-1] with one entry per kernel name (sorted by
 * name); *count receives the number of names.  Aggregates persist until
 * ntt_stats_reset().  Enabling adds two event records per launch. */
typedef struct {
  char name[64];      /* e.g. "row_fwd_f64l_log12_2pass" */
  uint64_t launches;  /* launches recorded */
  uint64_t words;     /* coefficient words covered, summed over launches */
  double total_ms;    /* summed device time between each launch's two events */
} ntt_kernel_stat;

ntt_status ntt_stats_enable(int on);
ntt_status ntt_stats_reset(void);
ntt_status ntt_stats_collect(ntt_kernel_stat* out, uint32_t cap, uint32_t* count);

/* Testing aid for the bounded waits of persistent launches (NTT_FLAG_FUSED):
 * polls = polls before a wait gives up (0 restores the default, 2^20);
 * force_expire != 0 makes every wait's target unreachable, so each wait gives
 * up after `polls` polls and the call reports NTT_ETIMEOUT while every kernel
 * still exits normally.  Process-wide; affects calls issued afterwards. */
ntt_status ntt_debug_wait_limit(uint32_t polls, uint32_t force_expire);

/* Host-only helpers (no device needed). */

/* Admission check of one modulus for (N, word_bits): NTT_OK or the error a
 * plan would report for it. */
ntt_status ntt_check_modulus(uint32_t N, uint64_t q, uint32_t word_bits);

/* The root psi a plan would use for (N, q). */
ntt_status ntt_find_root(uint32_t N, uint64_t q, uint64_t* psi);

/* Thread-local description of the last error on this thread ("" if none). */
const char* ntt_last_error(void);

/* Library version string. */
const char* ntt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NTT_MI355X_H */
