/*
 * mick.h - C ABI of libmick, the k-input RNS-CKKS ciphertext multiply on
 * AMD MI355X (gfx950).
 *
 * The library multiplies k ciphertexts (k = 2..12) that share one secret key
 * s and one modulus Q_l = q_0 ... q_{l-1}, relinearises the degree-k result
 * with evaluation keys for s^2 .. s^k by hybrid key switching (ModUp by fast
 * basis conversion, key inner product, ModDown), and applies k - 1
 * rescalings combined into one multi-level rescale, following
 * "Multi-Input Ciphertext Multiplication for Homomorphic Encryption"
 * (Sec. II: RNS-CKKS, BConv, ModDown, rescale; Sec. III: the combined ModDown
 * of eq. (product3); Sec. IV: the relocated ModDown of eqs. (moddown improved)
 * and (scBconv) with P^-1 folded into the keys; Sec. V-A: eq. (d_u formula
 * for n-ct mult), the keys of eq. (evks of ct mult for s^t) and eq. (extended
 * relin); Sec. V-B: Algorithm 1 and eq. (multi rs)).
 *
 * Conventions (binding for every call):
 *  - Residues are uint32, canonical in [0, m).  A polynomial over l limbs is
 *    stored limb-major, uint32[l][N]; limb j holds the residues mod q_j.  A
 *    ciphertext is uint32[2][l][N] (c0 then c1), in the NTT domain.
 *  - Primes: q_i is the (i+1)-th largest prime below 2^30 with q = 1 mod 2N,
 *    p_i the same below 2^31.  psi_m is the smallest x >= 2 with
 *    x^N = -1 mod m.  NTT(a)[k] = a(psi^(2 brv(k) + 1)) mod m, brv the
 *    log2(N)-bit reversal.
 *  - Hybrid key switching with dnum digits: alpha = ceil(L / dnum); digit b
 *    holds q_{b alpha} .. q_{min((b+1) alpha, l) - 1} at level l.
 *  - Rescaling drops the highest active primes first (q_{l-1}, q_{l-2}, ...);
 *    the dropped residue enters eq. (1-rs) as its representative in
 *    [0, q_{l-1}), so mu rescales compute floor(x / (q_{l-1} ... q_{l-mu})).
 *  - Random streams (keys, encryption noise; the paper fixes no generator):
 *    SplitMix64 in counter mode, draw(key, n) = mix64(key + (n+1) G) with
 *    G = 0x9E3779B97F4A7C15; a stream key is h = mix64(seed + G), then
 *    h = mix64((h ^ w) + G) for w in (tag, a, b, c), the tag being up to 8
 *    ASCII bytes little-endian.  Uniform mod m: draw(n) mod m (drawn directly
 *    as NTT-domain values).  Ternary of weight h: partial Fisher-Yates, step
 *    i swaps in position i + draw(2i) mod (N - i), sign + if draw(2i+1) is
 *    even.  Gaussian (sigma = 3.2): the smallest x in [-19, 19] whose
 *    cumulative threshold floor(2^64 C(x) / S) exceeds draw(n), the
 *    cumulative sums of exp(-x^2 / 2 sigma^2) taken in FP64 from x = -19.
 *    Secret weight h = 64.  Tags: SK; PK_A (limb); PK_E; EVK_A (t, b, row);
 *    EVK_E (t, b); ENC_V, ENC_E0, ENC_E1 (ct_id).
 *  - "Device" pointers are HIP device memory owned by the caller; "host"
 *    pointers are ordinary host memory owned by the caller.  Calls taking a
 *    stream (a hipStream_t passed as void*, NULL = the default stream) are
 *    asynchronous on that stream unless stated otherwise; the caller keeps
 *    the buffers alive until the stream work completes.  The library keeps
 *    no caller pointer after a call returns.
 *  - Every call returns MICK_OK (0) or a negative status; nothing throws or
 *    aborts.  mick_last_error() gives a thread-local message for the last
 *    failing call on the calling thread.
 */
#ifndef MICK_H
#define MICK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MICK_OK = 0,
  MICK_E_ARG = -1,    /* NULL pointer, size or range error in an argument */
  MICK_E_LEVEL = -2,  /* level < k, level > L, or mu >= level */
  MICK_E_KEY = -3,    /* k larger than the key set's k_max */
  MICK_E_NOMEM = -4,  /* device or host allocation failed */
  MICK_E_HIP = -5,    /* a HIP runtime call failed (detail in mick_last_error) */
  MICK_E_RANGE = -6,  /* a decrypted coefficient does not fit the output type */
  MICK_E_WS = -7,     /* workspace smaller than mick_workspace_bytes() */
  MICK_E_BUSY = -8,   /* a queued job's workspace exceeds the queue's memory budget,
                         or a job asked to be cancelled is already running */
  MICK_E_CANCELLED = -9, /* per-job status: removed from a queue by mick_queue_cancel */
  MICK_PENDING = 1    /* per-job status only: accepted by a queue, not yet complete */
};

typedef struct mick_params mick_params;
typedef struct mick_keys mick_keys;
typedef struct mick_plan mick_plan;

const char* mick_strerror(int status);
const char* mick_last_error(void);

/* ---------------------------------------------------------------- params
 * Ring degree N = 2^log_n (13 <= log_n <= 16), L ciphertext primes
 * (1 <= L <= 60), K special primes (1 <= K <= 24), dnum digits with
 * alpha = ceil(L / dnum) <= 32 primes each and at most 16 digits.  dnum = 1
 * with K >= L is the setting of the paper's evaluation (Sec. VI).
 * Builds the primes, NTT twiddle tables, basis conversion tables and
 * rescaling constants of Sec. II and Sec. V-B, and
 * uploads them to the current HIP device (synchronous).  The handle is
 * immutable and may be shared by threads and streams; free it with
 * mick_params_destroy (NULL-safe) after all work using it has completed. */
int mick_params_create(int log_n, int L, int K, int dnum, mick_params** out);
/* The scale of a multiply's output (Sec. II rescaling: each rescale divides
 * the scale by the dropped prime): prod_u scales_host[u] over
 * prod q_{level-k+1} .. q_{level-1}, the k - 1 primes the multiply drops at
 * `level`.  The library tracks no scale of its own: the ring arithmetic of
 * the multiply does not depend on it, so it is the caller's (Sec. V-B, the
 * scale after mu rescales of a product of k ciphertexts).  Host only. */
int mick_output_scale(const mick_params* prm, const double* scales_host, int k, int level, double* out_host);
void mick_params_destroy(mick_params* prm);
/* Host copies of q_0..q_{L-1} (L values) and p_0..p_{K-1} (K values). */
int mick_params_moduli(const mick_params* prm, uint32_t* q_host, uint32_t* p_host);
/* log_n, L, K, dnum, alpha in out5_host[0..4]. */
int mick_params_shape(const mick_params* prm, int* out5_host);

/* ---------------------------------------------------------------- keys
 * Seeded key generation (Sec. II public key; Sec. V-A eq. (evks of ct mult
 * for s^t) generalised to dnum digits: the q_j rows of key (t, b) carry
 * P G_b s^t with G_b = Qhat_b [Qhat_b^-1]_{Q_b}).  Keys for t = 2..k_max and
 * every digit live in device memory owned by the handle; the device copy
 * of each evaluation key has its q rows multiplied by [P^-1]_{q_j}
 * (Sec. IV).  Synchronises `stream` before returning.  2 <= k_max <= 12. */
int mick_keygen(const mick_params* prm, uint64_t seed, int k_max, void* stream, mick_keys** out);
void mick_keys_destroy(mick_keys* keys);
int mick_keys_kmax(const mick_keys* keys);
/* Canonical key material copied to host memory (synchronous):
 *  what = 0: secret s as int64 coefficients, N values (t, b ignored);
 *  what = 1: public key (b, a), uint32[2][L][N], NTT domain;
 *  what = 2: evaluation key (t, b) in the form of eq. (evks of ct mult for
 *            s^t), unscaled, uint32[2][L+K][N], rows q_0..q_{L-1},
 *            p_0..p_{K-1}, NTT domain. */
int mick_keys_export(const mick_keys* keys, int what, int t, int b, void* host_out, void* stream);

/* ---------------------------------------------------------------- codec
 * CKKS canonical embedding in FP64 on the host (the paper does not describe
 * encoding): N/2 slots, slot j at zeta_j = exp(i pi (5^j mod 2N) / N);
 * m_i = round((2/N) Re sum_j scale z_j zeta_j^-i), half away from zero.
 * n_slots must be N/2. */
int mick_encode(const mick_params* prm, const double* re_host, const double* im_host, size_t n_slots,
                double scale, int64_t* m_host);
/* z_j = m(zeta_j) / scale, the inverse of mick_encode up to rounding. */
int mick_decode(const mick_params* prm, const int64_t* m_host, double scale, double* re_host, double* im_host,
                size_t n_slots);

/* ---------------------------------------------------------------- encryption
 * Public-key encryption (Sec. II): (c0, c1) = (m + v b + e0, v a + e1) at
 * `level` (1..L), v ternary of weight N/2, e0 and e1 Gaussian, drawn from
 * the streams of (seed, ct_id).  m_host: N int64 coefficients (already
 * scaled).  ct_dev: device uint32[2][level][N], NTT domain.  Synchronises
 * `stream` before returning (host inputs are staged). */
int mick_encrypt(const mick_params* prm, const mick_keys* keys, const int64_t* m_host, int level, uint64_t seed,
                 uint64_t ct_id, uint32_t* ct_dev, void* stream);
/* Coefficient-domain residues of c0 + c1 s over q_0..q_{level-1}, copied to
 * res_host uint32[level][N] (synchronous). */
int mick_decrypt_residues(const mick_params* prm, const mick_keys* keys, const uint32_t* ct_dev, int level,
                          uint32_t* res_host, void* stream);
/* c0 + c1 s reconstructed by CRT over the active primes and centred into
 * (-Q/2, Q/2]; MICK_E_RANGE if a coefficient needs more than 62 bits
 * (Sec. II decryption, read over every active limb). */
int mick_decrypt(const mick_params* prm, const mick_keys* keys, const uint32_t* ct_dev, int level, int64_t* m_host,
                 void* stream);

/* ---------------------------------------------------------------- hot path
 * Operation codes for mick_workspace_bytes. */
enum { MICK_OP_RELIN = 1, MICK_OP_RESCALE = 2, MICK_OP_MUL_RELIN_RESCALE = 3 };

/* Device workspace needed by one call of `op` at (k, level); for
 * MICK_OP_RESCALE, k is read as mu.  0 for invalid arguments. */
size_t mick_workspace_bytes(const mick_params* prm, int op, int k, int level);

/* Tensor product, eq. (d_u formula for n-ct mult): from k NTT-domain
 * ciphertexts at `level` (cts_host: host array of k device pointers, each
 * uint32[2][level][N]) computes d_0..d_k, d_t = sum over l in {0,1}^k with
 * |l| = t of prod_u c^u_{l_u}, pointwise per limb.  d_dev: device
 * uint32[k+1][level][N], NTT domain.  2 <= k <= 12. */
int mick_mul_k(const mick_params* prm, const uint32_t* const* cts_host, int k, int level, uint32_t* d_dev,
               void* stream);

/* Relinearisation of eq. (extended relin) with one ModDown per output
 * polynomial (Sec. III): (c0*, c1*) = (d_0, d_1) + ceil(P^-1 sum_t d_t ek_t)
 * using the relocated ModDown of Sec. IV.  d_dev: device uint32[k+1][level]
 * [N] (NTT domain, as written by mick_mul_k); ct_out_dev: device
 * uint32[2][level][N], NTT domain.  ws: device workspace of at least
 * mick_workspace_bytes(MICK_OP_RELIN, k, level) bytes. */
int mick_relin_k(const mick_params* prm, const mick_keys* keys, const uint32_t* d_dev, int k, int level,
                 uint32_t* ct_out_dev, void* ws, size_t ws_bytes, void* stream);

/* mu consecutive rescalings of an NTT-domain ciphertext by Algorithm 1
 * (Sec. V-B): mu INTTs, the rescale chain of the dropped limbs, and
 * level - mu NTTs.  ct_in_dev uint32[2][level][N] -> ct_out_dev
 * uint32[2][level-mu][N] (must not overlap the input).  1 <= mu < level,
 * mu <= 16. */
int mick_rescale_multi(const mick_params* prm, const uint32_t* ct_in_dev, int level, int mu, uint32_t* ct_out_dev,
                       void* ws, size_t ws_bytes, void* stream);

/* The whole k-input multiply: tensor product, relinearisation with the
 * relocated ModDown (Sec. IV), and mu = k - 1 rescalings combined in the
 * coefficient domain by eq. (multi rs) followed by one NTT (the RS* of
 * Sec. IV).  cts_host: host array of k device pointers uint32[2][level][N];
 * ct_out_dev: device uint32[2][level-k+1][N], NTT domain.  k <= level <= L. */
int mick_mul_relin_rescale(const mick_params* prm, const mick_keys* keys, const uint32_t* const* cts_host, int k,
                           int level, uint32_t* ct_out_dev, void* ws, size_t ws_bytes, void* stream);

/* The same multiply for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no workspace argument and no allocation of any kind; the
 * workspace is a static device array of 64 MiB (67108864 bytes) inside the
 * library, one per device, held until the process ends.  MICK_E_WS when
 * mick_workspace_bytes(prm, MICK_OP_MUL_RELIN_RESCALE, k, level) exceeds it
 * (for instance N = 2^16 beyond small levels); nothing is launched then.
 * Every call on one device shares that array: calls that overlap on a
 * device (other streams, other threads) race, so the caller serialises
 * them.  The multiply writes every workspace word it reads, so nothing has
 * to be cleared between calls. */
int mick_mul_relin_rescale_noalloc(const mick_params* prm, const mick_keys* keys, const uint32_t* const* cts_host,
                                   int k, int level, uint32_t* ct_out_dev, void* stream);

/* n_jobs (1..64) independent multiplies of the same (k, level) in one
 * sequence of launches, each kernel covering every job; the key inner
 * product reads each evaluation key element once for up to 8 jobs.
 * cts_dev: device uint32[n_jobs][k][2][level][N] (job-major, contiguous);
 * outs_dev: device uint32[n_jobs][2][level-k+1][N].  Results are
 * bit-identical to n_jobs calls of mick_mul_relin_rescale.  ws: at least
 * mick_batch_workspace_bytes() bytes. */
size_t mick_batch_workspace_bytes(const mick_params* prm, int n_jobs, int k, int level);
int mick_mul_relin_rescale_batch(const mick_params* prm, const mick_keys* keys, const uint32_t* cts_dev, int n_jobs,
                                 int k, int level, uint32_t* outs_dev, void* ws, size_t ws_bytes, void* stream);

/* One k-input multiply of a heterogeneous batch. */
typedef struct mick_job {
  int k;                     /* 2..12, at most the key set's k_max */
  int level;                 /* k..L */
  const uint32_t* cts[12];   /* k device pointers, uint32[2][level][N] each */
  uint32_t* out;             /* device uint32[2][level-k+1][N] */
  int* status;               /* host, optional: the job's own status (see below) */
} mick_job;

/* Workspace for mick_mul_relin_rescale_jobs: a job table plus one multiply
 * workspace per job.  A job with a status pointer whose (k, level) is out of
 * range counts no workspace (it will be left out); any other such job makes
 * the result 0. */
size_t mick_jobs_workspace_bytes(const mick_params* prm, const mick_job* jobs, int n_jobs);

/* n_jobs (1..65536) multiplies of one parameter set whose k and level may
 * differ, each bit-identical to mick_mul_relin_rescale.  Every stage of the
 * multiply is a single launch over a device job table (the tensor product
 * and the rescale are launched once per distinct k); each workgroup looks
 * its job up in the table.  jobs: host array; the table is copied into the
 * workspace (the copy reads `jobs` before the call returns).
 * Failure isolation: a job with a status pointer is validated on its own;
 * if it is invalid its error code (MICK_E_ARG, MICK_E_LEVEL, MICK_E_KEY) is
 * written there and it is left out while the other jobs run; a valid one
 * gets MICK_OK.  An invalid job without a status pointer fails the whole
 * call before anything is launched. */
int mick_mul_relin_rescale_jobs(const mick_params* prm, const mick_keys* keys, const mick_job* jobs, int n_jobs,
                                void* ws, size_t ws_bytes, void* stream);

/* The same in two steps.  mick_jobs_plan validates the jobs, writes the job
 * table (the device work queue) into the workspace with an asynchronous
 * copy on `stream` and returns a host-side plan; mick_plan_execute enqueues
 * only kernel launches that read the table, so it can be captured into a HIP
 * graph and replayed.  The plan refers to the workspace and to the jobs'
 * buffers, which must stay allocated while it is used; mick_plan_destroy
 * (NULL-safe) frees only the host object. */
int mick_jobs_plan(const mick_params* prm, const mick_keys* keys, const mick_job* jobs, int n_jobs, void* ws,
                   size_t ws_bytes, void* stream, mick_plan** out);
int mick_plan_execute(const mick_plan* plan, void* stream);
void mick_plan_destroy(mick_plan* plan);

/* ---------------------------------------------------------------- basis conversion
 * The fast basis conversion of Sec. II, eq. (basis conversion), standalone,
 * for n_polys polynomials of one digit: src_dev uint32[n_polys][na][N], the
 * digit's na primes q_{b alpha} .. in the coefficient domain (canonical);
 * dst_dev uint32[n_polys][level + K - na][N], the conversion into every
 * other active q prime in ascending order, then p_0..p_{K-1}:
 * out_e = sum_a [x_a qhat_a^-1]_{q_a} qhat_a mod m_e.  method 0: 64-bit
 * multiply-add chains on the vector ALUs (the arithmetic of the fused ModUp
 * kernel); method 1: int8 matrix cores on signed-byte splits with exact
 * recombination.  Both give the same residues; digits of at most 8 primes.
 * The conversion tables of a (level, digit) are built on first use (device
 * memory from the registered allocator, kept until the parameters are
 * destroyed).  Exposed to measure the two forms; the multiply itself runs
 * the conversion inside its ModUp kernel. */
int mick_bconv(const mick_params* prm, const uint32_t* src_dev, int n_polys, int level, int digit, uint32_t* dst_dev,
               int method, void* stream);

/* ---------------------------------------------------------------- tree multiply
 * Sec. V-C: the n inputs are partitioned into groups, recursively.  A node
 * multiplies the results of its children as polynomials in s (a group of g
 * inputs is the product of g ciphertexts, eq. (d_u formula for n-ct mult));
 * every node but the root then rescales each polynomial of its product by
 * (fan-in - 1) levels with Algorithm 1 (Sec. V-B) in the NTT domain; the
 * root relinearises its degree-n product with the keys for s^2..s^n and
 * applies the relocated ModDown and (fan-in - 1)-level rescale of Sec. IV and
 * eq. (multi rs).  The multiplicative depth is that of the tree (the flat
 * multiply is the single group n, depth n - 1).
 *
 * A tree is an array of prefix tokens: g > 0 is a group of g consecutive
 * inputs, -m (m >= 2) an internal node whose m subtrees follow.  Table II's
 * "(4,3)|(2,2)" is {-2, -2, 2, 2, 3}.  Every subtree is evaluated at the
 * level at which its result enters its parent: its inputs first drop their
 * top limbs (the placement Table II's (I)NTT counts imply).
 *
 * mick_tree_plan writes the partition of n inputs (2..32) with the fewest
 * rescale units (one per polynomial rescaled before relinearisation) at
 * depth ceil(log2 n) (Sec. V-C, Table II); returns the number of tokens.
 * mick_tree_shape validates a tree and reports its inputs, depth and units
 * (any output pointer may be NULL).
 * mick_mul_tree multiplies n = 2..12 ciphertexts cts_host[u] (device
 * uint32[2][level][N], NTT domain) with keys up to s^n; the output is
 * device uint32[2][level - depth][N], NTT domain; its scale is Delta^n over
 * the product of every prime dropped by the tree's rescales (the caller
 * tracks scales).  ws: at least mick_tree_workspace_bytes() bytes (0 for an
 * invalid tree or level). */
int mick_tree_plan(int n, int* tokens, int max_tokens);
int mick_tree_shape(const int* tokens, int n_tokens, int* n_inputs, int* depth, int* rs_units);
size_t mick_tree_workspace_bytes(const mick_params* prm, const int* tokens, int n_tokens, int level);
int mick_mul_tree(const mick_params* prm, const mick_keys* keys, const uint32_t* const* cts_host, int level,
                  const int* tokens, int n_tokens, uint32_t* ct_out_dev, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- work queue
 * A host-driven queue of multiplies over one or more parameter sets (for
 * instance the four ring degrees of a mixed workload), with admission by
 * device memory.  The queue owns one device workspace arena of `capacity`
 * bytes (from the registered allocator), allocated at creation.
 *
 *  - mick_queue_push appends jobs to a FIFO; it launches nothing.  A job
 *    with a status pointer is accepted or refused on its own: refused, its
 *    error code is written there (MICK_E_BUSY if its workspace alone exceeds
 *    the queue's capacity); accepted, MICK_PENDING is written, then MICK_OK
 *    when mick_queue_poll or mick_queue_drain sees it complete.  Jobs
 *    without a status pointer are all or none: one invalid such job rejects
 *    the call and nothing is appended.
 *  - mick_queue_cancel removes the pending jobs with a given id (status
 *    MICK_E_CANCELLED); MICK_E_BUSY if that id has already been launched,
 *    MICK_E_ARG if no job with it is pending or running.
 *  - mick_queue_run admits pending jobs in FIFO order while the workspace of
 *    each fits a free block of the arena (first fit; it stops at the first
 *    job that does not fit, so admission stays in arrival order), groups the
 *    admitted jobs by parameter set and launches each group as one job-table
 *    plan (see mick_jobs_plan) on `stream`, smaller ring degrees first, each
 *    group followed by its own completion event.  It returns the number of
 *    jobs launched (0 if none fitted or none were pending) and does not wait.
 *  - mick_queue_poll writes the ids of completed jobs (at most max) to
 *    done_ids, returns their number and frees their workspace.  Completion
 *    follows each group's event, so groups launched on different streams may
 *    complete in any order.
 *  - mick_queue_drain runs and polls until every pushed job has completed,
 *    waiting on the oldest running group whenever nothing more fits; the
 *    ids of the jobs it completes are discarded (poll first to keep them).
 *  - mick_queue_info reports pending jobs, running jobs and arena bytes in
 *    use (any pointer may be NULL).
 *  - mick_queue_destroy (NULL-safe) waits for running groups, then frees the
 *    arena.
 * The queue keeps the jobs' ciphertext and output pointers until they
 * complete; the caller keeps those buffers, the parameter sets and the keys
 * alive meanwhile.  A queue is driven by one host thread at a time.
 * Results are bit-identical to mick_mul_relin_rescale of each job alone. */
typedef struct mick_queue mick_queue;

typedef struct mick_qjob {
  uint64_t id;               /* caller's tag, returned by mick_queue_poll */
  int set;                   /* index into the queue's parameter sets */
  int k;                     /* 2..12, at most that set's key k_max */
  int level;                 /* k..L of that set */
  const uint32_t* cts[12];   /* k device pointers, uint32[2][level][N] each */
  uint32_t* out;             /* device uint32[2][level-k+1][N] */
  int* status;               /* host, optional: kept by the queue until the job completes */
} mick_qjob;

/* prms, keys: host arrays of n_sets (1..16) handles, keys[i] generated for
 * prms[i].  capacity: arena bytes; a job whose workspace alone exceeds it is
 * rejected by mick_queue_push. */
int mick_queue_create(const mick_params* const* prms, const mick_keys* const* keys, int n_sets, size_t capacity,
                      mick_queue** out);
/* Device workspace one job holds while it runs (what admission counts). */
size_t mick_queue_job_bytes(const mick_queue* q, int set, int k, int level);
int mick_queue_push(mick_queue* q, const mick_qjob* jobs, int n_jobs);
int mick_queue_run(mick_queue* q, void* stream);
int mick_queue_poll(mick_queue* q, uint64_t* done_ids, int max);
int mick_queue_cancel(mick_queue* q, uint64_t id);
int mick_queue_drain(mick_queue* q, void* stream);
int mick_queue_info(const mick_queue* q, int* pending, int* running, size_t* bytes_in_use);
void mick_queue_destroy(mick_queue* q);

/* ---------------------------------------------------------------- schedule
 * Three settings of a parameter set change how the multiply runs, never its
 * result:
 *  - the split of log N into a first transform pass over 2^a rows and a
 *    second over 2^(log N - a) (a in {7, 8} where the passes fit: N = 2^14
 *    and 2^15 have both, N = 2^13 only a = 7, N = 2^16 only a = 8);
 *  - the tensor-product method (mick_params_set_tensor_method);
 *  - ModUp targets per workgroup (1 or 2; 2 only for digits of 5 to 8
 *    primes, where each source word loaded then feeds two conversions).
 * mick_autotune times the fused multiply of a batch of two jobs at
 * k = min(8, L) and level L on the current device (synthetic keys and
 * inputs, allocated for the run and freed) under every combination, in
 * three interleaved rounds, and keeps the combination with the smallest
 * median time.  With a cache file it first looks up the (device, N, L, K,
 * dnum) entry and appends the result after timing (NULL: the path in the
 * environment variable MICK_AUTOTUNE_CACHE, else no cache).
 * mick_autotune_report copies the last timing run's table (configs
 * [max][3]: a, tensor method, ModUp targets; us: microseconds per multiply)
 * and returns its length (0 after a cache hit).  Changing the split
 * rebuilds the parameter tables (device work, synchronous): call these
 * before jobs are queued with the parameters, never while work using them
 * is in flight.  mick_params_schedule reports a. */
int mick_autotune(mick_params* prm, const char* cache_path);
int mick_autotune_report(const mick_params* prm, int max, int* configs, double* us);
int mick_params_set_schedule(mick_params* prm, int first_pass_log);
int mick_params_schedule(const mick_params* prm);
int mick_params_set_modup_targets(mick_params* prm, int targets);
int mick_params_modup_targets(const mick_params* prm);
/* How the fused multiply forms d_0..d_k of eq. (d_u formula for n-ct mult)
 * (every method gives the same residues):
 *  0  one linear factor at a time, prod_{v<=u} (c0^v + c1^v Y), each new
 *     coefficient an exact sum of two products reduced once;
 *  1  a balanced binary tree of products of polynomials in Y, each node
 *     coefficient an exact sum of its products reduced once;
 *  2  the same tree with the reduced-multiplication forms at its nodes
 *     (Karatsuba, Sec. II, for two linear factors and, on two levels, for
 *     two cubics; the 3-parallel fast filter iterated as Sec. V-A suggests,
 *     for two quadratics).
 * The setting is read at launch; change it only while no work using the
 * parameters is in flight.  mick_params_tensor_method reports it. */
int mick_params_set_tensor_method(mick_params* prm, int method);
int mick_params_tensor_method(const mick_params* prm);

/* ---------------------------------------------------------------- allocator
 * Device memory of the library's own objects (parameter tables, keys,
 * queue arenas, temporary buffers of encryption and decryption) comes from
 * this allocator; by default hipMalloc / hipFree.  alloc(bytes, ctx) returns
 * device memory aligned to 256 bytes or NULL; release(ptr, ctx) frees it.
 * Process-wide; each object keeps the pair in force at its creation and
 * frees its memory with it.  Pass NULL, NULL to restore the default. */
typedef void* (*mick_alloc_fn)(size_t bytes, void* ctx);
typedef void (*mick_free_fn)(void* ptr, void* ctx);
int mick_set_allocator(mick_alloc_fn alloc, mick_free_fn release, void* ctx);

/* Forward / inverse negacyclic NTT of n_limbs limbs in place, limb i taken
 * mod prime index first_prime + i (prime index j < L is q_j, L + i is p_i).
 * Exposed for testing and benchmarking of the transform itself. */
int mick_ntt(const mick_params* prm, uint32_t* data_dev, int n_limbs, int first_prime, int inverse, void* stream);

/* ---------------------------------------------------------------- instrumentation
 * Not part of the paper's method: timing support for benchmarks.  While
 * enabled, every kernel launch of the library is bracketed by a pair of HIP
 * events recorded on the launch's stream (process-wide switch). */
int mick_profile_enable(int on);
/* Restricts the recording to the named launch sites (comma-separated names
 * as mick_profile_collect reports them, e.g. "modup_bconv_passA"); NULL or
 * "" selects every site (the default).  MICK_E_ARG for an unknown name, the
 * selection then unchanged.  Needs no device. */
int mick_profile_select(const char* sites);
/* Waits for the recorded events, then returns the number of launch sites
 * seen (at most `max`) with, per site, a static name, the summed kernel time
 * in milliseconds and the number of launches; clears the records. */
int mick_profile_collect(int max, const char** names, double* total_ms, int* launches);

#ifdef __cplusplus
}
#endif

#endif /* MICK_H */
