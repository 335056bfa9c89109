/*
 * lfs.h -- C ABI of the MI355X (gfx950) library for flow-based sampling of
 * lattice phi^4 theory, after arXiv 2208.08903 (GomalizingFlow.jl).
 *
 * The library computes, on one GPU, the data-parallel hot path of the method:
 * Gaussian prior draws, the RealNVP flow of checkerboard affine coupling layers
 * with convolutional s/t networks (forward with log q, and its hand-written
 * backward), the lattice action and its force, log-weights and the reverse-KL
 * loss, the independence Metropolis-Hastings chain, the HMC baseline, and Adam.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every pointer argument is a DEVICE pointer to contiguous memory, unless
 *    the argument is documented as host memory.  The caller owns every buffer,
 *    including the workspace; the library never allocates or frees device
 *    memory inside these calls.  Its only global state is the static device
 *    scratch of lfs_flow_forward_noalloc and that array's per-device address.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *    Calls are asynchronous on that stream: inputs must stay unchanged and
 *    outputs must not be read until the stream reaches the call.
 *  - Arguments are validated synchronously, before anything is enqueued.  An
 *    invalid call returns a negative lfs_status and enqueues nothing.  A failed
 *    kernel launch returns LFS_EDEVICE.  No exception, print or abort crosses
 *    the ABI.
 *  - Lattice fields are stored [B][n_0]...[n_{d-1}] row-major (last axis
 *    fastest), one sample after another: index b*V + site, V = L^dim.  The
 *    lattice is periodic in every direction.
 *  - Site parity is p(n) = (sum_mu n_mu) mod 2 with 0-based coordinates.
 *  - An empty batch (B == 0, n_chains == 0) is a no-op for the per-sample
 *    entry points (prior draws, flow forward, action, MH chains, HMC,
 *    observables): they return LFS_OK after checking the shape arguments and
 *    read no pointer.  Reductions over the batch (flow backward, the
 *    log-weights loss, batch-norm batch statistics) reject it with EINVAL.
 *  - Results for sample b depend only on sample b's inputs (never on the batch
 *    size or the sample's position in the batch), except for reductions over
 *    the batch (g_params, loss), which use a fixed order.  All results are
 *    bitwise reproducible run to run.
 */
#ifndef LFS_H
#define LFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (negative = error). */
typedef enum lfs_status {
  LFS_OK = 0,
  LFS_EINVAL = -1,       /* invalid argument: shape, null pointer, range */
  LFS_EUNSUPPORTED = -2, /* valid but not supported (e.g. hidden not in {8,16,32}) */
  LFS_EWORKSPACE = -3,   /* workspace smaller than lfs_workspace_bytes() */
  LFS_EDEVICE = -4       /* HIP launch / device error */
} lfs_status;

/* Arithmetic form of the flow and of the per-sample sums.
 *   LFS_PLAIN_FP32: convolutions with FP32 operands and FP32 accumulation;
 *                   log-det and action sums accumulated in FP32.
 *   LFS_BF16_CONV:  convolution operands rounded to BF16 (matrix cores),
 *                   FP32 accumulation; log-det, action, log-weights and all
 *                   ratios accumulated in FP64. */
typedef enum lfs_precision { LFS_PLAIN_FP32 = 0, LFS_BF16_CONV = 1 } lfs_precision;

/* Kernel family used for the flow.  AUTO picks the fused LDS-resident kernels
 * when the shape has one, else the generic kernels (same results up to
 * floating-point summation order). */
typedef enum lfs_algo { LFS_ALGO_AUTO = 0, LFS_ALGO_GENERIC = 1, LFS_ALGO_FUSED = 2 } lfs_algo;

/* Flow architecture (paper Sec. 1, coupling-layer and composition equations;
 * the example parameter file: hidden_sizes [8, 8], kernel_size 3, inC 1, outC 2).
 *   dim        lattice dimension, 2 or 3
 *   L          lattice extent, even and >= 2 (the checkerboard needs even L)
 *   n_layers   number of coupling layers N >= 1; layer l freezes the sites of
 *              parity (l + parity0) mod 2 and updates the others
 *   hidden     channels C of the two hidden convolutions of the default
 *              network: 8, 16 or 32 (ignored when n_hidden > 0)
 *   final_tanh 1: s = tanh(o_0); 0: s = o_0
 *   parity0    0 or 1
 *   precision  lfs_precision
 *   algo       lfs_algo
 * General networks (the parameter file's hidden_sizes and kernel_size):
 *   kernel     odd kernel size K per axis, 1..7; 0 means 3
 *   n_hidden   number of hidden convolutions, 1..LFS_MAX_HIDDEN; 0 means two
 *              of `hidden` channels
 *   hidden_sizes  their channel counts, 1..64 each (first n_hidden entries)
 *   batch_norm 0 or 1 (the parameter file's use_bn): 1 normalises every hidden
 *              convolution's output per channel before its LeakyReLU,
 *              y = gamma (a - mean) / sqrt(var + 1e-5) + beta, with batch or
 *              running statistics (lfs_flow_forward_bn); such a flow runs only
 *              through the _bn entry points
 * A network equal to the default (kernel 3, two hidden convolutions of 8, 16
 * or 32 channels, no batch norm) runs on the fused or generic kernels; any
 * other runs on the general-network kernels (LFS_ALGO_FUSED then reports
 * EUNSUPPORTED). */
#define LFS_MAX_HIDDEN 4
typedef struct lfs_flow_desc {
  int32_t dim;
  int32_t L;
  int32_t n_layers;
  int32_t hidden;
  int32_t final_tanh;
  int32_t parity0;
  int32_t precision;
  int32_t algo;
  int32_t kernel;
  int32_t n_hidden;
  int32_t hidden_sizes[LFS_MAX_HIDDEN];
  int32_t batch_norm;
} lfs_flow_desc;

/* Statistics a batch-norm flow normalises with. */
typedef enum lfs_bn_mode { LFS_BN_BATCH = 0, LFS_BN_RUNNING = 1 } lfs_bn_mode;

/* Persistent state of one independence Metropolis-Hastings chain (device POD,
 * caller-owned; zero-initialise a new chain).
 *   w_cur      log-weight of the current configuration
 *   idx_cur    global proposal number of the current configuration
 *   n_acc      accepted proposals (the seeding proposal is not counted)
 *   n_seen     proposals seen so far (the global number of the next one)
 *   has_state  0 until the first proposal has seeded the chain */
typedef struct lfs_chain_state {
  double w_cur;
  int64_t idx_cur;
  int64_t n_acc;
  int64_t n_seen;
  int32_t has_state;
  int32_t reserved;
} lfs_chain_state;

/* Human-readable name of a status code (static string). */
const char* lfs_status_string(int32_t status);

/* Library version string (static). */
const char* lfs_version(void);

/* Number of FP32 parameters of the packed flow parameter vector.
 * Layout, per layer l = 0..N-1 in order, with C = hidden and T = 3^dim taps:
 *   W1[C][1][T]  b1[C]  W2[C][C][T]  b2[C]  W3[2][C][T]  b3[2]
 * Taps are row-major over delta in {-1,0,1}^dim, axis 0 slowest; channel 0 of
 * the last convolution is s, channel 1 is t.  A general network stores, per
 * layer, W_i[cout_i][cin_i][T] then b_i[cout_i] for each convolution in order
 * (cin = 1, w_1, .., w_n; cout = w_1, .., w_n, 2), T = K^dim, taps row-major
 * over {-K/2..K/2}^dim; with batch norm a hidden convolution's b_i is followed
 * by gamma_i[cout_i] then beta_i[cout_i].  Returns 0 for an invalid desc. */
size_t lfs_param_count(const lfs_flow_desc* desc);

/* Number of FP32 entries of a batch-norm flow's statistics vector: per layer,
 * per hidden convolution i in order, mean[w_i] then var[w_i].  Returns 0
 * without batch norm or for an invalid desc.  Before training the running
 * statistics are mean 0, var 1. */
size_t lfs_bn_stats_count(const lfs_flow_desc* desc);

/* Workspace bytes needed by lfs_flow_forward (for_backward = 0) or
 * lfs_flow_backward (for_backward = 1) at batch size B.  Writes *bytes (0 for
 * B == 0).  The size depends on the current device's compute-unit count.
 * Errors: EINVAL (desc, B < 0, bytes NULL), EUNSUPPORTED (ALGO_FUSED on a shape
 * without fused kernels). */
int32_t lfs_workspace_bytes(const lfs_flow_desc* desc, int32_t B, int32_t for_backward,
                            size_t* bytes);

/* Prior draw (paper Sec. 1, the point-wise independent trivial distribution;
 * example parameter file: Normal{Float32}(0, 1)).
 * Writes z[B][V] (FP32, V = sites per sample, a multiple of 4) with standard
 * normals and, if logr is not NULL, logr[B] = -1/2 sum z^2 - (V/2) ln(2 pi)
 * (FP64 sum of the FP32 values).  Random numbers: Philox4x32-10 (Salmon et
 * al., SC'11) under key (lo32(key), hi32(key)); sample b, sites 4j..4j+3 use
 * counter (j, lo32(counter0+b), hi32(counter0+b), 0); each output word x maps
 * to u = (floor(x/2^9) + 1/2) 2^-23; words (u0,u1) and (u2,u3) give two
 * Box-Muller pairs r cos(2 pi u_b), r sin(2 pi u_b), r = sqrt(-2 ln u_a).
 * Errors: EINVAL if B < 0, V <= 0, V % 4 != 0, z == NULL or z not 16-byte
 * aligned. */
int32_t lfs_prior_normal(uint64_t key, uint64_t counter0, int32_t B, int32_t V, float* z,
                         double* logr, void* stream);

/* Prior draw with one random stream per sample, for batches that mix samples of
 * different requests (same definition as lfs_prior_normal; sample b uses key
 * keys[b] and counter counters[b], so lfs_prior_normal(key, c0, ...) equals
 * keys[b] = key, counters[b] = c0 + b).
 *   keys, counters  [B] uint64, device memory
 *   z               [B][V] FP32 output, 16-byte aligned;  logr [B] FP64 or NULL
 * Errors: EINVAL (B < 0, V <= 0, V % 4 != 0, nulls, misaligned z). */
int32_t lfs_prior_normal_streams(int32_t B, int32_t V, const uint64_t* keys,
                                 const uint64_t* counters, float* z, double* logr, void* stream);

/* Flow forward in the sampling direction, phi = F^{-1}(z) (paper Sec. 1,
 * untrivializing map and coupling-layer equation).  For every layer the
 * frozen sublattice is fed (active sites zeroed) through
 * conv(1->C)+LeakyReLU(0.01), conv(C->C)+LeakyReLU(0.01), conv(C->2), all 3^dim
 * periodic cross-correlations with bias; s = tanh(o_0) (or o_0), t = o_1; the
 * active sites become x exp(s) + t and the log-determinant grows by the sum
 * of s over them.
 *   params    [lfs_param_count] FP32, packed as documented above
 *   z         [B][V] FP32 prior sample (read only)
 *   phi       [B][V] FP32 output (may alias z)
 *   logq      [B] FP64 output: log r(z) - log|det dF^{-1}/dz|
 *   logdet    [B] FP64 output or NULL: log|det dF^{-1}/dz|
 *   saved_x   [(N+1)][B][V] FP32 output or NULL: the field entering each
 *             layer, then phi; required later by lfs_flow_backward
 *   ws        workspace of at least lfs_workspace_bytes(desc, B, 0) bytes
 * Errors: EINVAL (desc, B < 0, nulls, a desc with batch norm), EUNSUPPORTED
 * (hidden), EWORKSPACE. */
int32_t lfs_flow_forward(const lfs_flow_desc* desc, const float* params, int32_t B,
                         const float* z, float* phi, double* logq, double* logdet,
                         float* saved_x, void* ws, size_t ws_bytes, void* stream);

/* lfs_flow_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels and results, bit for bit, with the workspace taken from a
 * static device array of LFS_NOALLOC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends (its address is looked up once
 * per device, on the first call with that device current).  The call allocates
 * and frees nothing.  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (different streams, or host threads) race and must
 * be serialised by the caller.  Nothing in the array needs to start at zero.
 * Arguments as lfs_flow_forward, without ws and ws_bytes.
 * Errors: as lfs_flow_forward; LFS_EWORKSPACE when the workspace this flow and
 * batch need (lfs_workspace_bytes(desc, B, 0)) exceeds LFS_NOALLOC_SCRATCH_BYTES
 * (the fused forwards need only their weight fragments, at most 85 KB per
 * layer, at any batch; the generic kernels' hidden activations grow with B). */
#define LFS_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
int32_t lfs_flow_forward_noalloc(const lfs_flow_desc* desc, const float* params, int32_t B,
                                 const float* z, float* phi, double* logq, double* logdet,
                                 float* saved_x, void* stream);

/* Vector-Jacobian product of lfs_flow_forward's outputs (phi, log q) with
 * respect to its inputs (params, z): the hand-written backward of the
 * coupling stack.  Layers are processed in reverse; each layer recomputes its
 * hidden activations from its saved input field (only the N+1 boundary
 * fields are kept).  For the shifted reverse-KL loss of the paper, mean over
 * the batch of log q + S, pass g_phi = dS/dphi / B and g_logq = 1/B.
 *   saved_x   [(N+1)][B][V] FP32, as written by lfs_flow_forward
 *   g_phi     [B][V] FP32 cotangent of phi
 *   g_logq    cotangent of log q, the same for every sample
 *   g_params  [lfs_param_count] FP32 output (overwritten, sum over the batch
 *             in a fixed order)
 *   g_z       [B][V] FP32 output or NULL (includes d log r / dz = -z)
 *   ws        workspace of at least lfs_workspace_bytes(desc, B, 1) bytes
 * Errors: as lfs_flow_forward, and EINVAL for B == 0 (a batch reduction). */
int32_t lfs_flow_backward(const lfs_flow_desc* desc, const float* params, int32_t B,
                          const float* saved_x, const float* g_phi, double g_logq,
                          float* g_params, float* g_z, void* ws, size_t ws_bytes, void* stream);

/* lfs_flow_backward with a cotangent of log q per sample (what an autograd
 * engine hands over for a [B] output):
 *   g_logq    [B] FP64 device, required
 * g_z then includes -g_logq[b] z[b].  Everything else as lfs_flow_backward;
 * equal entries give the same bits as lfs_flow_backward with that scalar.
 * Errors: as lfs_flow_backward; EINVAL also for g_logq NULL. */
int32_t lfs_flow_backward_vec(const lfs_flow_desc* desc, const float* params, int32_t B,
                              const float* saved_x, const float* g_phi, const double* g_logq,
                              float* g_params, float* g_z, void* ws, size_t ws_bytes, void* stream);

/* Training pair that keeps each layer's second hidden activation instead of
 * recomputing it in the backward (the coupling networks of paper Sec. 1: the
 * backward needs h2 = LeakyReLU(W2 * h1 + b2) at every site of every layer).
 * Saving costs device memory and write bandwidth in the forward; recomputing
 * costs the second hidden convolution again in the backward.
 *
 * lfs_saved_h_bytes: bytes of the saved activations at batch size B, written
 * to *bytes, for the shapes whose fused backward reads them: 2D L = 32,
 * hidden 16, plain FP32: h2 and s, N B (C V + V / 2) x 4; 3D L = 16, hidden 16 or 32, BF16
 * convolutions (plane-streaming kernels): h1 and h2 in BF16, a LeakyReLU
 * sign word of each and s per site, N B V (4 C + 12).  0 for every other flow
 * (its backward recomputes; saved_h below is then ignored and may be NULL).
 * With s saved the backward runs the affine backward instead of recomputing
 * the third convolution.
 * Errors: EINVAL (desc, B < 0, bytes NULL). */
int32_t lfs_saved_h_bytes(const lfs_flow_desc* desc, int32_t B, size_t* bytes);

/* lfs_flow_forward that also writes saved_h (device, lfs_saved_h_bytes bytes,
 * a layout private to the library, read only by lfs_flow_backward_saved with
 * the same desc, params and B).  saved_x is required.  Every output is
 * bitwise what lfs_flow_forward writes.
 * Errors: as lfs_flow_forward; EINVAL also for saved_x NULL (B > 0), or
 * saved_h NULL where lfs_saved_h_bytes is not 0. */
int32_t lfs_flow_forward_train(const lfs_flow_desc* desc, const float* params, int32_t B,
                               const float* z, float* phi, double* logq, double* logdet,
                               float* saved_x, float* saved_h, void* ws, size_t ws_bytes,
                               void* stream);

/* lfs_flow_backward reading the activations lfs_flow_forward_train saved
 * instead of recomputing them.  g_logq_vec: [B] FP64 device cotangents of
 * log q, or NULL to use g_logq for every sample.  The results equal those of
 * lfs_flow_backward / lfs_flow_backward_vec up to the rounding of the second
 * hidden convolution (the forward's and the backward's tilings may sum in a
 * different order).  Workspace: lfs_workspace_bytes(desc, B, 1).
 * Errors: as lfs_flow_backward; EINVAL also for saved_h NULL where
 * lfs_saved_h_bytes is not 0. */
int32_t lfs_flow_backward_saved(const lfs_flow_desc* desc, const float* params, int32_t B,
                                const float* saved_x, const float* saved_h, const float* g_phi,
                                double g_logq, const double* g_logq_vec, float* g_params,
                                float* g_z, void* ws, size_t ws_bytes, void* stream);

/* lfs_flow_forward for flows with batch norm (the example parameter file's
 * use_bn, otherwise undefined by the paper).  Each hidden convolution's output
 * a is normalised per channel, over the batch and all sites, before its
 * LeakyReLU.  The network reads only the frozen sites, so the statistics do
 * too and the log-determinant is still the sum of s over the active sites.
 *   bn_mode   LFS_BN_BATCH (training): mean and biased variance of this batch
 *             (FP64 sums in a fixed order); the samples of a batch are coupled
 *             through them.  If bn_stats is not NULL it holds running
 *             statistics, updated in place after each layer's network as
 *             r = (1 - momentum) r + momentum s with the unbiased variance
 *             n/(n-1) var, n = B V.
 *             LFS_BN_RUNNING (sampling): normalise with bn_stats (read only);
 *             samples are independent.
 *   bn_stats  [lfs_bn_stats_count] FP32 device, or NULL in batch mode
 *   momentum  in [0, 1] (0.1 is customary); ignored in running mode
 * Other arguments as lfs_flow_forward.  A desc without batch norm ignores the
 * bn arguments and computes what lfs_flow_forward does.
 * Errors: as lfs_flow_forward; EINVAL also for a bn_mode other than the two,
 * running mode with bn_stats NULL, momentum outside [0, 1], or B == 0 in batch
 * mode (B == 0 in running mode is a no-op). */
int32_t lfs_flow_forward_bn(const lfs_flow_desc* desc, const float* params, int32_t B,
                            const float* z, float* phi, double* logq, double* logdet,
                            float* saved_x, int32_t bn_mode, float* bn_stats, double momentum,
                            void* ws, size_t ws_bytes, void* stream);

/* lfs_flow_backward for flows with batch norm.  In batch mode the statistics
 * are recomputed from saved_x and differentiated as functions of the whole
 * batch (g_a = gamma r (g_y - mean(g_y) - xhat mean(g_y xhat)) per channel,
 * r = 1/sqrt(var + 1e-5), xhat = (a - mean) r); bn_stats is not read and may
 * be NULL.  In running mode bn_stats (required) holds the statistics the
 * forward used and g_a = gamma r g_y.  The gamma and beta gradients are the
 * sums of g_y xhat and g_y.
 *   g_logq_vec  [B] FP64 device cotangents of log q, or NULL to use g_logq for
 *               every sample (as lfs_flow_backward_vec / lfs_flow_backward)
 * Other arguments and errors as lfs_flow_backward and lfs_flow_forward_bn. */
int32_t lfs_flow_backward_bn(const lfs_flow_desc* desc, const float* params, int32_t B,
                             const float* saved_x, const float* g_phi, double g_logq,
                             const double* g_logq_vec, int32_t bn_mode, const float* bn_stats,
                             float* g_params, float* g_z, void* ws, size_t ws_bytes, void* stream);

/* Lattice action (paper Sec. 1, action, Laplacian and potential equations):
 *   S = sum_n [ -phi(n) sum_mu (phi(n+mu) + phi(n-mu) - 2 phi(n))
 *               + m^2 phi(n)^2 + lambda phi(n)^4 ]
 * and, if force != NULL, force = force_scale * dS/dphi with
 *   dS/dphi(n) = -2 Lap phi(n) + 2 m^2 phi(n) + 4 lambda phi(n)^3.
 *   phi        [B][V] FP32
 *   m2, lam    FP64, [B] if per_sample else [1]
 *   precision  LFS_BF16_CONV: per-site terms and the sum in FP64;
 *              LFS_PLAIN_FP32: in FP32 (stored widened)
 *   S          [B] FP64 output
 *   force      [B][V] FP32 output or NULL
 * Errors: EINVAL (dim not 2/3, L < 2, B < 0, nulls). */
int32_t lfs_action(int32_t dim, int32_t L, int32_t B, const float* phi, const double* m2,
                   const double* lam, int32_t per_sample, int32_t precision, double* S,
                   float* force, double force_scale, void* stream);

/* Log-weights and loss (paper Sec. 1: target exp(-S)/Z, model density q, and
 * the shifted reverse Kullback-Leibler divergence):
 *   logw[b] = -S[b] - logq[b]   (FP64)
 *   loss    = (1/B) sum_b (logq[b] + S[b])   (FP64 scalar, fixed order), if
 *             loss != NULL.
 * Errors: EINVAL (B <= 0, nulls). */
int32_t lfs_log_weights(int32_t B, const double* S, const double* logq, double* logw,
                        double* loss, void* stream);

/* Independence Metropolis-Hastings chains (paper Sec. 1, the
 * Metropolis-Hastings test that corrects flow proposals to exp(-S)/Z).
 * Chain c reads proposals k = 0..n_prop-1 at logw[c*n_prop + k] and
 * log_u[c*n_prop + k].  The first proposal a chain ever sees seeds it
 * (accepted = 1, not counted).  Otherwise the proposal is accepted iff
 * log_u < logw - w_cur, evaluated as one FP64 subtraction and one compare.
 *   state     [n_chains] lfs_chain_state, read and updated
 *   cur_idx   [n_chains][n_prop] int64 output: global proposal number of the
 *             chain's configuration after each proposal
 *   accepted  [n_chains][n_prop] uint8 output, or NULL
 * n_chains == 0 or n_prop == 0 is a no-op.
 * Errors: EINVAL (n_chains < 0, n_prop < 0, nulls). */
int32_t lfs_mh_chain(int32_t n_chains, int32_t n_prop, const double* logw, const double* log_u,
                     lfs_chain_state* state, int64_t* cur_idx, uint8_t* accepted, void* stream);

/* Independence Metropolis-Hastings over ragged chunks: chain c takes the
 * proposals [offsets[c], offsets[c+1]) of the flat logw / log_u arrays, in order,
 * with its state in states[state_index[c]]; same decision rule and outputs as
 * lfs_mh_chain (cur_idx and accepted are written at the proposals' positions).
 * Used by the server, where one batch holds chunks of several requests.
 *   offsets      [n_chains + 1] int64, non-decreasing, offsets[0] >= 0
 *   state_index  [n_chains] int32, distinct
 * Errors: EINVAL (n_chains < 0, nulls). */
int32_t lfs_mh_chain_ragged(int32_t n_chains, const int64_t* offsets, const double* logw,
                            const double* log_u, lfs_chain_state* states,
                            const int32_t* state_index, int64_t* cur_idx, uint8_t* accepted,
                            void* stream);

/* HMC trajectory per chain, the paper's comparison baseline (Sec. 2.2):
 * H = 1/2 sum pi^2 + S(phi); n_steps leapfrog steps of size dt in
 * kick-drift-kick form with the force above; dH = H_end - H_start; accept iff
 * log_u < -dH, else phi is restored.  All arithmetic in FP64.
 *   phi       [B][V] FP64, updated in place
 *   pi0       [B][V] FP64 momenta (read only)
 *   log_u     [B] FP64
 *   m2, lam   FP64, [B] if per_sample else [1]
 *   dH        [B] FP64 output;  accepted [B] uint8 output
 * Errors: EINVAL (shape, B < 0, n_steps < 0, nulls); EUNSUPPORTED if V > 4096. */
int32_t lfs_hmc_step(int32_t dim, int32_t L, int32_t B, double* phi, const double* pi0,
                     const double* log_u, const double* m2, const double* lam, int32_t per_sample,
                     int32_t n_steps, double dt, double* dH, uint8_t* accepted, void* stream);

/* Adam step t >= 1 (example parameter file: opt = Adam, base_lr = 1e-3), FP32:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
 * Errors: EINVAL (n <= 0, t < 1, nulls). */
int32_t lfs_adam_step(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1,
                      float b2, float eps, int64_t t, void* stream);

/* ---- chain-quality analysis ----------------------------------------------
 * Sec. 1: the statistical error of a Monte Carlo average falls as
 * 1/sqrt(N_indep) with N_indep = N_conf / (2 tau_ac), tau_ac the autocorrelation
 * time; Sec. 2.2 and the conclusions name the condensate, zero-momentum
 * two-point functions, the autocorrelation time and the effective sample size
 * as the analysis quantities, without formulas.  The estimators below are the
 * standard ones, named in each comment.  All sums are FP64 in a fixed order
 * (bitwise reproducible). */

/* Per-configuration observables.  Time runs along the first lattice axis:
 * Phi_b(t) is the sum of phi[b] over the L^(d-1) sites whose first coordinate
 * is t (a contiguous block in the row-major field layout).
 *   M[b]    = (1/V) sum_n phi[b][n]                       (condensate)
 *   C[b][t] = (1/V) sum_{t0} Phi_b(t0) Phi_b((t0 + t) mod L),  t = 0 .. L-1
 *             (zero-momentum two-point function of one configuration; ensemble
 *             means and the connected part are formed over configurations)
 *   phi  [B][V] FP32 (fp64 == 0) or FP64 (fp64 != 0), device
 *   M    [B] FP64 output or NULL;  C  [B][L] FP64 output or NULL (not both NULL)
 * B == 0 is a no-op.  Errors: EINVAL (dim not 2 or 3, L < 2, B < 0, phi NULL,
 * both outputs NULL); EUNSUPPORTED if L > 4096. */
int32_t lfs_observables(int32_t dim, int32_t L, int32_t B, const void* phi, int32_t fp64, double* M,
                        double* C, void* stream);

/* Bytes of device workspace lfs_autocorr needs (0 for invalid sizes). */
size_t lfs_autocorr_workspace_bytes(int32_t n_series, int64_t n, int32_t w_max);

/* Integrated autocorrelation time of n_series series of length n (the windowed
 * estimator with the automatic window of Madras and Sokal):
 *   xbar = (1/n) sum_k x_k,  Gamma(t) = (1/(n-t)) sum_{k<n-t} (x_k - xbar)(x_{k+t} - xbar)
 *   tau(W) = 1/2 + sum_{t=1..W} Gamma(t)/Gamma(0); the window W is the smallest
 *   W >= 1 with W >= c tau(W), searched up to T = min(w_max, n-1); if none,
 *   W = T and found = 0.  tau_ac = tau(W), N_indep = n / (2 tau_ac).
 * Element k of series s is x[s*ldx + k], or x[s*ldx + index[s*n + k]] when
 * index is given (e.g. an MH chain's current-configuration numbers, so that
 * repeated configurations are read in place).
 *   x        FP64 device, series s at x + s*ldx (ldx >= n without index)
 *   index    [n_series][n] int64 device, or NULL; an entry outside [0, ldx)
 *            makes that series' gamma, tau and n_indep NaN and its window -1
 *   gamma    [n_series][w_max+1] FP64 output or NULL (lags beyond T: NaN)
 *   tau      [n_series] FP64 output (NaN when Gamma(0) == 0: constant series, n == 1)
 *   window   [n_series] int32 output or NULL (0 when Gamma(0) == 0)
 *   found    [n_series] uint8 output or NULL;  n_indep [n_series] FP64 output or NULL
 *   ws       lfs_autocorr_workspace_bytes(n_series, n, w_max) bytes of device memory
 * Errors: EINVAL (n_series < 1, n < 1, w_max < 0, c <= 0, ldx too small, x,
 * tau or ws NULL); EWORKSPACE; EUNSUPPORTED if w_max > 8192 or n_series > 65535. */
int32_t lfs_autocorr(int32_t n_series, int64_t n, const double* x, int64_t ldx, const int64_t* index,
                     int32_t w_max, double c, double* gamma, double* tau, int32_t* window,
                     uint8_t* found, double* n_indep, void* ws, size_t ws_bytes, void* stream);

/* Normalised reweighting effective sample size of n_series sets of n
 * log-weights w = log p - log q (up to a constant, e.g. lfs_log_weights):
 *   ESS = (sum_k e^{w_k})^2 / (n sum_k e^{2 w_k})  in [1/n, 1],
 * evaluated with w_k - max_k w_k.  Entries must be finite or -inf; all -inf
 * gives NaN.
 *   logw  FP64 device, set s at logw + s*ldw;  ess  [n_series] FP64 output
 * Errors: EINVAL (n_series < 1, n < 1, ldw < n, NULLs). */
int32_t lfs_ess(int32_t n_series, int64_t n, const double* logw, int64_t ldw, double* ess, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LFS_H */
