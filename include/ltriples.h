/*
 * ltriples — perturbative-triples energy E(T) of one local-natural-orbital
 * (LNO) domain over high-spin restricted-open-shell, semicanonical orbitals
 * with spin-unrestricted amplitudes, on AMD Instinct MI355X (gfx950).
 *
 * What is computed (Szabo, Csoka, Kallay, Nagy, arXiv:2311.10048,
 * Sec. "Open-Shell LNO-CCSD(T) Ansatz", eq. cim_pt_energy summed over the
 * central index, and Sec. "Correlation energy calculation in the LIS" for
 * the inputs): with D = e_i + e_j + e_k - e_a - e_b - e_c,
 *
 *   W^{abc}_{ijk} = P(i/jk)P(a/bc)[ sum_e t^{ae}_{jk}<ei||bc> - sum_m t^{bc}_{im}<ma||jk> ]
 *   V^{abc}_{ijk} = P(i/jk)P(a/bc)[ t^a_i <jk||bc> + f_ia t^{bc}_{jk} ]
 *   E(T) = 1/36 sum_{ijkabc} W (W + V) / D = E4 + E_ST + E_DT,
 *
 * summed over the four spin blocks aaa, aab, abb, bbb.  Two-electron
 * integrals are density fitted in a natural-auxiliary-function basis shared
 * by both spins (Sec. "Natural auxiliary functions"):
 * (pq|rs) = sum_Q B^Q_pq B^Q_rs, <pq||rs> = (pr|qs) - (ps|qr).
 *
 * Conventions
 *  - All input arrays are FP64, row-major, C-contiguous, in DEVICE memory,
 *    owned by the caller and only read.  Layouts:
 *      t1a [noa][nva]            t1b [nob][nvb]
 *      t2aa [noa][noa][nva][nva] antisymmetric in (i,j) and in (a,b)
 *      t2bb [nob][nob][nvb][nvb] antisymmetric in (I,J) and in (A,B)
 *      t2ab [noa][nob][nva][nvb] t^{aB}_{iJ} at [i][J][a][B], no symmetry
 *      Boo_x [naux][no_x][no_x], Bov_x [naux][no_x][nv_x],
 *      Bvv_x [naux][nv_x][nv_x]   (x = a, b; oo and vv symmetric in p,q)
 *      eo_x [no_x], ev_x [nv_x]   semicanonical orbital energies (Eh)
 *      fov_x [no_x][nv_x]         occupied-virtual Fock block
 *  - SOMOs are alpha occupied and beta virtual orbitals.
 *  - Outputs are FP64 in device memory.  Low-precision copies of the inputs
 *    live in the caller's workspace.  The energy epilogue (V, D, the
 *    division and all reductions) is always FP64.
 *  - A work item is one unique occupied triplet (block, p, q, r):
 *      block 0 aaa (i<j<k), 1 aab (i<j alpha, K beta),
 *      2 abb (I<J beta, k alpha), 3 bbb (I<J<K).
 *  - Results are deterministic.  Energies are bitwise identical across runs,
 *    batch sizes, tile configurations and orders of the item list for the
 *    same inputs, precision and item set (each block's items are processed
 *    in canonical order); adjoints are bitwise identical across runs for a
 *    fixed batching (other batchings agree to rounding).
 *
 * Errors: every entry point returns LT_OK (0) or a negative code, and
 * ltriples_last_error() (thread-local) describes it.  Argument, shape,
 * precision, workspace and orbital-energy errors are found before anything
 * is enqueued; a HIP, rocBLAS or rocSOLVER failure (LT_EHIP) may leave
 * earlier work of the call enqueued.
 */
#ifndef LTRIPLES_H
#define LTRIPLES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LT_OK 0
#define LT_EINVAL (-1)      /* null pointer or negative dimension */
#define LT_ESHAPE (-2)      /* inconsistent or too large dimensions, or a bad item list */
#define LT_EDENOM (-3)      /* max occupied e >= min virtual e (some D >= 0), occupied-
                               virtual gap below 1e-100, or an |e| above 1e100 */
#define LT_EPREC (-4)       /* unsupported precision */
#define LT_EWORKSPACE (-5)  /* workspace too small */
#define LT_EHIP (-6)        /* HIP runtime error */
#define LT_ENONFINITE (-7)  /* NaN/Inf in the orbital energies, or in any input
                               when options.check_finite is set */

/* Arithmetic of the W contractions.  LT_FP64: FP64 matrix cores.
 * LT_FP32: FP32 matrix cores, FP32 accumulation.  LT_BF16X3: each FP32
 * operand split as hi = bf16(x), lo = bf16(x - hi), products
 * hi*hi + hi*lo + lo*hi on BF16 matrix cores with FP32 accumulation.
 * LT_BF16: single BF16 product (ablation only). */
typedef enum {
  LT_FP64 = 0,
  LT_FP32 = 1,
  LT_BF16X3 = 2,
  LT_BF16 = 3
} ltriples_precision;

/* One LIS domain: sizes and device pointers in the layouts above.  A pointer
 * may be NULL only when its array has zero elements.  Size limits (LT_ESHAPE
 * beyond them): nva, nvb <= 46340; noa, nob <= 4096; naux <= 2^24; and all
 * FP64 input arrays together at most 2^37 elements (1 TiB), more than one
 * device can hold. */
typedef struct ltriples_domain {
  int32_t noa, nob, nva, nvb, naux;
  const double *t1a, *t1b;
  const double *t2aa, *t2bb, *t2ab;
  const double *Boo_a, *Bov_a, *Bvv_a;
  const double *Boo_b, *Bov_b, *Bvv_b;
  const double *eo_a, *ev_a, *eo_b, *ev_b;
  const double *fov_a, *fov_b;
} ltriples_domain;

/* Per-phase timings of one call (filled only when requested through
 * ltriples_options.stats).  Times are HIP-event times on the call's stream. */
typedef struct ltriples_stats {
  double total_ms;              /* first to last enqueued kernel */
  double setup_ms;              /* operand layouts and integral builds */
  double triples_gemm_ms;       /* sum over the triplet-contraction launches */
  double epilogue_ms;           /* sum over energy epilogues and per-item sums */
  int64_t triples_gemm_launches;
  double triples_gemm_flops;    /* 2*M*N*K of those launches (unpadded shapes) */
  double algorithmic_flops;     /* W-contraction flops of the item list, as
                                   counted by ltriples_flops() */
  int64_t n_items;
} ltriples_stats;

/* Options; a NULL options pointer means all defaults (zeros). */
typedef struct ltriples_options {
  /* bytes of workspace the per-batch triples intermediates (contraction
   * outputs and per-tile partial energies) may use; 0 = default, capped by
   * the work: 8 GiB for energies, 16 GiB for the spin-adapted closed-shell
   * energy, 32 GiB for adjoints.  Smaller budgets mean smaller item batches;
   * energies are bitwise unchanged (adjoints agree to rounding, as for any
   * other batching). */
  size_t workspace_budget;
  /* optional HOST array [n_items][4] of (block, p, q, r) restricting the
   * energy to these items (NULL = all unique triplets of the domain) */
  const int32_t* items;
  int32_t n_items;
  /* optional DEVICE array [n_items][3] receiving {E4, E_ST, E_DT} per item,
   * in the order of `items` (or of the full enumeration) */
  double* e_items;
  /* items per batch (0 = automatic) */
  int32_t batch_items;
  /* optional HOST pointer: when set, the call records HIP events around
   * each phase and launch, waits for the stream before returning, and
   * fills *stats */
  ltriples_stats* stats;
  /* ltriples_energy_batched only: 1 = capture the launch sequence into a
   * hipGraph on the first call and replay it on later calls with the same
   * shapes, pointers, workspace and options (requires a caller workspace) */
  int32_t graph;
  /* the largest operand builds (<ei||bc>, (jb|EC), (be|KC) and the same-spin
   * (ov|ov) behind <qr||yz>) run in chunks of their leading occupied index
   * of at most this many MiB each (0 = default 2048).  Smaller chunks shrink
   * the staging and scratch parts of the workspace; results are bitwise
   * unchanged. */
  int32_t build_chunk_mib;
  /* 1 = tile-shape autotuning of the triplet contraction kernels: the first
   * launch of each shape class in the process (per device: precision or
   * number of BF16 products, output layout, 32-row blocks of output rows,
   * log2 of the columns) times
   * every candidate tile configuration on its own data and keeps the
   * fastest for all later launches of the class, with or without this
   * flag.  Every configuration sums each output element in the same order,
   * so the choice changes no result bit.  Tuning waits for the stream; it
   * is skipped under graph capture (the default or an earlier choice is
   * used).  ltriples_autotune_reset() forgets the choices.  When the
   * environment variable LTRIPLES_TUNE_CACHE names a file, choices are read
   * from it (JSON, per GPU architecture) before any tuning and every new
   * choice is written back to it, so later processes, and graph captures,
   * start from tuned tiles. */
  int32_t autotune;
  /* Accepted for interface compatibility; every call is deterministic
   * whatever its value.  All reductions run in a fixed order with a fixed
   * decomposition: energies, parts and per-item values are bitwise
   * identical across runs, batch sizes, tile configurations (tuned or
   * forced), build chunk sizes and item-list orders; adjoints are bitwise
   * identical across runs for a fixed batching (a different batching
   * changes the order of the reverse-product sums, so they agree to
   * rounding only).  No atomics are used in any reduction. */
  int32_t deterministic;
  /* 1 = scan every input array for NaN and infinity on the device before
   * anything else is computed, and return LT_ENONFINITE if one is found
   * (the scan enqueues one fill and one reduction kernel and waits for the
   * stream once).  The orbital energies are always checked (see
   * ltriples_energy). */
  int32_t check_finite;
  /* Forced tile configuration of the triplet contraction kernels, per
   * output layout: [0] same-spin S, [1] mixed G, [2] mixed Y.  0 =
   * automatic (tuned choice, else the measured default); k = 1..8 forces
   * configuration k of the precision's table for every launch of that
   * layout (no tuning).  Tables (output rows x columns per work-group):
   *   BF16X3 and BF16: 32x128, 64x128, 96x128, 128x128, 192x128, 256x128,
   *                    320x128, 384x128 (4 waves; 1: 1x4 waves, 4..8: 2x2)
   *   FP32:  32x128, 64x128, 96x128, 128x128, 192x128, 256x128, 320x128,
   *          384x128
   *   FP64:  32x64, 64x64, 128x64, 192x64, 256x64, 320x64, 384x64, 512x64
   * Configurations only change the time: every one sums each output
   * element over the same segments and stages in the same order, so the
   * result is bitwise that of the automatic choice.  Values outside 0..8
   * give LT_EINVAL. */
  int32_t tile_override[3];
  /* ltriples_energy_batched only: 0 = the domains run one after another,
   * sharing one workspace region for their operands and intermediates.
   * > 0 = launch groups: the domains, in descending order of their triples
   * flops, are packed into groups of at most 16 consecutive domains whose
   * regions together take at most this many bytes (a domain that alone
   * exceeds it forms a group of its own).  The domains of a group are
   * prepared side by side; then, spin block by spin block and item batch by
   * item batch, each triples contraction launch takes one batch of every
   * domain of the group (BF16X3 and BF16; FP32 and FP64 launch per domain),
   * followed by each domain's epilogue.  Each domain's batches, epilogues
   * and reductions are those of a call on it alone, so every result bit is
   * unchanged; the workspace grows to the largest group's regions. */
  size_t group_budget;
} ltriples_options;

/* Host-only validation of sizes, pointers, precision and item list.  Makes
 * no HIP call and reads no device memory. */
int ltriples_validate(const ltriples_domain* d, int32_t precision,
                      const ltriples_options* o);

/* Host-only: workspace bytes ltriples_energy needs for this domain,
 * precision and options. */
int ltriples_workspace_size(const ltriples_domain* d, int32_t precision,
                            const ltriples_options* o, size_t* bytes);

/* Host-only: algorithmic W-contraction flop count of the item list (the
 * GEMMs of the spin-block working equations over the full virtual cube,
 * 2 flops per multiply-add); n_items_out receives the number of items. */
int ltriples_flops(const ltriples_domain* d, const ltriples_options* o,
                   double* flops, int64_t* n_items_out);

/* E(T) of one domain, enqueued on `stream` (a hipStream_t; NULL = default).
 *   e_out  device double[1]: E(T)
 *   parts  device double[4][3] or NULL: per block {E4, E_ST, E_DT}
 *   ws     device workspace of ws_bytes >= ltriples_workspace_size(), or
 *          NULL: the library then allocates it with hipMallocAsync on
 *          `stream` and releases it with hipFreeAsync on every return path
 *          (the allocation adds no wait for the stream).
 * Host waits: the call reads the orbital energies back to the host with
 * copies ordered on `stream` (after whatever the caller enqueued there) and
 * waits for the stream, to check that they are finite (LT_ENONFINITE), at
 * most 1e100 in magnitude, and that every virtual energy exceeds every
 * occupied one by at least 1e-100 (LT_EDENOM), so every denominator D lies
 * in [-6e100, -3e-100]; it then copies its item tables to the workspace and
 * waits for the stream once more before enqueuing any kernel (and once more
 * with options.check_finite).  The kernels themselves are asynchronous on
 * `stream`.
 * Fewer than 3 occupied orbitals in total, or empty virtual spaces, give
 * E = 0 and LT_OK. */
int ltriples_energy(const ltriples_domain* d, int32_t precision,
                    const ltriples_options* o, double* e_out, double* parts,
                    void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): E(T) of one
 * domain exactly as ltriples_energy computes it (same kernels, bitwise the
 * same result), with the whole workspace in a fixed device array that the
 * library holds on each GPU it runs on, from the first call there until the
 * process ends (ltriples_noalloc_capacity() bytes, 256 MiB).  The call makes
 * no hipMalloc, hipFree or other allocating call.  When the domain's plan
 * does not fit the array, it is refitted with smaller item batches and build
 * chunks (which change no result bit); a domain that does not fit even with
 * single-item batches gives LT_EWORKSPACE before anything is enqueued.
 * options.stats and options.autotune must be unset (LT_EINVAL); the other
 * options and every error code are as ltriples_energy, and so are the host
 * waits.  All calls on one GPU share its array, which keeps the last call's
 * contents (every word a call reads is written by that call first): calls
 * that overlap on one GPU (on different streams or from different threads)
 * race on it and must be serialised by the caller. */
int ltriples_energy_noalloc(const ltriples_domain* d, int32_t precision,
                            const ltriples_options* o, double* e_out,
                            double* parts, void* stream);

/* Bytes of the fixed per-device array of ltriples_energy_noalloc. */
size_t ltriples_noalloc_capacity(void);

/* The central localized molecular orbital of a domain and the Laplace
 * quadrature of its (T) share (Sec. "Correlation energy calculation in the
 * LIS", eqs. laplace_transform and local_pt).
 *   spin   0: the central orbital is an alpha orbital, 1: beta
 *   c      DEVICE double[no_spin]: the central orbital in the domain's
 *          occupied orbitals of that spin (normally of unit norm; any vector
 *          is accepted, the share is quadratic in it)
 *   nq     number of quadrature points, 1..64
 *   s, w   HOST double[nq]: points t_q > 0 and weights w_q with
 *          1/x ~ sum_q w_q exp(-t_q x) for the positive denominators x = -D
 *          (the paper uses 3-4 points chosen per system; any quadrature,
 *          e.g. a minimax exponential sum over the domain's range of -D) */
typedef struct ltriples_central {
  int32_t spin;
  const double* c;
  int32_t nq;
  const double* s;
  const double* w;
} ltriples_central;

/* Host-only: workspace bytes of ltriples_energy_central. */
int ltriples_central_workspace_size(const ltriples_domain* d, const ltriples_central* c,
                                    int32_t precision, const ltriples_options* o,
                                    size_t* bytes);

/* The (T) share of the central orbital c of eq. local_pt: one third of the
 * triples energy of the occupied triplets that hold c once (with the other
 * two indices j < k of its spin, j of its spin and K of the other, or
 * J < K of the other spin), over the unique virtual ranges, with 1/D
 * replaced by the Laplace sum -sum_q w_q exp(t_q D) and the central
 * orbital's half of each point's factor exp(t_q D) absorbed into it:
 *   dE_c = -(1/3) sum_q w_q sum W_c (W_c + V_c) exp(t_q D'),
 *   W_c = sum_i c_i exp(t_q e_i / 2) W_{i..}  (likewise V_c),
 * D' the denominator without the central orbital's energy.  For c = e_i and
 * a quadrature exact on the domain's denominators this is one third of the
 * energy of the items that contain orbital i; the shares of an orthonormal
 * basis of both spins' occupied orbitals add up to the energy with the
 * Laplace denominators.  The cost is about 3 n_q / o of the whole domain's.
 *   e_out  device double[1]; parts device double[4][3] or NULL: per block
 *          (aaa, aab, abb, bbb) {E4, E_ST, E_DT} (the blocks of the central
 *          spin's triplets only; the others are zero)
 *   ws     device workspace >= ltriples_central_workspace_size(), or NULL
 *          (stream-ordered allocation, as ltriples_energy)
 * Precisions, batching, chunking, tiles, stats and host waits as
 * ltriples_energy; options.items, options.e_items and options.graph must be
 * unset (LT_EINVAL).  LT_EINVAL also for a bad spin, nq, point (t_q <= 0 or
 * not finite) or weight, LT_ESHAPE when the central spin has no occupied
 * orbital.  Exponentials overflow (giving infinities) only when some
 * t_q |e| exceeds about 700. */
int ltriples_energy_central(const ltriples_domain* d, const ltriples_central* c,
                            int32_t precision, const ltriples_options* o, double* e_out,
                            double* parts, void* ws, size_t ws_bytes, void* stream);

/* Debug dump of one triplet's connected triples amplitude W (the quantity of
 * the master formula, eq. cim_pt_energy, before V and the denominator enter):
 * runs the forward path of ltriples_energy for the single item `item`
 * (HOST int32[4], (block, p, q, r) as options.items) in `precision`, and
 * writes W over the item's full virtual cube to `w` (DEVICE FP64,
 * row-major): [a][b][c] with v_s^3 entries for a same-spin block, [a][b][C]
 * with v_s * v_s * v_t entries for a mixed one (a, b of the pair's spin s,
 * C of the odd index's spin t).  W is formed from the contraction outputs
 * exactly as the energy epilogues read them (the unique virtual range), and
 * extended by its antisymmetry in the virtual indices of equal spin (zero
 * where two of them coincide).  The item's energy goes to `e_out` (DEVICE,
 * one double).  ws / ws_bytes: as ltriples_energy with options.items = item
 * (size from ltriples_workspace_size with those options), or NULL.  Errors
 * as ltriples_energy; LT_EINVAL for a NULL item or w. */
int ltriples_debug_w(const ltriples_domain* d, int32_t precision, const int32_t* item,
                     double* w, double* e_out, void* ws, size_t ws_bytes, void* stream);

/* Gradient outputs of ltriples_backward: caller-owned device FP64 buffers in
 * the layouts of the corresponding ltriples_domain inputs.  A NULL field is
 * not written.  Gradients of inputs that carry a symmetry are returned
 * projected onto it: dE/dt2aa and dE/dt2bb antisymmetrised in (i,j) and in
 * (a,b), dE/dBoo and dE/dBvv symmetrised in their two orbital indices (a
 * finite difference moving all images of one element together sees 4x
 * resp. 2x the returned off-diagonal element). */
typedef struct {
  double *t1a, *t1b, *t2aa, *t2bb, *t2ab;
  double *Boo_a, *Bov_a, *Bvv_a, *Boo_b, *Bov_b, *Bvv_b;
  double *fov_a, *fov_b;               /* dE/df_ia (f_ov enters V linearly) */
  double *eo_a, *ev_a, *eo_b, *ev_b;   /* dE/de: D of eq. cim_pt_energy is the
                                          sum of the three occupied minus the
                                          three virtual orbital energies */
} ltriples_domain_grad;

/* Host-only: workspace bytes of ltriples_backward. */
int ltriples_backward_workspace_size(const ltriples_domain* d, int32_t precision,
                                     const ltriples_options* o, size_t* bytes);

/* Adjoint of ltriples_energy: gbar * dE/dx for x in T1, T2, the DF factors,
 * f_ov and the semicanonical orbital energies.  E is the energy
 * of eq. cim_pt_energy as read by ltriples_energy (all occupied triplets, or
 * the item subset of options.items).  The connected W is recomputed per item
 * batch, never stored; the work is about three times the forward flops.
 * The orbital-energy gradient costs one more reduction per epilogue tile and
 * is computed only when one of its four output pointers is set.
 *   gbar   device pointer to one double (the incoming adjoint dL/dE)
 *   grad   host struct of device output pointers (see ltriples_domain_grad)
 *   ws     device workspace >= ltriples_backward_workspace_size(), or NULL
 *          (stream-ordered allocation, as ltriples_energy)
 * Precision LT_FP64 or LT_FP32 (the contractions and operand gradients in
 * that precision, the epilogue, the integral gradients and the DF
 * back-contraction in FP64), or LT_BF16X3 (the forward contraction
 * recomputed from split BF16 products as in ltriples_energy, everything
 * else as LT_FP32; the workspace keeps both the FP32 operands and their
 * split copies); LT_BF16 gives LT_EPREC.  options.e_items
 * must be NULL.  Enqueued on `stream`; the call synchronises the stream once
 * after uploading its work descriptors.  Errors as ltriples_energy. */
int ltriples_backward(const ltriples_domain* d, int32_t precision,
                      const ltriples_options* o, const double* gbar,
                      const ltriples_domain_grad* grad, void* ws,
                      size_t ws_bytes, void* stream);

/* Host-only self-check of the launch plan (no HIP calls).  With
 * backward != 0 it builds the adjoint pass's reverse-contraction descriptors
 * against a placeholder workspace base and verifies that every memory range
 * they address lies inside its planned buffer, that operands are 16-byte
 * aligned with row strides that are multiples of 4 elements, and that the
 * output blocks of one launch do not overlap (element by element for plans
 * below 256 MiB).  LT_OK, or an error code with a message. */
int ltriples_plan_check(const ltriples_domain* d, int32_t precision,
                        const ltriples_options* o, int32_t backward);

/* Host-only: workspace bytes of ltriples_energy_batched for ndom domains. */
int ltriples_workspace_size_batched(const ltriples_domain* ds, int32_t ndom,
                                    int32_t precision, const ltriples_options* o,
                                    size_t* bytes);

/* E(T) of ndom independent domains in one call (Sec. "Open-Shell LNO-CCSD(T)
 * Ansatz": the LNO energy is a sum of independent per-orbital domain
 * contributions, eq. lno_ccsdpt_energy), enqueued on `stream`.
 *   ds      HOST array [ndom] of domains (device pointers as above)
 *   e_out   device double[ndom]; parts device double[ndom][4][3] or NULL
 *   ws      device workspace >= ltriples_workspace_size_batched(), or NULL
 *           (stream-ordered allocation, as ltriples_energy; no graph then)
 * Each domain's result is bitwise identical to ltriples_energy on that
 * domain alone, with or without launch groups (options.group_budget, which
 * ltriples_workspace_size_batched must be given too).  Item lists, per-item
 * outputs and stats are not available
 * here (LT_EINVAL).  With options.graph = 1 (and a caller workspace) the
 * launch sequence is captured into a hipGraph on the first call and replayed
 * on later calls whose shapes, pointers and options match; the graph reads
 * the inputs at replay time.  The orbital energies of every domain are read
 * back once per call (copies ordered on `stream`, then a wait for it) to
 * check the denominators. */
int ltriples_energy_batched(const ltriples_domain* ds, int32_t ndom,
                            int32_t precision, const ltriples_options* o,
                            double* e_out, double* parts, void* ws,
                            size_t ws_bytes, void* stream);

/* Drops every cached hipGraph of ltriples_energy_batched. */
int ltriples_graph_reset(void);

/* Forgets every tile configuration chosen by options.autotune. */
int ltriples_autotune_reset(void);

/* One closed-shell (SOMO-free) domain in spatial orbitals, for the domains
 * whose orbital sets become spin independent once the domain Fock matrix is
 * spin averaged (section "Approximate long-range spin polarization").
 *   t1 [no][nv], tau [no][no][nv][nv] with tau^{ab}_{ij} = tau^{ba}_{ji}
 *   (not checked), Boo [naux][no][no], Bov [naux][no][nv], Bvv
 *   [naux][nv][nv], eo [no], ev [nv], fov [no][nv]; FP64, device pointers. */
typedef struct ltriples_rhf_domain {
  int32_t no, nv, naux;
  const double *t1, *tau;
  const double *Boo, *Bov, *Bvv;
  const double *eo, *ev, *fov;
} ltriples_rhf_domain;

/* Host-only: workspace bytes of ltriples_energy_rhf. */
int ltriples_rhf_workspace_size(const ltriples_rhf_domain* d, int32_t precision,
                                const ltriples_options* o, size_t* bytes);

/* Host-only: W-contraction flops ltriples_energy_rhf executes,
 * 12 nv^3 (nv + no) per unordered occupied triple, and its number of items
 * (the unordered triples i <= j <= k that are not all equal). */
int ltriples_rhf_flops(const ltriples_rhf_domain* d, double* flops, int64_t* n_items_out);

/* Closed-shell E(T) of one domain (the closed-shell limit of the method,
 * section "Summary and conclusions"; the SOMO-free domains of the long-range
 * spin-polarization approximation), in the spin-adapted form over spatial
 * orbitals: W^{abc}_{ijk} as the sum over the six joint permutations of the
 * pairs (ia), (jb), (kc) of one connected term, and
 * E = 1/3 sum_{ijk} sum_{abc} (4W^{abc} + W^{bca} + W^{cab})(V^{abc} - V^{cba}) / D
 * with V = W + the t1 and f_ov disconnected terms.  Each unordered occupied
 * triple i <= j <= k costs three contractions of nv x nv^2 outputs over
 * 2 (nv + no) rows; the energy of all its orderings is summed over unique
 * virtual tiles.  parts = {E4, E_ST, E_DT} from the W, t1 and f_ov parts of V.
 *   e_out  device double[1]; parts device double[3] or NULL
 *   ws     device workspace >= ltriples_rhf_workspace_size(), or NULL
 * Precisions, batching (options.batch_items, workspace_budget; here the
 * default budget is 16 GiB), build chunks, check_finite, autotune and stats
 * as ltriples_energy; tile_override[0]
 * forces the contraction's tile (the other entries are not used);
 * options.items, options.e_items and options.graph must be unset (LT_EINVAL).
 * Errors as ltriples_energy. */
int ltriples_energy_rhf(const ltriples_rhf_domain* d, int32_t precision,
                        const ltriples_options* o, double* e_out, double* parts,
                        void* ws, size_t ws_bytes, void* stream);

/* Host-only: workspace bytes of ltriples_energy_rhf_spin_block. */
int ltriples_rhf_spin_block_workspace_size(const ltriples_rhf_domain* d, int32_t precision,
                                           const ltriples_options* o, size_t* bytes);

/* The same closed-shell E(T) through the spin-block path with identical
 * alpha and beta data, E = 2 E_aaa + 2 E_aab (the bbb and abb blocks equal
 * the aaa and aab ones and are not computed; about 2x the contraction work
 * of ltriples_energy_rhf).  The same-spin amplitudes
 * tau^{ab}_{ij} - tau^{ba}_{ij} are formed in the workspace.  Arguments,
 * options and errors as ltriples_energy_rhf (ws sized by
 * ltriples_rhf_spin_block_workspace_size); the adjoint
 * ltriples_backward_rhf differentiates this form. */
int ltriples_energy_rhf_spin_block(const ltriples_rhf_domain* d, int32_t precision,
                                   const ltriples_options* o, double* e_out, double* parts,
                                   void* ws, size_t ws_bytes, void* stream);

/* Gradient outputs of ltriples_backward_rhf: caller-owned device FP64
 * buffers in the layouts of the ltriples_rhf_domain inputs; a NULL field is
 * not written.  dE/dtau is projected onto tau^{ab}_{ij} = tau^{ba}_{ji};
 * dE/dBoo and dE/dBvv are symmetrised in their orbital indices. */
typedef struct ltriples_rhf_grad {
  double *t1, *tau, *Boo, *Bov, *Bvv, *eo, *ev, *fov;
} ltriples_rhf_grad;

/* Host-only: workspace bytes of ltriples_backward_rhf. */
int ltriples_backward_rhf_workspace_size(const ltriples_rhf_domain* d, int32_t precision,
                                         const ltriples_options* o, size_t* bytes);

/* Adjoint of ltriples_energy_rhf: gbar * dE/dx for every closed-shell
 * input.  The spin-block adjoint runs on the aliased alpha/beta data over
 * the aaa and aab items with 2 gbar; the alpha and beta gradients of each
 * shared input are added, and dE/dtau collects the mixed-spin gradient
 * (symmetrised) and twice the same-spin ones (tau enters the same-spin
 * amplitudes as tau^{ab}_{ij} - tau^{ba}_{ij}).  Precision LT_FP64, LT_FP32
 * or LT_BF16X3 (as ltriples_backward); options as ltriples_energy_rhf;
 * errors as ltriples_backward. */
int ltriples_backward_rhf(const ltriples_rhf_domain* d, int32_t precision,
                          const ltriples_options* o, const double* gbar,
                          const ltriples_rhf_grad* grad, void* ws, size_t ws_bytes,
                          void* stream);

/* Three-index integrals of one LIS for the natural-auxiliary-function step
 * (section "Natural auxiliary functions", eq. naf_w): J_s[X][p][q] for each
 * spin over all nx auxiliary functions and all n_s = no_s + nv_s orbitals of
 * that spin (occupied first, then virtual), symmetric in (p, q) (not
 * checked; the W build reads p <= q only).  Device pointers, FP64. */
typedef struct ltriples_naf_input {
  int32_t no_a, nv_a, no_b, nv_b, nx;
  const double *Ja, *Jb;
} ltriples_naf_input;

/* Outputs of ltriples_naf: the factors in the NAF basis in the
 * ltriples_domain layouts ([naux][..][..]), each with room for nx rows of
 * which the first naux are written; eigenvalues (device double[nx],
 * decreasing) may be NULL, and so may any factor block. */
typedef struct ltriples_naf_output {
  double *Boo_a, *Bov_a, *Bvv_a, *Boo_b, *Bov_b, *Bvv_b;
  double* eigenvalues;
} ltriples_naf_output;

/* Host-only: workspace bytes of ltriples_naf. */
int ltriples_naf_workspace_size(const ltriples_naf_input* in, size_t* bytes);

/* Natural auxiliary functions shared by both spins: W_s = sum_{p<=q}
 * J_s[X][pq] J_s[Y][pq], W = (W_a + W_b)/2, its eigenvectors U with
 * eigenvalue > eps kept in order of decreasing eigenvalue, and
 * B^Q_pq = sum_X U[X][Q] J_s[X][p][q] sliced into the occupied-occupied,
 * occupied-virtual and virtual-virtual blocks of each spin.  *naux_out
 * (host) receives the number kept.  W and the compressed factors are formed
 * by rocBLAS GEMMs and W is diagonalised by rocSOLVER (syevd) on `stream`;
 * the call waits for the stream once to count the kept eigenvalues.  The
 * sign of each NAF is the eigensolver's; (pq|rs) = sum_Q B^Q_pq B^Q_rs does
 * not depend on it.  ws as the other entry points (NULL: stream-ordered
 * allocation on `stream`).
 * LT_EHIP also covers a rocBLAS/rocSOLVER failure or an eigensolver that
 * did not converge. */
int ltriples_naf(const ltriples_naf_input* in, double eps, const ltriples_naf_output* out,
                 int32_t* naux_out, void* ws, size_t ws_bytes, void* stream);

/* Description of the last error on this thread ("" if none). */
const char* ltriples_last_error(void);

/* Library version string. */
const char* ltriples_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LTRIPLES_H */
