// Internal declarations shared by the HIP translation units of ltriples.
// gfx950 (CDNA4) only: wave64, MFMA matrix cores, 160 KB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace lt {

// ---------------------------------------------------------------------------
// Matrix-core traits.  Lane layouts were checked on gfx950 with an in-bounds
// probe: for every shape below the A operand of lane l is A[row(l)][k(l)],
// the B operand is B[k(l)][col(l)], and accumulator element r of lane l is
// C[c_row(l, r)][col(l)].
// ---------------------------------------------------------------------------
template <typename T> struct MF;

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <> struct MF<float> {            // v_mfma_f32_32x32x2_f32
  static constexpr int BR = 32, BC = 32, KS = 2, NACC = 16;
  typedef f32x16 acc_t;
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int a_row(int l) { return l & 31; }
  __device__ static inline int a_k(int l) { return l >> 5; }
  __device__ static inline int c_row(int l, int r) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }
  __device__ static inline int c_col(int l) { return l & 31; }
};

template <> struct MF<double> {           // v_mfma_f64_16x16x4_f64
  static constexpr int BR = 16, BC = 16, KS = 4, NACC = 4;
  typedef f64x4 acc_t;
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int a_row(int l) { return l & 15; }
  __device__ static inline int a_k(int l) { return l >> 4; }
  __device__ static inline int c_row(int l, int r) { return (l >> 4) + 4 * r; }
  __device__ static inline int c_col(int l) { return l & 15; }
};

// ---------------------------------------------------------------------------
// Segmented GEMM:  C[m][n] = sum_s sign_s sum_k Lt_s[k][m] * R_s[k][n].
// Both operands are k-major (row k contiguous in m resp. n), with row
// strides that are multiples of 4 elements and 16-byte aligned rows.
// ---------------------------------------------------------------------------
template <typename T> struct Seg {
  const T* L; int64_t lks;
  const T* R; int64_t rks;
  int32_t K; float sign;
};

// Prepared operands of one spin block (sigma = spin of the same-spin pair,
// tau = spin of the odd index of a mixed block).  All row lengths padded.
template <typename T> struct ItemOps {
  int32_t kind;                 // 0: S (same spin), 1: G (mixed), 2: Y (mixed), 3: closed shell
  int32_t o_s, v_s, o_t, v_t;
  // occupied orbitals the contractions sum over (the internal m, M): the
  // first oi_s (oi_t) of the o_s (o_t) orbitals that index the operand
  // blocks.  Equal to o_s, o_t except for a central-orbital share, whose
  // rotated central orbitals follow the LIS orbitals and are never summed.
  int32_t oi_s, oi_t;
  int64_t ld_vs, ld_vt, ld_np, ld_cb;
  const T* T2T;    // [o_s][o_s][v_s][ld_vs]   T2T[i][j][e][a] = t^{ae}_{ij}
  const T* Tp;     // [o_s][o_s][ld_np]        Tp[i][m][p(a<b)] = t^{ab}_{im}
  const T* As;     // [o_s][v_s][ld_np]        As[i][e][p(b<c)] = <ei||bc>
  const T* GamT;   // [o_s][o_s][o_s][ld_vs]   GamT[j][k][m][a] = <ma||jk>
  const T* LmixT;  // [o_s][o_t][v_t][ld_vs]   LmixT[i][K][E][a] = t^{aE}_{iK}
  const T* Mst;    // [o_s][v_t][ld_cb]        Mst[j][E][C*v_s+b] = (jb|EC)
  const T* Mts;    // [o_t][v_s][ld_cb]        Mts[K][e][C*v_s+b] = (be|KC)
  const T* Tmix;   // [o_s][o_t][ld_cb]        Tmix[i][K][C*v_s+b] = t^{bC}_{iK}
  const T* ZpT;    // [o_s][o_t][o_t][ld_vs]   ZpT[j][K][M][a] = (aj|MK)
  const T* TmT;    // [o_s][o_t][v_s][ld_vt]   TmT[i][K][e][C] = t^{eC}_{iK}
  const T* OOT;    // [o_t][o_s][o_s][ld_vt]   OOT[K][j][m][C] = (jm|CK)
  // closed-shell (kind 3) operands over spatial orbitals, tau the spatial
  // amplitudes; T2T above holds T2T[i][j][e][a] = tau^{ae}_{ij}
  int64_t ld_vv;
  const T* RVc;    // [o][v][ld_vv]            RVc[r][e][b*v+c] = (rc|be)
  const T* RVs;    // [o][v][ld_vv]            RVs[q][e][b*v+c] = (qb|ce)
  const T* Tf;     // [o][o][ld_vv]            Tf[x][m][b*v+c] = tau^{bc}_{xm}
  const T* Ts;     // [o][o][ld_vv]            Ts[x][m][b*v+c] = tau^{bc}_{mx}
  const T* Gcs;    // [o][o][o][ld_vs]         Gcs[x][y][m][a] = (ya|mx)
  const int32_t* items;  // [n][3] occupied triplets of the batch
};

template <typename T> struct GemmArgs {
  int32_t M, N, nbatch, mt, nt;
  int32_t mode;                 // 0: single strided segment per batch, 1: item
  // output: out + b*obs + (m/mdiv)*s_mq + (m%mdiv)*s_mr + (n/ndiv)*s_nq + (n%ndiv)*s_nr
  T* out; int64_t obs;
  int64_t s_mq, s_mr, s_nq, s_nr;
  int32_t mdiv, ndiv;
  // mode 0
  const T* L; int64_t lks, lbs;
  const T* R; int64_t rks, rbs;
  int32_t K;
  // mode 1
  ItemOps<T> ops;
};

// ---------------------------------------------------------------------------
// BF16 split operands.  A prepared FP32 operand viewed as [nblk][K][ld]
// (block, contraction row k, column) is stored as two bf16 arrays
// hi = bf16(x), lo = bf16(x - hi), each in "octet" layout
// [nblk][K16/8][ld][8] with K16 = K rounded up to 16 (extra rows zero): one
// 16-byte word holds 8 consecutive k of one column, which is exactly one
// lane's operand of the 32x32x16 BF16 matrix instruction, and every K step
// of 16 lies inside one zero-padded block.  Allocations carry one extra
// 128-column row of slack so whole-wave loads past the last column stay in
// bounds (such lanes only feed discarded output rows/columns).
// ---------------------------------------------------------------------------
typedef uint16_t bf16_t;

struct Seg8 {
  const bf16_t *Lh, *Ll; int64_t lq;   // L octet (q, m) at L + q*lq + m*8
  const bf16_t *Rh, *Rl; int64_t rq;   // R octet (q, n) at R + q*rq + n*8
  int32_t K; float sign;
};

struct ItemOps8 {
  int32_t kind;                          // 0: S, 1: G, 2: Y, 3: closed shell (as ItemOps)
  int32_t o_s, v_s, o_t, v_t;
  int32_t oi_s, oi_t;                    // summed occupied orbitals (as ItemOps)
  int64_t ld_vs, ld_vt, ld_np, ld_cb;
  // hi/lo octet tensors; block = leading indices, K = contraction rows
  const bf16_t *T2Th, *T2Tl;     // blk (i,j)  K v_s  ld_vs
  const bf16_t *Tph, *Tpl;       // blk i      K oi_s ld_np
  const bf16_t *Ash, *Asl;       // blk i      K v_s  ld_np
  const bf16_t *GamTh, *GamTl;   // blk (j,k)  K oi_s ld_vs
  const bf16_t *LmixTh, *LmixTl; // blk (i,K)  K v_t  ld_vs
  const bf16_t *Msth, *Mstl;     // blk j      K v_t  ld_cb
  const bf16_t *Mtsh, *Mtsl;     // blk K      K v_s  ld_cb
  const bf16_t *Tmixh, *Tmixl;   // blk i      K oi_t ld_cb   (t^{bC}_{iM} over M)
  const bf16_t *Tmx2h, *Tmx2l;   // blk K      K oi_s ld_cb   (t^{bC}_{mK} over m)
  const bf16_t *ZpTh, *ZpTl;     // blk (j,K)  K oi_t ld_vs
  const bf16_t *TmTh, *TmTl;     // blk (i,K)  K v_s  ld_vt
  const bf16_t *OOTh, *OOTl;     // blk (K,j)  K oi_s ld_vt
  // closed-shell (kind 3), as ItemOps; T2T above is the spatial one
  int64_t ld_vv;
  const bf16_t *RVch, *RVcl;     // blk r      K v_s  ld_vv
  const bf16_t *RVsh, *RVsl;     // blk q      K v_s  ld_vv
  const bf16_t *Tfh, *Tfl;       // blk x      K oi_s ld_vv
  const bf16_t *Tsh, *Tsl;       // blk x      K oi_s ld_vv
  const bf16_t *Gcsh, *Gcsl;     // blk (x,y)  K oi_s ld_vs
  const int32_t* items;
};

// Items of one domain in a launch that covers several domains: their own
// output shape, output array and segment descriptors.
struct Chunk16 {
  int32_t M, N, nbatch;
  float* out; int64_t obs, ldo;
  const Seg8* tab;                       // [nbatch][6]
};
constexpr int kMaxChunk16 = 16;          // domains per launch

struct GemmArgs16 {
  int32_t M, N, nbatch, mt, nt;
  int32_t nprod;                         // 3: hi*hi + hi*lo + lo*hi, 1: hi*hi
  float* out; int64_t obs, ldo;
  int32_t kind;                          // 0: S, 1: G, 2: Y, 3: closed shell (segments 6, 6, 4, 4)
  const Seg8* tab;                       // [nbatch][6] segment descriptors of the launch's items
  // nchunk > 0: the launch covers ch[0..nchunk) instead (M and N above are
  // then the largest chunk's, for the tile choice; out, obs, ldo, tab and
  // nbatch are unused).  Chunk c owns the work-groups [cblk[c], cblk[c+1]),
  // filled in by the launcher for the chosen tile shape.
  int32_t nchunk;
  int32_t cblk[kMaxChunk16 + 1];
  Chunk16 ch[kMaxChunk16];
};

// `tune`: on the first launch of a shape class (device, products, output
// kind, 32-row blocks, log2 N) time every candidate tile configuration on
// this launch and keep the fastest for the class (not under graph capture;
// waits for the stream).  Without it the class keeps a tuned choice if one
// exists (in this process or in the tuning cache file), else the default
// table.  `force` >= 0 runs configuration `force` of the table instead.
hipError_t launch_gemm_bf16(const GemmArgs16& g, hipStream_t s, bool tune = false, int force = -1);
void reset_gemm_bf16_tuning();
// tab[n][s] = descriptor of segment s of item n (ops.kind, ops.items), s < 6;
// unused slots get K = 0.
hipError_t launch_seg8_table(const ItemOps8& ops, int32_t nitems, Seg8* tab, hipStream_t s);

// hi/lo octet tensors from FP32 in[b*ibs + k*iks + c], c < ncol, k < K
// (zero elsewhere, rows padded to 16).
hipError_t launch_split8(bf16_t* hi, bf16_t* lo, int64_t nblk, int32_t K, int64_t ld, int32_t ncol,
                         const float* in, int64_t ibs, int64_t iks, hipStream_t s);

// ---------------------------------------------------------------------------
// Energy epilogues (FP64): W assembly from the contraction outputs, V, D,
// per-tile partial sums of {E4, E_ST, E_DT}.
// ---------------------------------------------------------------------------
constexpr int ET = 16;   // epilogue tile edge

template <typename T> struct EpiSame {
  int32_t o, v; int64_t ld_np;
  const T* S; int64_t s_item;          // S[item][a][ld_np]
  const int32_t* items;                // [n][3]
  int32_t nt, ntri;
  const double *eo, *ev, *t1, *f, *t2; // t2 [o][o][v][v] (input)
  const double* U; int64_t ld_v;       // U[q][r][y][ld_v] = <qr||yz>
  double* part;                        // [n][ntri][3]
  // Laplace weights of a central-orbital share (null otherwise): the item's
  // occupied index in slot lap_slot is the rotated central orbital
  // lap_o0 + q (its orbital energy set to zero in eo), and 1/D is replaced
  // by lap[2q + 1] * exp(lap[2q] * D)
  const double* lap; int32_t lap_o0, lap_slot;
};

template <typename T> struct EpiMixed {
  int32_t o_s, v_s, o_t, v_t; int64_t ld_np, ld_cb;
  const T* G; int64_t g_item;          // G[item][a][ld_cb]
  const T* Y; int64_t y_item;          // Y[item][C][ld_np]
  const int32_t* items;
  int32_t nts, ntt, ntiles;
  const double *eo_s, *ev_s, *eo_t, *ev_t, *t1_s, *t1_t, *f_s, *f_t;
  const double* t2ss;                  // [o_s][o_s][v_s][v_s] (input)
  const double* U; int64_t ld_vs;      // U_s[i][j][a][ld_vs] = <ij||ab>
  // (jb|KC) at ov + j*ov_o + b*ov_v + K*ov_O + C*ov_V ; t^{bC}_{jK} likewise
  const double* ov; int64_t ov_o, ov_v, ov_O, ov_V;
  const double* tm; int64_t tm_o, tm_v, tm_O, tm_V;
  double* part;                        // [n][ntiles][3]
  const double* lap; int32_t lap_o0, lap_slot;   // as EpiSame
};

// ---------------------------------------------------------------------------
// Launchers (all asynchronous on `s`)
// ---------------------------------------------------------------------------
// `tune`, `force`: as launch_gemm_bf16, for the triplet contractions (mode 1).
template <typename T> hipError_t launch_gemm(const GemmArgs<T>& g, hipStream_t s, bool tune = false,
                                             int force = -1);
void reset_gemm_tuning();

// Tile choices persisted across processes in the JSON file named by the
// environment variable LTRIPLES_TUNE_CACHE (no file: both calls do nothing).
// Entries are keyed by kernel family, the device's architecture name and
// four integers of the shape class.  get returns -1 when absent.
int tune_cache_get(const char* family, int dev, int k0, int k1, int k2, int k3);
void tune_cache_put(const char* family, int dev, int k0, int k1, int k2, int k3, int cfg);

// out[d0][d1][d2][d3] (out strides os0..os2, unit stride in d3)
//   = in[d0*s0 + d1*s1 + d2*s2 + d3*s3] - (in2 ? in2[d0*u0 + ... + d3*u3] : 0)
template <typename Tin, typename Tout>
hipError_t launch_copy4d(Tout* out, int64_t os0, int64_t os1, int64_t os2,
                         int64_t d0, int64_t d1, int64_t d2, int64_t d3,
                         const Tin* in, int64_t s0, int64_t s1, int64_t s2, int64_t s3,
                         const Tin* in2, int64_t u0, int64_t u1, int64_t u2, int64_t u3,
                         hipStream_t s);

// out[r][p(x<y)] = in[r*rs + x*xs + y*ys] - (antisym ? in[r*rs + y*xs + x*ys] : 0)
// for x < y < n, p(x,y) = y(y-1)/2 + x; out row stride ldo.
template <typename Tin, typename Tout>
hipError_t launch_pack_pairs(Tout* out, int64_t ldo, int64_t rows, int32_t n,
                             const Tin* in, int64_t rs, int64_t xs, int64_t ys,
                             bool antisym, hipStream_t s);

template <typename T> hipError_t launch_epi_same(const EpiSame<T>& a, int32_t nitems, hipStream_t s);
template <typename T> hipError_t launch_epi_mixed(const EpiMixed<T>& a, int32_t nitems, hipStream_t s);
// Closed-shell (spin-adapted) energy epilogue.  For an occupied triple
// i <= j <= k the contraction writes three cubes A = F(i,j,k)[a][b*v+c],
// B = F(j,i,k)[b][a*v+c], C = F(k,i,j)[c][a*v+b] (see the driver in
// lt_api.hip); W^{abc} = A[a][b][c] + B[b][a][c] + C[c][a][b].
template <typename T> struct EpiRhf {
  int32_t o, v, nt, ntiles;           // 16-wide virtual tiles, ntiles = nt(nt+1)/2 (a-tile <= b-tile)
  const T* W; int64_t w_item, cube;   // A of item n at W + n*w_item; B, C at + cube, + 2 cube
  const int32_t* items;               // [n][3] occupied triples i <= j <= k, not all equal
  const double *eo, *ev, *t1, *f;     // orbital energies, t1 [o][v], f_ov [o][v]
  const double* tau;                  // [o][o][v][v] spatial amplitudes
  const double* ov;                   // [o][v][o][v] (ia|jb)
  double* part;                       // [n][ntiles][3]
};
template <typename T> hipError_t launch_epi_rhf(const EpiRhf<T>& a, int32_t nitems, hipStream_t s);
// Debug dumps of one item's W over its full virtual cube (FP64, row-major),
// formed from the contraction outputs exactly as the epilogues read them:
// same spin from S (v^3 entries), mixed from G and Y (v_s * v_s * v_t).
template <typename T> hipError_t launch_dump_w_same(const T* S, int64_t ld_np, int32_t v, double* w,
                                                    hipStream_t s);
template <typename T> hipError_t launch_dump_w_mixed(const T* G, int64_t ld_cb, const T* Y, int64_t ld_np,
                                                     int32_t vs, int32_t vt, double* w, hipStream_t s);

// e_items[dst[b]][0..2] = sum over t of part[b][t][0..2] (fixed order)
hipError_t launch_reduce_items(const double* part, int32_t nitems, int32_t ntiles,
                               const int32_t* dst, double* e_items, hipStream_t s);
// parts[blk][q] = sum of e_items[n][q] over n in [first[blk], first[blk]+count[blk]) of the
// block-ordered index list `order`; e_out = sum of parts.
hipError_t launch_reduce_final(const double* e_items, const int32_t* order,
                               const int32_t* first, const int32_t* count,
                               double* parts, double* e_out, hipStream_t s);
hipError_t launch_zero(double* p, int64_t n, hipStream_t s);
// Central-orbital share inputs.  coef[q][i] = c[i] * exp(lap[2q] * eo[i] / 2)
// for q < nq, i < o: the central orbital with the point's orbital factor.
hipError_t launch_central_coef(double* coef, const double* c, const double* eo, const double* lap, int32_t o,
                               int32_t nq, hipStream_t s);
// One occupied axis (length o) of in[pre][o][post] extended by nq rotated
// orbitals: out[x][p][y] = in[x][p][y] for p < o and
// sum_i coef[p - o][i] in[x][i][y] for o <= p < o + nq.
hipError_t launch_aug_axis(double* out, const double* in, const double* coef, int64_t pre, int32_t o,
                           int32_t nq, int64_t post, hipStream_t s);
// flag[0] = 1 if any element of the listed arrays is NaN or infinite (flag
// zeroed beforehand by the caller; untouched otherwise)
struct FiniteScan {
  const double* p[17];
  int64_t n[17];
  int32_t narr;
};
hipError_t launch_scan_finite(const FiniteScan& a, int32_t* flag, hipStream_t s);
// n 32-bit words of zeros
hipError_t launch_zero32(void* p, int64_t n, hipStream_t s);

// ---------------------------------------------------------------------------
// Adjoint (backward) pass
// ---------------------------------------------------------------------------
// Descriptor-driven reverse GEMM.  Output block b accumulates
//   out[r*ldo + c] += sum_{s in [beg,end)} sign_s sum_{x < K_s} A_s(x, r) B_s(x, c)
// for r < rows, c < cols, with A_s(x, r) = A[r*lda + x] (contraction index
// contiguous) and B_s(x, c) = TB ? B[c*ldb + x] : B[x*ldb + c].  Row strides
// are multiples of 4 elements, rows 16-byte aligned and readable up to the
// next multiple of 4 past the contraction length.  Distinct blocks of one
// launch must not overlap in memory.
template <typename T> struct RSeg {
  const T* A; int64_t lda;
  const T* B; int64_t ldb;
  int32_t K; float sign;
};
template <typename T> struct RBlk {
  T* out; int64_t ldo;
  int32_t rows, cols, beg, end;
  int32_t store;                   // 1: out = sum (partial of a split target), 0: out += sum
  int32_t pad;
};
// Split targets: out[r*ldo + c] += sum_{j < nchunk} part[j*rows*cols + r*cols + c]
// (FP64 sum in chunk order).
template <typename T> struct RRed {
  T* out; int64_t ldo;
  const T* part;
  int32_t rows, cols, nchunk, pad;
};
template <typename T> hipError_t launch_rreduce(const RRed<T>* reds, int32_t nred, int32_t max_elems,
                                                hipStream_t s);
template <typename T> struct RArgs {
  int32_t nblk, mt, nt, max_rows, max_cols;
  const RBlk<T>* blks;
  const RSeg<T>* segs;
};
template <typename T> hipError_t launch_rgemm(RArgs<T> g, bool tb, hipStream_t s);

// Backward epilogues: recompute W (and V, D) from the contraction outputs of
// one batch and write the adjoints of those outputs,
//   dX  = gbar (2W + V) / D   placed at the positions W reads (with signs),
//   dXV = gbar W / D          likewise for the singles/f_ov intermediates,
// every element of the item's output layout written (zeros where W reads
// nothing).  With `ep` set they also reduce q = gbar W (W + V) / D^2, the
// adjoint of -D, per work-group tile: ep[item][tile][64] holds the sums over
// the tile's elements with a fixed first (slots 0-15), second (16-31) and
// third (32-47) virtual index, and the tile total at slot 48.
template <typename T> struct BwdSame {
  EpiSame<T> e;                        // part unused
  const double* gbar;
  T* dS; T* dSV;                       // [item][a][ld_np], item stride e.s_item
  double* ep;                          // [item][ntri][64] or null
};
template <typename T> struct BwdMixed {
  EpiMixed<T> e;
  const double* gbar;
  T *dG, *dGV;                         // [item][a][ld_cb], stride e.g_item
  T *dY, *dYV;                         // [item][C][ld_np], stride e.y_item
  double* ep;                          // [item][ntiles][64] or null
};
template <typename T> hipError_t launch_bwd_same(const BwdSame<T>& a, int32_t nitems, hipStream_t s);
template <typename T> hipError_t launch_bwd_mixed(const BwdMixed<T>& a, int32_t nitems, hipStream_t s);

// Orbital-energy adjoint of one batch from the tile sums above.  D =
// e_i + e_j + e_k - e_a - e_b - e_c, so dE/de_virtual gathers +q over the
// positions where the index occurs and dE/de_occupied gathers -q over the
// items that contain it.  Two fixed-order passes: per item and index
// (ri[item][ld_ri]: spin-s virtuals, spin-t virtuals, item total), then over
// the batch's items into the outputs (accumulated; null outputs skipped).
struct EpsReduce {
  int32_t mixed, nitems, nwg;          // nwg: tiles per item of the epilogue grid
  int32_t nt_s, nt_t;                  // virtual tiles per spin (nt_t mixed only)
  int32_t o_s, v_s, o_t, v_t;
  const double* ep;                    // [item][nwg][64]
  double* ri; int64_t ld_ri;
  const int32_t* items;                // [item][3]: (i, j, k) resp. (i, j, K)
  double *eo_s, *ev_s, *eo_t, *ev_t;
};
hipError_t launch_eps_reduce(const EpsReduce& r, hipStream_t s);

// P[X][pair] = J[X][p][q] for p <= q (pair-packed rows of n (n + 1) / 2)
hipError_t launch_naf_pack(double* P, const double* J, int32_t n, int32_t nx, hipStream_t s);

// e_out[0] = 2 in[0]; parts[x] = 2 (in[1 + x] + in[4 + x]) when parts is set
hipError_t launch_rhf_combine(const double* in, double* e_out, double* parts, hipStream_t s);

// out[x0*o0 + x1*o1 + x2*o2 + x3*o3] += scale * in[x0*i0 + x1*i1 + x2*i2 + x3*i3]
// over x < d (a bijection: each output element written by one thread).
template <typename Tin>
hipError_t launch_perm_acc(double* out, const int64_t d[4], const int64_t os[4], const Tin* in,
                           const int64_t is[4], double scale, hipStream_t s);
// Pair-packed rows to squares: for r0 < R0, r1 < R1, x, y < n
//   out[r0*o0 + r1*o1 + x*ox + y*oy] += x < y ? s_up * in[r0*i0 + r1*i1 + p(x,y)]
//                                     : x > y ? s_lo * in[r0*i0 + r1*i1 + p(y,x)] : 0
template <typename Tin>
hipError_t launch_unpack_acc(double* out, int64_t R0, int64_t R1, int32_t n, int64_t o0, int64_t o1,
                             int64_t ox, int64_t oy, const Tin* in, int64_t i0, int64_t i1, double s_up,
                             double s_lo, hipStream_t s);
// In-place projections: t[o][o][v][v] antisymmetrised in (0,1) and (2,3);
// b[Q][n][n] symmetrised in (1,2).
hipError_t launch_antisym4(double* t, int64_t o, int64_t v, hipStream_t s);
hipError_t launch_sym3(double* b, int64_t Q, int64_t n, hipStream_t s);

}  // namespace lt
