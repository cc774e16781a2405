// Internal declarations shared by the host orchestration (adc.cpp, engine.cpp)
// and the device kernels (kernels.hip).  Complex numbers are interleaved
// (re, im) float64 pairs (double2) in every tensor.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <shared_mutex>
#include <string>
#include <vector>

namespace adc {

struct cplx {
  double re, im;
};

// ---------------------------------------------------------------- GEMM
// Optional N-d layout of a GEMM output: with nm > 0 the row index m is split
// in the mixed radix md[0..nm) (last digit fastest) and its C offset is
// sum_q digit_q * ms[q] (instead of m * scm); likewise nn/nd/ns for columns.
// Lets one GEMM write straight into an output whose M or N labels are not one
// fused stride.  Each group's extent must stay below 2^31.
struct OutMap {
  int nm, nn;
  int64_t md[3], ms[3], nd[3], ns[3];
};

// C[b] = alpha * op(A[b]) op(B[b]) + beta * C[b] with element strides
// (complex elements) A(m,k) at A + m*sam + k*sak + b*sab, B(k,n) at
// B + k*sbk + n*sbn + b*sbb, C(m,n) at C + m*scm + n*scn + b*scb.
// conjA / conjB conjugate the operand.  beta == 0 never reads C.
struct GemmDesc {
  int64_t M, N, K, batch;
  const double2* A; int64_t sam, sak, sab;
  const double2* B; int64_t sbk, sbn, sbb;
  double2* C; int64_t scm, scn, scb;
  cplx alpha, beta;
  int conjA, conjB;
  int tag;  // kernel instance: 0 generic, 1 ladder assembly, 2 ladder contraction
  // split-K: nsplit > 1 writes raw partial sums of K-chunks of length kchunk
  // to P[((s*batch + b)*M + m)*N + n]; a reduction applies alpha/beta into C
  int64_t kchunk;
  int nsplit;
  double2* P;
  int tile;  // -1 heuristic, 0 small tiles, 1 large tiles
  OutMap om;
  int c32 = 0;  // C holds complex64 (float2) elements
};
void launch_splitk_reduce(const GemmDesc& g, hipStream_t s);
// prec: 0 = FP64 MFMA, 1 = FP32 MFMA (operands rounded to fp32, fp32
// accumulate), 2 = split-bf16 (three bf16 MFMA products, fp32 accumulate).
void launch_zgemm(const GemmDesc& g, int prec, hipStream_t s);

// ---------------------------------------------------------------- split-bf16 planes
// One problem of a grouped split-bf16 GEMM (BfGemm.probs): shape M x N, the
// first tile of its range of the grid, the plane rows its A and B rows start
// at (row r of A is plane row arow + (r / amd) * ams + r % amd with the
// GEMM's ams, likewise B with bmd, bms), and its output at C + coff with row
// stride ldc (unit column stride, in the GEMM's C element type).
struct GroupProb {
  int64_t tile0;
  int64_t M, N;
  int64_t arow, brow, amd, bmd;
  int64_t coff, ldc;
};
// C(m,n) = alpha * sum_k A(m,k) B(n,k) + beta C (note: B is given row-major in n)
// with A, B as bf16 split planes [4][rows][Kp] (re hi, re lo, im hi, im lo).
struct BfGemm {
  int64_t M, N, Kp;
  const unsigned short* A; int64_t lda;   // rows per plane of A (>= M)
  const unsigned short* B; int64_t ldb;   // rows per plane of B (>= N)
  double2* C; int64_t scm, scn;
  cplx alpha, beta;
  int tag;
  int64_t kchunk;
  int nsplit;
  double2* P;
  int tile;  // -1 heuristic, else a tile code of launch_bf16p
  OutMap om;
  // optional row maps of the operands: row r of A is stored at plane row
  // (r / amd) * ams + r % amd (amd = 0: row r); likewise B with bmd, bms
  int64_t amd = 0, ams = 0, bmd = 0, bms = 0;
  int colmajor = 0;  // set by launch_bf16p: tiles walk down columns (N > M)
  int c32 = 0;       // C holds complex64 (float2) elements
  // grouped GEMM (direct-load tiles, no split-K): nprob problems in device
  // memory, gtiles tiles in all; M, N, C offsets and row maps come from the
  // problems, the planes, Kp, ams, bms, alpha, beta and c32 from here
  const GroupProb* probs = nullptr;
  int nprob = 0;
  int64_t gtiles = 0;
};
void launch_bf16p(const BfGemm& g, hipStream_t s);
// true while work on stream s is being captured into a graph
bool capturing(hipStream_t s);
// the tile launch_bf16p takes for g.tile < 0
int bf16p_pick_tile(const BfGemm& g);
void launch_splitk_reduce_bf(const BfGemm& g, hipStream_t s);
// dst planes [4][rows][Kp] from src(r, k) = src[r*srow + k*sk] (conj: negate im), zero for k >= K
void launch_split_planes(const double2* src, int64_t rows, int64_t K, int64_t srow, int64_t sk, int conj,
                         unsigned short* dst, int64_t Kp, hipStream_t s);
// Split planes [4][rows][Kp] of an operand given as an N-d view: row r and
// column k (< K) are split in mixed radices md/kd (last digit fastest, at most
// four digits each) with source strides ms/ks; zero for K <= k < Kp.
struct SplitNd {
  const double2* src;
  unsigned short* dst;
  int nm, nk;
  int64_t md[4], ms[4], kd[4], ks[4];
  int64_t rows, K, Kp;
  int conj;
};
// tiled = 1 stages 64 x 32 blocks through LDS so that reads run along the
// rows (for sources whose unit stride is a row digit)
void launch_split_nd(const SplitNd& p, int tiled, hipStream_t s);
void launch_ladder_pack_planes(const double2* W, int64_t ldw, int a0, int b0, int nv, unsigned short* V, int64_t ldv,
                               int64_t r0, int64_t pbase, int64_t npairs, const int2* pv, int64_t Kp, hipStream_t s);
// Upper half of the packed <ab||cd> rows of one a-block, as split planes:
// W[(a-a0)*(nv-a0) + c-a0][(b-b0)*(nv-a0) + d-a0] = sum_Q L_ac L_bd holds only
// c, d >= a0; row ab (pair index p) gets <ab||cd> for pairs cd >= p and zero
// padding; the part below p is left for launch_ladder_mirror_planes.  W holds
// complex128 (w32 = 0) or complex64 (w32 = 1) elements
void launch_ladder_pack_planes_upper(const void* W, int w32, int64_t ldw, int a0, int b0, int nv, unsigned short* V,
                                     int64_t ldv, int64_t pbase, int64_t npairs, const int2* pv, int64_t Kp,
                                     hipStream_t s, int64_t vrow0 = 0);
// (vrow0: pair p goes to V row p - vrow0, for a group of rows starting there)
// split planes [4][ldv][Kp]: V[pl][r][0:c1] = 0 for r < rows
void launch_planes_zero_cols(unsigned short* V, int64_t ldv, int64_t rows, int64_t c1, int64_t Kp, hipStream_t s);
// lower part of a row group's diagonal block: V[r][col0 + c] = conj V[c][col0 + r], c < r < n
void launch_ladder_mirror_block(unsigned short* V, int64_t ldv, int64_t n, int64_t Kp, int64_t col0, hipStream_t s);
// T [4][ncols][Kt] with T[q][koff + r] = conj V[r][c0 + q] (r < rows, q < ncols), zero elsewhere
void launch_ladder_transpose_planes(const unsigned short* V, int64_t ldv, int64_t rows, int64_t c0, int64_t ncols,
                                    int64_t Kp, unsigned short* T, int64_t Kt, int64_t koff, hipStream_t s);
// dst [4][rows][Kt] = columns c0 .. c0 + Kt of src [4][rows][Kp]
void launch_planes_copy_cols(const unsigned short* src, int64_t rows, int64_t Kp, int64_t c0, unsigned short* dst,
                             int64_t Kt, hipStream_t s);
// V[p][q] = conj(V[q][p]) for q < p < n on split planes [4][ldv][Kp] (the
// packed <ab||cd> matrix is Hermitian)
void launch_ladder_mirror_planes(unsigned short* V, int64_t ldv, int64_t n, int64_t Kp, hipStream_t s);
// The same upper-half pack for the pairs pbase .. pbase + npairs whose first
// index a is spread over blocks of an exact-range assembly: blk[a] = {a0 of
// a's block, complex64 offset of the block's W in Wall, its row stride}; a
// block's W holds sum_Q L_ac L_bd at [(a-a0)*m + c-a0][(b-a0-1)*m + d-a0],
// m = nv - a0, c, d >= a0
struct LadBlk {
  int64_t a0, woff, ldw;
};
void launch_ladder_pack_planes_grouped(const void* Wall, const LadBlk* blk, int nv, unsigned short* V, int64_t ldv,
                                       int64_t pbase, int64_t npairs, const int2* pv, int64_t Kp, hipStream_t s);

// ---------------------------------------------------------------- permute
// out[sum_d idx_d * ostr[d]] = alpha * op(in[sum_d idx_d * istr[d]]) + beta * out[...]
// over the index box od[0..nd)
void launch_permute(int nd, const int64_t* od, const int64_t* istr, const int64_t* ostr, const double2* in,
                    double2* out, cplx alpha, cplx beta, int conj, hipStream_t s);
// M[i][i] += d[i] (real) for an n x n matrix
void launch_add_diag(double2* M, const double* d, int64_t n, hipStream_t s);
// R[r][i] = AX[r][i] - w[r] X[r][i]
void launch_resid(const double2* AX, const double2* X, const double* w, double2* R, int rows, int64_t n,
                  hipStream_t s);

// ---------------------------------------------------------------- misc
void launch_fill(double2* p, int64_t n, cplx v, hipStream_t s);
void launch_scale_real(double2* p, const double* w, int64_t n, int64_t period, int invert, hipStream_t s);
// out[r][c] = X[r][c] + conj(X[c][r]) (n x n), out may not alias X
void launch_herm_add(const double2* X, double2* out, int64_t n, hipStream_t s);
// M (n1 x n1, n1 = no*nv, index (i,a) i-major): M[(i,a),(i,A)] += f[a][A]  (diag_occ)
// or M[(i,a),(I,a)] += h[i][I] (diag_vir)
void launch_m11_add_delta(double2* M, const double2* f, int no, int nv, int which, hipStream_t s);
// denominators: t[i][j][a][b] = num / (e_i + e_j - e_a - e_b)   (or * when invert=0)
void launch_div_d2(double2* t, const double* eps, int no, int nv, hipStream_t s);
void launch_div_d1(double2* t, const double* eps, int no, int nv, hipStream_t s);

// Packed ISR vector <-> unpacked doubles tensor conversions.
// kind: 0 EE [k][o][o][v][v], 1 IP [k][o][o][v], 2 EA [k][o][v][v].
// unpack: Ya antisymmetric in every pair; Yp (optional) zero except packed positions.
// split-bf16 planes [4][k*o*v][Kp] of the EE doubles in the ring layout
// (rows (z,i,a), columns (k,c) < o*v, zero beyond), from the doubles with the
// occupied pair packed, Yij [k][v][P_o][v]
void launch_ee_ring_planes(const double2* Yij, int k, int no, int nv, unsigned short* dst, int64_t Kp,
                           hipStream_t s);
// straight from the packed EE vectors Y (row z at Y + z*ldY + off): the
// split-bf16 planes [4][k*v][Kpy] of Yij read as rows (z,a), columns
// (pair ij, b) (zero beyond P_o*v), and, when rq is given, the ring-layout
// planes above into rq [4][k*o*v][Kpr]; the same values as
// launch_unpack_doubles(3) followed by the split (and launch_ee_ring_planes)
void launch_ee_pair_planes(const double2* Y, int64_t ldY, int64_t off, int k, int no, int nv, unsigned short* yq,
                           int64_t Kpy, unsigned short* rq, int64_t Kpr, hipStream_t s);
// kind 0: EE [k][o][o][v][v]; 1: IP [k][o][o][nv] (also EE with nv = P_v:
// occupied pair unpacked); 2: EA [k][no][v][v] (also EE with no = P_o:
// virtual pair unpacked); 3: EE [k][v][P_o][v] (virtual pair unpacked, the
// occupied pair index in the middle).  planes (optional): split-bf16 planes
// of the result read as row-major [rows][pK], written as [4][rows][pKp] with
// zero columns beyond pK (pK = 0: the whole result as one row)
void launch_unpack_doubles(int kind, const double2* Y, int64_t ldY, int64_t off, int k, int no, int nv,
                           double2* Ya, double2* Yp, hipStream_t s, unsigned short* planes = nullptr,
                           int64_t pK = 0, int64_t pKp = 0);
// S[z][off + packed] = alpha * U[z][...] + D[packed] * Y[z][off + packed] (+ S if accumulate)
void launch_pack_doubles(int kind, const double2* U, double2* S, const double2* Y, int64_t ld, int64_t off,
                         int k, int no, int nv, const double* eps, cplx alpha, int accumulate,
                         const int2* pair_o, const int2* pair_v, hipStream_t s);
// antisymmetrisers on [k][p][p][q][q]-like tensors: out += X - swap(pair)
// pair 0 swaps dims 1,2 ; pair 1 swaps dims 3,4 ; pair 2 swaps both pairs (P(ij)P(ab)).
void launch_antisym_add(const double2* X, double2* out, int64_t k, int64_t d1, int64_t d2, int64_t d3,
                        int64_t d4, int which, cplx alpha, hipStream_t s);

// Ladder: from W[(a - a0)*nv + c][(b - b0)*nv + d] (row length ldw) build the
// packed rows V[r][pair(c,d)] = W_ab,cd - W_ab,dc for the npairs pairs
// (a,b) = pair_v[pbase + r].
void launch_ladder_pack(const double2* W, int64_t ldw, int a0, int b0, int nv, double2* V, int64_t pbase,
                        int64_t npairs, const int2* pair_v, hipStream_t s);

// EE doubles: S[z][off + packed(ij,ab)] = P(ij) A0 + P(ab) A1 + P(ij)P(ab) A2 at
// (i<j, a<b) + D Y (A2 may be null); A0..A2 are [k][o][o][v][v]
void launch_pack_ee(const double2* A0, const double2* A1, const double2* A2, double2* S, const double2* Y, int64_t ld,
                    int64_t off, int k, int no, int nv, const double* eps, const int2* po, const int2* pv,
                    hipStream_t s, int a32 = 0);
// the same from half-stored accumulators: A0 [k][o][o][P_v] (antisymmetric in
// a,b), A1 [k][P_o][v][v] (antisymmetric in i,j), A2 [k][o][o][v][v] or null
void launch_pack_ee_half(const double2* A0, const double2* A1, const double2* A2, double2* S, const double2* Y,
                         int64_t ld, int64_t off, int k, int no, int nv, const double* eps, const int2* po,
                         const int2* pv, hipStream_t s, int a32);
// dst[o][p][i] = src[o][a][b][i] over the pairs p = (a < b) of n (anti = 1:
// src[o][a][b][i] - src[o][b][a][i]): src is [outer][n][n][inner], dst
// [outer][n(n-1)/2][inner]
void launch_pack_pairs(const double2* src, double2* dst, int64_t outer, int n, int64_t inner, const int2* pairs,
                       hipStream_t s, int anti = 0);

// adjoint helpers
// gf[a][A] += sum_i gX[(i,a),(i,A)] (which 0) or gf[i][I] += sum_a gX[(i,a),(I,a)] (which 1)
void launch_m11_delta_adjoint(const double2* gX, double2* gf, int no, int nv, int which, hipStream_t s);
// G[(x-x0)*nv + y][b*nv + d] = Gamma'[pair(x,b)][pair(y,d)] with the signs of
// the antisymmetric extension (zero when x==b or y==d), for x in [x0, x1)
void launch_expand_gamma(const double2* Gam, int64_t Pv, int x0, int x1, int nv, double2* G, hipStream_t s);
// dL[Q][p][q] = (G[Q][p][q] + conj(G[Q][q][p])) / 2
void launch_herm_project(const double2* G, double2* dL, int64_t nq, int64_t n, hipStream_t s);

// Davidson helpers
// partial[r*nb + blk] = sum_i conj(X[r][i]) Y[r][i] over the block's chunk
void launch_row_dots(const double2* X, int64_t ldx, const double2* Y, int64_t ldy, int rows, int64_t n,
                     double2* partial, int nb, hipStream_t s);
// N[r][i] = R[r][i] / den,  den = w[r] - D[i] floored at |den| >= 1e-4
void launch_precondition(const double2* R, double2* N, const double* D, const double* w, int rows, int64_t n,
                         hipStream_t s);
int row_dot_blocks(int64_t n);
// per Cholesky vector Q of L [nq][n][n]: out[3Q] = max |Re L_pr - Re L_rp| +
// |Im L_pr + Im L_rp|, out[3Q+1] = max |component|, out[3Q+2] = number of
// non-finite components (one block per Q)
void launch_check_L(const double2* L, int64_t nq, int64_t n, double* out, hipStream_t s);

// device Davidson iteration (davidson.hip)
// eigenpairs of the Hermitian part of G (n x n, row stride ldg, n at most
// heev_device_max()) in one workgroup: w ascending, U [n][ldu] columns.
// Aw, Vw are n*n workspaces for the matrix and the rotations; mode 2 keeps
// both in LDS, mode 1 the matrix only, mode 0 neither (heev_lds_bytes(n,
// mode) of dynamic LDS beside heev_static_lds()).  A non-finite G gives NaN
// eigenvalues.
int heev_device_max();
size_t heev_lds_bytes(int n, int mode);
size_t heev_static_lds();
void heev_allow_lds(size_t bytes);
void launch_heev_jacobi(const double2* G, int ldg, int n, double2* Aw, double2* Vw, int mode, double2* U, int ldu,
                        double* w, hipStream_t s);
// out[r][c] (row stride ldo) = sum_s part[s][r][c] over rows x cols parts;
// above 64 parts in two stages through stage [sum_parts_slices(nparts)][rows
// x cols] (a fixed summation order either way)
int sum_parts_slices(int nparts);
void launch_sum_parts(const double2* part, int nparts, int rows, int cols, double2* stage, double2* out, int ldo,
                      hipStream_t s);
// C[j][r] /= (w[r] - lam[j]) (j < n1, r < rows; |den| held at >= 1e-4)
void launch_shift_scale(double2* C, const double* lam, const double* w, int64_t n1, int rows, hipStream_t s);
// G[j][a] = conj(G[a][j]) for c0 <= j < m, a < c0
void launch_gram_mirror(double2* G, int ldg, int c0, int m, hipStream_t s);
// when *flag != 0: G[0:mc][0:mc] = diag(w[0:mc])
void launch_gram_diag(const double* flag, const double* w, int mc, double2* G, int ldg, hipStream_t s);
// Out[r][i] = alpha sum_a C[a][r] In[a][i] + beta Out[r][i] (r < nr, a < m,
// C row stride ldc; Out must not overlap In), a memory-bound kernel for a
// few rows over a long dim; with flag, only when *flag != 0
void launch_combine_cols(const double* flag, const double2* C, int ldc, int m, int nr, const double2* In,
                         double2* Out, int64_t dim, cplx alpha, cplx beta, hipStream_t s);
// out[r] = sum_b partial[r*nb + b] (the partials of launch_row_dots)
void launch_row_sums(const double2* partial, int nb, int rows, double2* out, hipStream_t s);
// convergence test of k roots with par = {tol, dwtol}; rep = [status, w[k],
// |r|[k], conv[k], -, -, collapse], status 1 all converged, 0 not, -1
// non-finite; collapse = 1 when m + (unconverged roots) > mmax; wold <- w
void launch_dav_converge(const double* w, const double2* rn2, double* wold, int k, int m, int mmax,
                         const double* par, double* rep, hipStream_t s);
// when *flag != 0: rows r < mc of Out become sum_a U[a][r] In[a] (a < m, via
// the temporary T [mc][dim]; Out may be In) and rows mc .. m of Out zero
void launch_collapse(const double* flag, const double2* U, int ldu, int m, int mc, const double2* In, double2* T,
                     double2* Out, int64_t dim, hipStream_t s);
// N_r -= (a_r / b_r) P_r, or N_r = 0 where flags[r] != 0
void launch_olsen(double2* N, const double2* P, const double2* a, const double2* b, const double* flags, int rows,
                  int64_t dim, hipStream_t s);
// canonical orthonormalisation coefficients C [k][k] from Gram eigenpairs
// (lam ascending, U): kept directions first, *count = kept (-1: non-finite)
void launch_canon(const double* lam, const double2* U, int ldu, int k, double2* C, double* count, hipStream_t s);

// ---------------------------------------------------------------- engine
struct Tensor {
  double2* p = nullptr;
  // complex64 elements (float2) at p: only as the output of ctr() GEMMs and
  // the input of launch_pack_ee (accumulators of reduced-precision builds)
  bool f32 = false;
  std::vector<int64_t> d;
  std::vector<int64_t> st;  // element strides; empty = contiguous row-major
  int64_t size() const {
    int64_t s = 1;
    for (auto x : d) s *= x;
    return s;
  }
};

struct Tape;

// thrown by Pool::get in arena mode when a block does not fit the arena
struct ArenaFull {
  size_t need;
};

// Calls that synchronise the whole device (hipDeviceSynchronize, hipFree)
// must not run while another thread records a stream into a graph: such a
// call would wait on the capturing stream and break its capture.  Captures
// hold this gate shared (several lanes may capture at once), those calls
// hold it exclusively.
std::shared_mutex& capture_gate();

class Pool {
 public:
  ~Pool();
  Tape* tape = nullptr;  // while set, allocations are registered and frees deferred
  double2* get(int64_t n_complex);
  void put(double2* p);
  // Arena mode: blocks come from the device range [base, base + bytes)
  // (first fit, 256-byte aligned) instead of hipMalloc, and put() returns
  // them to it; a block that does not fit throws ArenaFull.  end_arena()
  // drops the arena's bookkeeping and returns the peak bytes in use.
  void begin_arena(void* base, size_t bytes);
  size_t end_arena();
  bool in_arena() const { return arena_base_ != nullptr; }
  // Hold mode (for graph capture): blocks handed out from begin_hold() on
  // are recycled only among themselves, and end_hold() returns them; they
  // stay reserved (never handed out again) until passed to put() one by one.
  void begin_hold();
  std::vector<double2*> end_hold();
  void release_all();
  void trim();  // return cached (unused) blocks to the device
  size_t bytes_in_use() const { return in_use_; }

 private:
  struct Blk { void* p; size_t bytes; };
  std::vector<Blk> free_, used_;
  size_t in_use_ = 0;
  bool hold_ = false;
  std::vector<void*> touched_, cap_free_;
  struct Span { size_t off, len; };
  char* arena_base_ = nullptr;
  size_t arena_bytes_ = 0, arena_peak_ = 0;
  std::vector<Span> arena_free_, arena_used_;  // free spans sorted by offset
};

// ---------------------------------------------------------------- reverse mode
// A tape of the device operations of one recomputed init + sigma.  The
// backward sweep (adjoint.cpp) walks it in reverse and forms, for a real
// objective f, gradients G_X = df/dRe X + i df/dIm X of every recorded tensor.
struct Ctx;
struct TapeOp;
using LadderBw = void (*)(Ctx& cx, const TapeOp& op, const double2* gS, double2* gY);

struct TapeOp {
  enum Kind { CTR, PERM, DIV_D2, DIV_D1, ANTISYM, HERM_ADD, M11_DELTA, PACK, UNPACK, LADDER, PACK_EE } kind;
  Tensor A, B, C;
  std::string la, lb, lc;
  bool cA = false, cB = false;
  cplx alpha{1.0, 0.0}, beta{0.0, 0.0};
  // kind-specific integers:
  //  ANTISYM  n = {k, d1, d2, d3, d4, which}
  //  HERM_ADD n = {size}
  //  M11_DELTA, DIV_*  n = {o, v, which}
  //  PACK / UNPACK  n = {kind, ld, off, k, o, v, accumulate}
  //  LADDER   n = {ldY, offY, ldS, offS, nrow, k}
  //  PACK_EE  A, B, C = A0, A1, S; n = {ld, off, k, o, v}; the tensor A2 rides in `extra`
  int64_t n[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const double* eps = nullptr;
  const int2* po = nullptr;
  const int2* pv = nullptr;
  Tensor extra;
  // arithmetic the op ran in (ctr()'s precision, or the ladder's); its
  // reverse rule runs in the same one
  int prec = 0;
  void* inst = nullptr;     // LADDER: the instance whose L_vv the ladder reads
  void* owner = nullptr;    // LADDER: the library handle
  LadderBw ladder_bw = nullptr;
};

struct Tape {
  bool recording = false;
  std::vector<TapeOp> ops;
  struct Alloc {
    uintptr_t base;
    size_t bytes;
    bool rg;           // its contents depend on the differentiated input
    bool ref;          // referenced by a recorded op: kept alive until the sweep ends
    bool needed;       // its values are read by the sweep (an operand of a recorded product)
    double2* grad;     // gradient buffer of the same size, or null (= zero gradient)
  };
  std::vector<Alloc> allocs;
  std::vector<double2*> deferred;  // frees postponed until the sweep ends
  int find(const void* p) const {
    const uintptr_t q = (uintptr_t)p;
    for (int i = (int)allocs.size() - 1; i >= 0; --i)
      if (q >= allocs[i].base && q < allocs[i].base + allocs[i].bytes) return i;
    return -1;
  }
  bool rg(const void* p) const {
    const int i = find(p);
    return i >= 0 && allocs[i].rg;
  }
  void add(const void* p, size_t bytes, bool rg_) { allocs.push_back({(uintptr_t)p, bytes, rg_, false, false, nullptr}); }
};

// Split-bf16 operand planes kept between contractions.  A device buffer
// registered as frozen promises not to change while registered; the planes
// ctr() splits from it are kept per layout (source, digit maps, conjugation,
// K) and reused.  Scope 0 holds trial-independent tensors until they are
// unregistered (their planes count against `limit` bytes); other scopes hold
// the buffers of one sigma build and are dropped by split_scope_end().
struct SplitCache {
  struct Range { const double2* p; int64_t n; int scope; };
  struct Entry {
    SplitNd key;  // dst unused
    unsigned short* planes;
    int64_t bytes;
    int scope;
  };
  std::vector<Range> frozen;
  std::vector<Entry> entries;
  // buffers of a scope whose elements were never written: only their cached
  // planes may be read (a contraction that would read them otherwise throws)
  std::vector<Range> only;
  int64_t persistent_bytes = 0, limit = 0;
  int next_scope = 1;
};

struct Ctx {
  Tape* tape = nullptr;  // non-null while recording
  hipStream_t stream = nullptr;
  Pool pool;
  int prec = 0;   // arithmetic of ctr() calls
  bool autotune = false;  // time GEMM variants per shape class (see gemm())
  int verbose = 0;        // >= 2: one line per GEMM launch on stderr
  int64_t max_temp = (int64_t)1 << 29;  // largest permuted copy (complex elements) before ctr() splits
  // nonzero: the workspace bytes a sigma build plans its passes and ladder
  // batches for (instead of the handle's mem_budget)
  size_t ws_override = 0;
  SplitCache scache;
  // page-locked host buffer of at least n doubles for the small reports the
  // device iteration sends back (kept and grown across calls, freed with the
  // context)
  double* pinned(size_t n);
  Ctx() = default;
  Ctx(const Ctx&) = delete;
  Ctx& operator=(const Ctx&) = delete;
  ~Ctx();

 private:
  double* pinned_ = nullptr;
  size_t pinned_n_ = 0;
};

// register a trial-independent buffer of n complex elements (scope 0); the
// planes of frozen buffers may use up to `extra_bytes` more
void split_freeze(Ctx& cx, const double2* p, int64_t n, int64_t extra_bytes);
// drop every scope-0 registration and its planes
void split_thaw_all(Ctx& cx);
// open a scope over buffers that stay unchanged until split_scope_end
int split_scope_begin(Ctx& cx, const std::vector<std::pair<const double2*, int64_t>>& bufs);
void split_scope_end(Ctx& cx, int scope);
// record planes [4][n] of the n elements at src, in their memory order, as a
// cache entry of the scope (the cache then owns and frees them); they serve
// every split that reads src in that order without K padding
void split_cache_put(Ctx& cx, int scope, const double2* src, int64_t n, unsigned short* planes);
// the same for a row-major [rows][K] source whose planes are [4][rows][Kp]
void split_cache_put_rows(Ctx& cx, int scope, const double2* src, int64_t rows, int64_t K, int64_t Kp,
                          unsigned short* planes);
// planes of sp (dst unused) owned by the cache: found, or split into a new
// entry of the scope whose frozen range holds the source; nullptr where
// ctr() would not cache them (the caller then splits into its own buffer)
unsigned short* split_planes_cached(Ctx& cx, const SplitNd& sp, int tiled);
// mark the n elements at src (a buffer of the scope) as held only by their
// cached planes; split_planes_only tells whether p points into such a buffer
void split_cache_planes_only(Ctx& cx, int scope, const double2* src, int64_t n);
bool split_planes_only(const Ctx& cx, const double2* p);

// the autotuner's table of tuned shape classes, read from / written to a text
// file (returns the entries read or written, -1 if the file cannot be opened)
int tune_cache_load(const char* path);
int tune_cache_save(const char* path);

// Device scratch of the allocation-free sigma entry point: a file-scope
// __device__ array of kScratchBytes per device.  scratch_address() takes its
// address on the current device (once per device, then cached) and returns
// nullptr if that fails.
constexpr size_t kScratchBytes = (size_t)128 << 20;
void* scratch_address();

// GEMM with automatic split-K when the output has too few tiles to fill the chip
void gemm(Ctx& cx, GemmDesc g);
void gemm_bf16p(Ctx& cx, BfGemm g);

// C[lc] = alpha * sum A[la]^(conj?) B[lb]^(conj?) + beta * C[lc]
void ctr(Ctx& cx, cplx alpha, const Tensor& A, const char* la, bool cA, const Tensor& B, const char* lb,
         bool cB, cplx beta, Tensor& C, const char* lc);
// C[lc] = alpha * op(A[la]) + beta * C[lc]
void perm(Ctx& cx, cplx alpha, const Tensor& A, const char* la, bool cA, cplx beta, Tensor& C, const char* lc);

Tensor tnew(Ctx& cx, std::vector<int64_t> d, bool zero = true);
// an uninitialised complex64 tensor (see Tensor::f32)
Tensor tnew32(Ctx& cx, std::vector<int64_t> d);
// record an op on the tape (no-op unless recording); marks the output as
// requiring a gradient when any input does
void tape_record(Ctx& cx, TapeOp op);
// reverse sweep over cx.tape (adjoint.cpp); the gradient buffers of the
// allocations stay in the tape for the caller to read
void tape_backward(Ctx& cx);
// gradient view of a recorded tensor (allocated zeroed on first use)
Tensor grad_view(Ctx& cx, const Tensor& t);
// drop the tape: deferred frees and gradient buffers go back to the pool
void tape_release(Ctx& cx);
// kernel launches that are recorded on the tape when one is active
void rec_div_d2(Ctx& cx, Tensor& t, const double* eps, int o, int v);
void rec_div_d1(Ctx& cx, Tensor& t, const double* eps, int o, int v);
void rec_antisym_add(Ctx& cx, const Tensor& X, Tensor& out, int64_t k, int64_t d1, int64_t d2, int64_t d3, int64_t d4,
                     int which, cplx alpha);
void rec_herm_add(Ctx& cx, const Tensor& X, Tensor& out, int64_t n);
void rec_m11_add_delta(Ctx& cx, Tensor& M, const Tensor& f, int o, int v, int which);
void rec_pack_doubles(Ctx& cx, int kind, const Tensor& U, double2* S, const double2* Y, int64_t ld, int64_t off,
                      int k, int o, int v, const double* eps, cplx alpha, int accumulate, const int2* po,
                      const int2* pv);
void rec_unpack_doubles(Ctx& cx, int kind, const double2* Y, int64_t ld, int64_t off, int k, int o, int v, Tensor& Ya,
                        const double* eps, const int2* po, const int2* pv);
void rec_pack_ee(Ctx& cx, const Tensor& A0, const Tensor& A1, const Tensor& A2, double2* S, const double2* Y,
                 int64_t ld, int64_t off, int k, int o, int v, const double* eps, const int2* po, const int2* pv);
// view of t with dimension `dim` restricted to [lo, hi)
Tensor tslice(const Tensor& t, int dim, int64_t lo, int64_t hi);
void tfree(Ctx& cx, Tensor& t);

inline cplx C1() { return {1.0, 0.0}; }
inline cplx C0() { return {0.0, 0.0}; }
inline cplx CR(double r) { return {r, 0.0}; }

struct HipError {
  hipError_t e;
  const char* where;
};
inline void hipcheck(hipError_t e, const char* where) {
  if (e != hipSuccess) throw HipError{e, where};
}

}  // namespace adc
