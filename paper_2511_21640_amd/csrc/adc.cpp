// C ABI of the sigma-build library: handle, validation, one-off device work
// (stored integral classes, MP amplitudes, the dense singles block), the
// matrix-free sigma build and the block Davidson solver.
//
// The ISR secular matrix (Section 2.1) is applied term by term.  Every term is
// a complex tensor contraction executed by ctr() (batched MFMA GEMMs plus
// permutes); the particle-particle ladder, whose <ab||cd> integrals are never
// stored, has its own batched path: for a block of virtual indices a the
// Coulomb block W[(a,c)][(b,d)] = sum_Q L^Q_ac L^Q_bd is one GEMM over Q, the
// antisymmetrised rows <ab||cd> = W_ab,cd - W_ab,dc (c<d) are packed, and a
// second GEMM contracts them with the packed trial vectors (Section 2.5,
// on-the-fly generation of the four-external integrals).
#include <hip/hip_runtime.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/adc.h"
#include "internal.h"

using namespace adc;
using zc = std::complex<double>;

namespace {

constexpr bool kSplitBf16Built = true;

struct Status {
  int code;
  const char* msg;
};

struct Inst {
  Ctx* cx = nullptr;      // the lane (stream + pool) this instance runs on
  int kind = 0, o = 0, v = 0, N = 0, k = 0;
  double x = 1.0;
  int64_t n1 = 0, n2 = 0, dim = 0, Po = 0, Pv = 0;
  double* eps = nullptr;  // device
  Tensor Loo, Lov, Lvo, Lvv;
  Tensor oooo, ooov, oovv, ovov, ovvv;
  Tensor ring;            // [k][c][j][b] = <kb||jc>
  Tensor t1;              // [o][o][v][v]
  Tensor ts;              // second-order singles [o][v] (properties: ground-state density)
  Tensor M11x;            // n1 x n1, M11(0..2) + x M11(3)
  Tensor M11b;            // n1 x n1, M11(3) (the x derivative of M11x)
  Tensor W;               // EE: [I][J][i][B] = sum_cd t*_IJcd <cd||iB>
  Tensor W5;              // EE: [J][A][a][B] = sum_kc conj(t[J,k,A,c]) conj(<kB||ac>)
  Tensor W6;              // EE: [I][B][J][i] = sum_kc t*_IkBc conj(<ik||Jc>)
  // EE: the trial-independent factors of the doubles terms that share their
  // output roles, concatenated along the summed index (one GEMM each):
  //   E0[i][a][b][c | k] = conj(<ic||ab>) | t_ikab                (P(ij) terms)
  //   E1[I][J][A][k | c | i] = conj(<IJ||kA>) | t_IJAc | conj(W_IJiA)  (P(ab) terms)
  Tensor E0, E1;
  // the singles-output terms that read the unpacked trial vectors in one
  // layout, summed into one factor per layout (x enters them; see build_sx)
  Tensor X1, X2;
  // EE outside a tape: E0 and t1 with the pair (a<b) packed, E1 with the
  // pair (I<J) packed, for the half-stored accumulators (E0, E1 are freed);
  // E0h carries a third block for the W5 term and E1h's third block also
  // holds the W6 term (see ee_init)
  Tensor E0h, E1h, th;
  // EE outside a tape: X1 antisymmetrised in (b,c) and packed, [o][v][P_v]
  // (X1 itself is then dropped)
  Tensor X1h;
  // ... X2 antisymmetrised in (j,k) and packed [P_o][o][v], t pair-packed in
  // (I,J) [P_o][v][v], and the split-bf16 planes of the ring matrix with rows
  // (j,b) and columns (k,c) (ringKp = o*v padded to 32)
  Tensor X2h, tIJ;
  Tensor oooo_p;  // <kl||ij> with the pair (k<l) packed, [P_o][o][o]
  Tensor oooo_pp; // <kl||ij> with both pairs packed, [P_o(kl)][P_o(ij)]
  Tensor ooov_p;  // <kl||ja> with the pair (k<l) packed, [P_o][o][v]
  Tensor tpp;     // t1 with both pairs packed, [P_o][P_v]
  // the Hermitian-half <ab||cd> assembly as grouped GEMMs over small
  // a-blocks (exact ranges up to a block), planned for one workspace size
  struct LadPlan {
    int64_t wbudget = -1;  // bytes of W the chunks were planned for
    struct Chunk {
      int a_begin = 0, a_end = 0, prob0 = 0, nprob = 0;
      int64_t pbase = 0, npairs = 0, gtiles = 0;
    };
    std::vector<Chunk> chunks;
    std::vector<GroupProb> probs;  // output offsets relative to the chunk's W
    std::vector<LadBlk> blk;       // per a
    int64_t wmax = 0;              // complex64 elements of the largest chunk's W
    GroupProb* dprobs = nullptr;   // device copies (handle allocations)
    LadBlk* dblk = nullptr;
  } lplan;
  unsigned short* ringq = nullptr;
  int64_t ringKp = 0;
  int2* pair_o = nullptr;
  int2* pair_v = nullptr;
  double* diag = nullptr; // device zeroth-order diagonal [dim]
  // split-bf16 planes [4][rows][K padded to 32] of L_vv, built on first use
  unsigned short* Lq = nullptr;     // rows (a,c) of L_vv, K = Q
  int64_t Kq = 0;
  std::vector<double> m11diag;  // host, real part of diag(M11x)
  // captured sigma builds (Davidson of small instances): one per (rows, precision)
  struct Graph {
    int rows = 0, prec = 0;
    double2* Yin = nullptr;   // staging input  [rows][dim]
    double2* Sout = nullptr;  // staging output [rows][dim]
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    std::vector<double2*> held;  // workspace blocks reserved for the graph
  };
  std::vector<Graph> graphs;
  bool graphs_off = false;  // a capture failed: sigma builds run eagerly
  // allocation-free sigma builds: the smallest row count per precision that
  // did not fit the scratch (0 = none seen)
  int noalloc_too_big[3] = {0, 0, 0};
  // reverse mode: the recorded one-off part of the first adc_sigma_backward
  // call, kept for the later calls (see BwCache)
  std::shared_ptr<struct BwCache> bw;
};

// The tape of the one-off work (integrals, amplitudes, intermediates) that
// adc_sigma_backward recomputes from L, and the instance copy J it recorded
// into: the first call records it, later calls record only the sigma build
// on top and cut the tape back to this length after their sweep.
struct BwCache {
  Tape T;
  Inst J;
  size_t n_ops = 0, n_allocs = 0, n_deferred = 0;
};

}  // namespace

// Instances are spread over lanes: lane 0 is the handle's stream, further
// lanes have their own non-blocking streams (default priority) and pools, so
// that independent instances overlap on the device.  Each instance lives on
// one lane; its tensors come from that lane's pool.
struct adc_handle {
  Ctx cx;                                   // lane 0
  std::vector<std::unique_ptr<Ctx>> extra;  // lanes 1 ..
  adc_options opt{};
  bool own_stream = false;
  double init_ms = 0.0;
  std::vector<Inst> inst;
  std::vector<std::vector<int>> lane_inst;  // instances of each lane, most expensive first
  std::vector<void*> raw;                   // plain device allocations
  std::mutex mu;                            // guards raw
  int device = 0;
  std::string tune_path;                    // autotuner cache file, if any
  void* scratch = nullptr;                  // device address of the allocation-free entry point's scratch
  Ctx& lane(int i) { return i == 0 ? cx : *extra[(size_t)i - 1]; }
  int n_lanes() const { return 1 + (int)extra.size(); }
};

namespace {

void* dmalloc(adc_handle* h, size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) {
    (void)hipGetLastError();
    throw HipError{hipErrorOutOfMemory, "hipMalloc"};
  }
  std::lock_guard<std::mutex> lock(h->mu);
  h->raw.push_back(p);
  return p;
}

Tensor tensor_view(double2* p, std::vector<int64_t> d, std::vector<int64_t> st) {
  Tensor t;
  t.p = p;
  t.d = std::move(d);
  t.st = std::move(st);
  return t;
}

int64_t npair(int64_t n) { return n * (n - 1) / 2; }

std::vector<int2> pair_table(int n) {
  std::vector<int2> t;
  for (int p = 0; p < n; ++p)
    for (int q = p + 1; q < n; ++q) t.push_back(make_int2(p, q));
  return t;
}

int64_t pad32(int64_t n) { return (n + 31) / 32 * 32; }

unsigned short* planes_alloc(Ctx& cx, int64_t rows, int64_t Kp) {
  return (unsigned short*)cx.pool.get((rows * Kp * 4 + 7) / 8);
}

void ensure_planes(adc_handle* h, Inst& I) {
  Ctx& cx = *I.cx;
  const int64_t v = I.v;
  if (!I.Lq) {
    I.Kq = pad32(I.N);
    I.Lq = (unsigned short*)dmalloc(h, (size_t)v * v * I.Kq * 8);
    launch_split_planes(I.Lvv.p, v * v, I.N, 1, v * v, 0, I.Lq, I.Kq, cx.stream);
  }
}

// ----------------------------------------------------------------------------
// particle-particle ladder:  S[z][offS + ij*Pv + ab] += alpha * sum_{c<d} <ab||cd> Y[z][offY + ij*Pv + cd]
// for rows ij in [0, nrow), z in [0, k).  L_vv is [Q][v][v].
// ----------------------------------------------------------------------------
void ladder_backward(Ctx& cx, const TapeOp& op, const double2* gS, double2* gY);

// Blocks of the half assembly: a block [a0, a0 + nb) computes
// W[(a-a0)*m + c-a0][(b-a0-1)*m + d-a0] = sum_Q L_ac L_bd, m = v - a0, for
// c, d >= a0 and b > a0, a superset of what its pairs need (c, d >= a,
// b > a).  nb is chosen per block for the least padded 128 x 128 tile work
// per needed element; the blocks are one grouped GEMM per chunk of at most
// wbytes of W.
void ladder_plan(adc_handle* h, Inst& I, int64_t wbytes, int64_t Kq) {
  auto& P = I.lplan;
  if (P.wbudget == wbytes && P.dprobs) return;
  P = Inst::LadPlan{};
  const int64_t v = I.v;
  const int64_t T = 128;  // tile of the grouped GEMM (tile code 9)
  auto tiles = [&](int64_t M, int64_t N) { return ((M + T - 1) / T) * ((N + T - 1) / T); };
  P.blk.assign((size_t)v, LadBlk{0, 0, 0});
  Inst::LadPlan::Chunk ch;
  int64_t wfill = 0;
  auto close_chunk = [&](int a_end) {
    ch.a_end = a_end;
    ch.nprob = (int)P.probs.size() - ch.prob0;
    ch.pbase = (int64_t)ch.a_begin * (2 * v - ch.a_begin - 1) / 2;
    ch.npairs = (int64_t)a_end * (2 * v - a_end - 1) / 2 - ch.pbase;
    P.wmax = std::max(P.wmax, wfill);
    P.chunks.push_back(ch);
  };
  ch.a_begin = 0;
  ch.prob0 = 0;
  for (int64_t a0 = 0; a0 < v - 1;) {
    const int64_t m = v - a0;
    int64_t best_nb = 1;
    double best = -1.0;
    for (int64_t nb = 1; nb <= std::min<int64_t>(32, v - 1 - a0); ++nb) {
      double need = 0.0;
      for (int64_t a = a0; a < a0 + nb; ++a) need += (double)(v - a) * (double)(v - a - 1) * (double)(v - a);
      const double padded = (double)tiles(nb * m, (v - a0 - 1) * m) * (double)(T * T);
      const double r = padded / need;
      if (best < 0.0 || r < best * 0.99) {
        best = r;
        best_nb = nb;
      }
    }
    const int64_t M = best_nb * m, N = (v - a0 - 1) * m;
    if (wfill > 0 && (wfill + M * N) * 8 > wbytes) {
      close_chunk((int)a0);
      ch = Inst::LadPlan::Chunk{};
      ch.a_begin = (int)a0;
      ch.prob0 = (int)P.probs.size();
      wfill = 0;
    }
    GroupProb g{};
    g.tile0 = ch.gtiles;
    g.M = M;
    g.N = N;
    g.arow = a0 * v + a0;
    g.brow = (a0 + 1) * v + a0;
    g.amd = m;
    g.bmd = m;
    g.coff = wfill;
    g.ldc = N;
    P.probs.push_back(g);
    for (int64_t a = a0; a < a0 + best_nb; ++a) P.blk[(size_t)a] = LadBlk{a0, wfill, N};
    ch.gtiles += tiles(M, N);
    wfill += M * N;
    a0 += best_nb;
  }
  close_chunk((int)(v - 1));
  (void)Kq;
  P.dprobs = (GroupProb*)dmalloc(h, sizeof(GroupProb) * P.probs.size());
  P.dblk = (LadBlk*)dmalloc(h, sizeof(LadBlk) * P.blk.size());
  // on the instance's own stream: a copy on the legacy default stream would
  // wait on (and break) another lane's stream capture
  Ctx& cx = *I.cx;
  hipcheck(hipMemcpyAsync(P.dprobs, P.probs.data(), sizeof(GroupProb) * P.probs.size(), hipMemcpyHostToDevice,
                          cx.stream), "plan");
  hipcheck(hipMemcpyAsync(P.dblk, P.blk.data(), sizeof(LadBlk) * P.blk.size(), hipMemcpyHostToDevice, cx.stream),
           "plan");
  hipcheck(hipStreamSynchronize(cx.stream), "plan sync");
  P.wbudget = wbytes;
}

void ladder(adc_handle* h, Inst& I, const double2* Y, int64_t ldY, int64_t offY, double2* S, int64_t ldS,
            int64_t offS, int64_t nrow, int k, cplx alpha, int prec) {
  Ctx& cx = *I.cx;
  if (cx.tape && cx.tape->recording) {
    TapeOp op{};
    op.kind = TapeOp::LADDER;
    op.A.p = const_cast<double2*>(Y);
    op.C.p = S;
    op.alpha = alpha;
    op.n[0] = ldY; op.n[1] = offY; op.n[2] = ldS; op.n[3] = offS; op.n[4] = nrow; op.n[5] = k;
    op.inst = &I;
    op.owner = h;
    op.ladder_bw = ladder_backward;
    op.prec = prec;
    tape_record(cx, op);
  }
  const int v = I.v;
  const int64_t Pv = I.Pv, N = I.N;
  if (Pv == 0 || nrow == 0 || k == 0) return;
  const size_t budget = cx.ws_override ? cx.ws_override / 4
                                       : (h->opt.mem_budget ? h->opt.mem_budget : (size_t)4 << 30);
  // W block: nb*v rows x (v-b0)*v cols, at most the workspace budget
  const int64_t per_a = (int64_t)v * v * v;
  int nb = (int)std::max<int64_t>(1, (int64_t)(budget / sizeof(double2)) / std::max<int64_t>(1, per_a));
  // a block of nb values of a assembles columns b > a0 for every a in it, so
  // the triangle b <= a inside the block (a fraction ~nb/v of the work) is
  // wasted: keep blocks near v/8 when the GEMMs stay large enough
  nb = std::min(nb, std::max(16, (v + 7) / 8));
  nb = std::min(nb, v - 1);
  double2* Wbuf = nullptr;  // per-block assembly output (not needed by the grouped assembly)
  // the k vectors' rows are stacked into one [k*nrow][Pv] operand (M = k*nrow);
  // split-bf16 splits them straight from Y and writes S through an output
  // map, the other precisions stage them in Yc, Sc
  const int64_t R = (int64_t)k * nrow;
  const bool bf = prec == ADC_SPLIT_BF16;
  const int64_t Kq = pad32(N);  // K of the L_vv planes
  double2* Yc = bf ? nullptr : cx.pool.get(R * Pv);
  double2* Sc = bf ? nullptr : cx.pool.get(R * Pv);
  if (!bf) {
    int64_t od[2] = {k, nrow * Pv}, is[2] = {ldY, 1}, os[2] = {nrow * Pv, 1};
    launch_permute(2, od, is, os, Y + offY, Yc, C1(), C0(), 0, cx.stream);
  }
  // packed <ab||cd> rows of several a-blocks are collected (up to a quarter of
  // the workspace) and contracted with the trial vectors in one GEMM, so that
  // the contraction runs on large N even where the a-blocks are small; in
  // split-bf16 without an explicit budget, all rows are taken as one group
  // whenever their planes fit 16 GiB, which enables the Hermitian half below
  const int64_t Kv = pad32(Pv);
  const int64_t row_bytes = bf ? Kv * 8 : Pv * (int64_t)sizeof(double2);
  const int64_t max_np = (int64_t)nb * (v - 1);
  const bool one_group = bf && !cx.ws_override && !h->opt.mem_budget && Pv * row_bytes <= ((int64_t)16 << 30);
  const size_t gbudget = one_group ? (size_t)(Pv * row_bytes) : budget / 4;
  const int64_t grp = std::min<int64_t>(Pv, std::max<int64_t>(max_np, (int64_t)gbudget / row_bytes));
  unsigned short* Yp = nullptr;
  unsigned short* Vp = nullptr;
  double2* Vbuf = nullptr;
  bool own_yp = false;
  // split-bf16 planes of L_vv: kept in the instance after their first use,
  // or, inside an allocation-free call that finds none, split for this call
  const unsigned short* Lq = nullptr;
  unsigned short* Lq_tmp = nullptr;
  if (bf) {
    if (!I.Lq && cx.pool.in_arena()) {
      Lq_tmp = planes_alloc(cx, (int64_t)v * v, pad32(N));
      launch_split_planes(I.Lvv.p, (int64_t)v * v, N, 1, (int64_t)v * v, 0, Lq_tmp, pad32(N), cx.stream);
      Lq = Lq_tmp;
    } else {
      ensure_planes(h, I);
      Lq = I.Lq;
    }
    Vp = planes_alloc(cx, grp, Kv);
    SplitNd sp{};
    sp.src = Y + offY; sp.rows = R; sp.K = Pv; sp.Kp = Kv; sp.conj = 0;
    sp.nm = 2; sp.md[0] = k; sp.md[1] = nrow; sp.ms[0] = ldY; sp.ms[1] = Pv;
    sp.nk = 1; sp.kd[0] = Pv; sp.ks[0] = 1;
    // inside a sigma build the trial rows' planes come from the build's
    // cache, where a contraction reading the packed doubles in this layout
    // may already have put them
    Yp = split_planes_cached(cx, sp, 0);
    if (!Yp) {
      Yp = planes_alloc(cx, R, Kv);
      own_yp = true;
      sp.dst = Yp;
      launch_split_nd(sp, 0, cx.stream);
    }
  } else {
    Vbuf = cx.pool.get(grp * Pv);
  }
  int64_t gbase = 0, gfill = 0;  // first pair of the collected rows, their number
  auto contract = [&]() {
    if (gfill == 0) return;
    if (bf) {
      BfGemm c{};
      c.M = R; c.N = gfill; c.Kp = Kv;
      c.A = Yp; c.lda = R;
      c.B = Vp; c.ldb = grp;
      // S[z][offS + r*Pv + gbase + q] += alpha * (...)
      c.C = S + offS + gbase; c.scn = 1;
      c.om.nm = 2; c.om.md[0] = k; c.om.md[1] = nrow; c.om.ms[0] = ldS; c.om.ms[1] = Pv;
      c.alpha = alpha; c.beta = C1(); c.tag = 2;
      gemm_bf16p(cx, c);
    } else {
      // Sc[r][gbase + q] = sum_cd Yc[r][cd] V[q][cd]
      GemmDesc c{};
      c.M = R; c.N = gfill; c.K = Pv; c.batch = 1;
      c.A = Yc; c.sam = Pv; c.sak = 1; c.sab = 0;
      c.B = Vbuf; c.sbk = 1; c.sbn = Pv; c.sbb = 0;
      c.C = Sc + gbase; c.scm = Pv; c.scn = 1; c.scb = 0;
      c.alpha = C1(); c.beta = C0();
      c.tag = 2;
      const int sp = cx.prec;
      cx.prec = prec;
      gemm(cx, c);
      cx.prec = sp;
    }
    gbase += gfill;
    gfill = 0;
  };
  // The packed <ab||cd> matrix is Hermitian (L^Q Hermitian: <cd||ab> =
  // conj <ab||cd>).  When all its rows fit one group, only the part cd >= ab
  // is assembled, which needs (ac|bd) for c, d >= a0 alone (about half of
  // the assembly work), and the rest is mirrored on the split planes.
  const bool half = bf && grp >= Pv;
  // the grouped exact-range assembly (planned once per instance and W size;
  // not inside an allocation-free call, which plans nothing)
  if (half && !cx.pool.in_arena() && !capturing(cx.stream)) ladder_plan(h, I, (int64_t)budget, Kq);
  if (half && I.lplan.dprobs && I.lplan.wbudget == (int64_t)budget) {
    const auto& P = I.lplan;
    float2* Wall = (float2*)cx.pool.get((P.wmax + 1) / 2);
    for (const auto& ch : P.chunks) {
      BfGemm g{};
      g.M = 1; g.N = 1; g.Kp = Kq;
      g.A = Lq; g.lda = (int64_t)v * v; g.ams = v;
      g.B = Lq; g.ldb = (int64_t)v * v; g.bms = v;
      g.C = (double2*)Wall; g.scn = 1; g.c32 = 1;
      g.alpha = C1(); g.beta = C0(); g.tag = 1; g.tile = 9;
      g.probs = P.dprobs + ch.prob0; g.nprob = ch.nprob; g.gtiles = ch.gtiles;
      g.nsplit = 1; g.kchunk = Kq;
      launch_bf16p(g, cx.stream);
      launch_ladder_pack_planes_grouped(Wall, P.dblk, v, Vp, grp, ch.pbase, ch.npairs, I.pair_v, Kv, cx.stream);
    }
    cx.pool.put((double2*)Wall);
    gfill = Pv;
  }
  // Several row groups in split-bf16 (the packed rows do not fit one
  // group): each group still assembles only its upper part (pairs cd >= ab);
  // the group's diagonal block is mirrored, its rows are contracted over all
  // columns (the columns of earlier groups zeroed), and the conjugate
  // transpose of its rows right of the block is contracted into the later
  // columns of S, which the later groups' rows would otherwise need.
  const bool mg = bf && !half;
  auto flush_mg = [&]() {
    if (gfill == 0) return;
    const int64_t g0 = gbase, n = gfill, g1 = g0 + n;
    launch_planes_zero_cols(Vp, grp, n, g0, Kv, cx.stream);
    launch_ladder_mirror_block(Vp, grp, n, Kv, g0, cx.stream);
    contract();
    if (g1 < Pv) {
      const int64_t g0a = g0 / 32 * 32, Kg = pad32(g1 - g0a), nc = Pv - g1;
      unsigned short* T = planes_alloc(cx, nc, Kg);
      launch_ladder_transpose_planes(Vp, grp, n, g1, nc, Kv, T, Kg, g0 - g0a, cx.stream);
      unsigned short* Yw = planes_alloc(cx, R, Kg);
      launch_planes_copy_cols(Yp, R, Kv, g0a, Yw, Kg, cx.stream);
      // S[z][offS + r*Pv + q] += alpha sum_{ab in group} Y[z][r][ab] conj <ab||q>, q >= g1
      BfGemm c{};
      c.M = R; c.N = nc; c.Kp = Kg;
      c.A = Yw; c.lda = R;
      c.B = T; c.ldb = nc;
      c.C = S + offS + g1; c.scn = 1;
      c.om.nm = 2; c.om.md[0] = k; c.om.md[1] = nrow; c.om.ms[0] = ldS; c.om.ms[1] = Pv;
      c.alpha = alpha; c.beta = C1(); c.tag = 2;
      gemm_bf16p(cx, c);
      cx.pool.put((double2*)Yw);
      cx.pool.put((double2*)T);
    }
  };
  if (!(half && gfill == Pv)) Wbuf = cx.pool.get((int64_t)nb * v * v * v);
  for (int a0 = (half && gfill == Pv) ? v - 1 : 0; a0 < v - 1;) {
    int nbc = nb;
    if (half || mg) {
      // blocks grow as the ranges of c, d shrink, keeping W near its size
      const int64_t m = v - a0;
      int64_t want = ((int64_t)nb * v * v * v) / std::max<int64_t>(1, m * m * (m - 1));
      want = std::min<int64_t>(want, std::max<int64_t>(nb, m / 4));
      nbc = (int)std::max<int64_t>(nb, want);
      // a block's rows fit one group
      while (mg && nbc > 1 &&
             (int64_t)std::min(v - 1, a0 + nbc) * (2 * v - std::min(v - 1, a0 + nbc) - 1) / 2 -
                     (int64_t)a0 * (2 * v - a0 - 1) / 2 > grp)
        --nbc;
    }
    const int a1 = std::min(v - 1, a0 + nbc);
    const int b0 = a0 + 1;
    const int64_t pbase = (int64_t)a0 * (2 * v - a0 - 1) / 2;
    const int64_t pend = (int64_t)a1 * (2 * v - a1 - 1) / 2;
    const int64_t np = pend - pbase;
    if (mg && gfill + np > grp) flush_mg();
    if (half || mg) {
      // W[(a-a0)*m + c-a0][(b-b0)*m + d-a0] = sum_Q L_ac L_bd, c, d >= a0
      const int64_t m = v - a0;
      const int64_t Mw = (int64_t)(a1 - a0) * m, Nw = (int64_t)(v - b0) * m;
      BfGemm g{};
      g.M = Mw; g.N = Nw; g.Kp = Kq;
      g.A = Lq + ((int64_t)a0 * v + a0) * Kq; g.lda = (int64_t)v * v; g.amd = m; g.ams = v;
      g.B = Lq + ((int64_t)b0 * v + a0) * Kq; g.ldb = (int64_t)v * v; g.bmd = m; g.bms = v;
      // W is stored as complex64: the GEMM accumulates in FP32 and the pack
      // rounds <ab||cd> to FP32 before splitting it
      g.C = Wbuf; g.scm = Nw; g.scn = 1; g.c32 = 1;
      g.alpha = C1(); g.beta = C0(); g.tag = 1;
      gemm_bf16p(cx, g);
      launch_ladder_pack_planes_upper(Wbuf, 1, Nw, a0, b0, v, Vp, grp, pbase, np, I.pair_v, Kv, cx.stream,
                                      mg ? gbase : 0);
      gfill += np;
      a0 = a1;
      continue;
    }
    if (gfill + np > grp) contract();
    // W[(a-a0)*v + c][(b-b0)*v + d] = sum_Q L_ac L_bd
    const int64_t Mw = (int64_t)(a1 - a0) * v, Nw = (int64_t)(v - b0) * v;
    if (bf) {
      BfGemm g{};
      g.M = Mw; g.N = Nw; g.Kp = Kq;
      g.A = Lq + (int64_t)a0 * v * Kq; g.lda = (int64_t)v * v;
      g.B = Lq + (int64_t)b0 * v * Kq; g.ldb = (int64_t)v * v;
      g.C = Wbuf; g.scm = Nw; g.scn = 1;
      g.alpha = C1(); g.beta = C0(); g.tag = 1;
      gemm_bf16p(cx, g);
      launch_ladder_pack_planes(Wbuf, Nw, a0, b0, v, Vp, grp, gfill, pbase, np, I.pair_v, Kv, cx.stream);
    } else {
      GemmDesc g{};
      g.M = Mw; g.N = Nw; g.K = N; g.batch = 1;
      g.A = I.Lvv.p + (int64_t)a0 * v; g.sam = 1; g.sak = (int64_t)v * v; g.sab = 0;
      g.B = I.Lvv.p + (int64_t)b0 * v; g.sbn = 1; g.sbk = (int64_t)v * v; g.sbb = 0;
      g.C = Wbuf; g.scm = Nw; g.scn = 1; g.scb = 0;
      g.alpha = C1(); g.beta = C0();
      g.tag = 1;
      const int sp = cx.prec;
      cx.prec = prec;
      gemm(cx, g);
      cx.prec = sp;
      launch_ladder_pack(Wbuf, Nw, a0, b0, v, Vbuf + gfill * Pv, pbase, np, I.pair_v, cx.stream);
    }
    gfill += np;
    a0 = a1;
  }
  if (mg) {
    flush_mg();
  } else {
    if (half) launch_ladder_mirror_planes(Vp, grp, Pv, Kv, cx.stream);
    contract();
  }
  if (Lq_tmp) cx.pool.put((double2*)Lq_tmp);
  if (own_yp) cx.pool.put((double2*)Yp);
  if (Vp) cx.pool.put((double2*)Vp);
  if (Vbuf) cx.pool.put(Vbuf);
  if (!bf) {
    int64_t od[2] = {k, nrow * Pv}, is[2] = {nrow * Pv, 1}, os[2] = {ldS, 1};
    launch_permute(2, od, is, os, Sc, S + offS, alpha, C1(), 0, cx.stream);
    cx.pool.put(Yc);
    cx.pool.put(Sc);
  }
  if (Wbuf) cx.pool.put(Wbuf);
}

// the unpacked trial vectors of one sigma build stay unchanged until the
// build ends: their split-bf16 planes are shared by the contractions that
// read them in the same layout
struct SplitScope {
  Ctx& cx;
  int id;
  SplitScope(Ctx& c, std::vector<std::pair<const double2*, int64_t>> bufs) : cx(c), id(split_scope_begin(c, bufs)) {}
  ~SplitScope() { split_scope_end(cx, id); }
};

// copy rows [k][n] with row stride ld (offset off) into a contiguous tensor, or back
void rows_in(Ctx& cx, const double2* src, int64_t ld, int64_t off, Tensor& dst, int k, int64_t n) {
  int64_t od[2] = {k, n}, is[2] = {ld, 1}, os[2] = {n, 1};
  launch_permute(2, od, is, os, src + off, dst.p, C1(), C0(), 0, cx.stream);
}
void rows_out(Ctx& cx, const Tensor& src, double2* dst, int64_t ld, int64_t off, int k, int64_t n, cplx beta) {
  Tensor s = tensor_view(src.p, {k, n}, {n, 1});
  Tensor d = tensor_view(dst + off, {k, n}, {ld, 1});
  perm(cx, C1(), s, "zp", false, beta, d, "zp");
}

// ============================================================================
// one-off work shared by the three kinds
// ============================================================================
// Stored integral classes (eq. 43): <pq||rs> = (pr|qs) - (ps|qr), the MP
// amplitudes t(1), t(2) and t_s(2), and the pieces of the singles block.
struct Pre {
  Tensor Lt, Ht, t2, ts;       // ladder / hole ladder of t(1), t(2), singles t(2)
};

void init_integrals(adc_handle* h, Inst& I) {
  Ctx& cx = *I.cx;
  const int o = I.o, v = I.v;
  I.oooo = tnew(cx, {o, o, o, o}, false);
  ctr(cx, C1(), I.Loo, "Qik", false, I.Loo, "Qjl", false, C0(), I.oooo, "ijkl");
  ctr(cx, CR(-1), I.Loo, "Qil", false, I.Loo, "Qjk", false, C1(), I.oooo, "ijkl");
  I.ooov = tnew(cx, {o, o, o, v}, false);
  ctr(cx, C1(), I.Loo, "Qik", false, I.Lov, "Qja", false, C0(), I.ooov, "ijka");
  ctr(cx, CR(-1), I.Lov, "Qia", false, I.Loo, "Qjk", false, C1(), I.ooov, "ijka");
  I.oovv = tnew(cx, {o, o, v, v}, false);
  ctr(cx, C1(), I.Lov, "Qia", false, I.Lov, "Qjb", false, C0(), I.oovv, "ijab");
  ctr(cx, CR(-1), I.Lov, "Qib", false, I.Lov, "Qja", false, C1(), I.oovv, "ijab");
  I.ovov = tnew(cx, {o, v, o, v}, false);
  ctr(cx, C1(), I.Loo, "Qij", false, I.Lvv, "Qab", false, C0(), I.ovov, "iajb");
  ctr(cx, CR(-1), I.Lov, "Qib", false, I.Lvo, "Qaj", false, C1(), I.ovov, "iajb");
  I.ovvv = tnew(cx, {o, v, v, v}, false);
  ctr(cx, C1(), I.Lov, "Qib", false, I.Lvv, "Qac", false, C0(), I.ovvv, "iabc");
  ctr(cx, CR(-1), I.Lov, "Qic", false, I.Lvv, "Qab", false, C1(), I.ovvv, "iabc");
  // ring matrix [k][c][j][b] = <kb||jc>  (Hermitian as an (ov) x (ov) matrix)
  I.ring = tnew(cx, {o, v, o, v}, false);
  perm(cx, C1(), I.ovov, "kbjc", false, C0(), I.ring, "kcjb");
}

void init_amplitudes(adc_handle* h, Inst& I, Pre& P) {
  Ctx& cx = *I.cx;
  const int o = I.o, v = I.v;
  // first-order doubles t_ij^ab = <ab||ij>/D = conj(<ij||ab>)/D
  Tensor& t = I.t1;
  t = tnew(cx, {o, o, v, v}, false);
  perm(cx, C1(), I.oovv, "ijab", true, C0(), t, "ijab");
  rec_div_d2(cx, t, I.eps, o, v);
  // second-order doubles: (particle ladder + hole ladder - ring) / D
  const int64_t Po = I.Po, Pv = I.Pv;
  P.Lt = tnew(cx, {o, o, v, v}, true);
  if (Po > 0) {
    Tensor tpk = tnew(cx, {Po * Pv}, false);
    rec_pack_doubles(cx, 0, t, tpk.p, nullptr, Po * Pv, 0, 1, o, v, I.eps, C1(), 0, I.pair_o, I.pair_v);
    Tensor Ltp = tnew(cx, {Po * Pv});
    ladder(h, I, tpk.p, Po * Pv, 0, Ltp.p, Po * Pv, 0, Po, 1, C1(), 0);
    rec_unpack_doubles(cx, 0, Ltp.p, Po * Pv, 0, 1, o, v, P.Lt, I.eps, I.pair_o, I.pair_v);
    tfree(cx, Ltp);
    tfree(cx, tpk);
  }
  P.Ht = tnew(cx, {o, o, v, v}, false);
  ctr(cx, CR(0.5), I.oooo, "klij", false, t, "klab", false, C0(), P.Ht, "ijab");
  P.t2 = tnew(cx, {o, o, v, v}, false);
  perm(cx, C1(), P.Lt, "ijab", false, C0(), P.t2, "ijab");
  perm(cx, C1(), P.Ht, "ijab", false, C1(), P.t2, "ijab");
  {
    Tensor R = tnew(cx, {o, v, o, v}, false);
    ctr(cx, C1(), t, "ikac", false, I.ovov, "kbjc", false, C0(), R, "iajb");
    Tensor Rr = tnew(cx, {o, o, v, v}, false);
    perm(cx, C1(), R, "iajb", false, C0(), Rr, "ijab");
    rec_antisym_add(cx, Rr, P.t2, 1, o, o, v, v, 2, CR(-1));
    tfree(cx, R);
    tfree(cx, Rr);
  }
  rec_div_d2(cx, P.t2, I.eps, o, v);
  // second-order singles
  P.ts = tnew(cx, {o, v});
  ctr(cx, CR(-0.5), I.ovvv, "jabc", false, t, "ijbc", false, C0(), P.ts, "ia");
  ctr(cx, CR(-0.5), I.ooov, "jkib", false, t, "jkab", false, C1(), P.ts, "ia");
  rec_div_d1(cx, P.ts, I.eps, o, v);
}

// Pieces of M11 that carry delta_aA (f_o, occupied x occupied) and delta_iI
// (f_v, virtual x virtual), split by order: second order (f2) and third order
// (f3).  The IP singles block is f_o, the EA singles block f_v, and the EE
// singles block contains both (see ee_m11).
void m11_fo(adc_handle* h, Inst& I, Pre& P, Tensor& f2, Tensor& f3) {
  Ctx& cx = *I.cx;
  const int o = I.o;
  const Tensor& t = I.t1;
  f2 = tnew(cx, {o, o});
  f3 = tnew(cx, {o, o});
  // -1/4 t(ikcd) <Ik||cd>  (order 2 with t(1), order 3 with t(2))
  ctr(cx, CR(-0.25), t, "ikcd", false, I.oovv, "Ikcd", false, C0(), f2, "iI");
  ctr(cx, CR(-0.25), P.t2, "ikcd", false, I.oovv, "Ikcd", false, C1(), f3, "iI");
  // -ts(kc) <Ik||ic>
  ctr(cx, CR(-1), P.ts, "kc", false, I.ooov, "Ikic", false, C1(), f3, "iI");
  // -1/2 t*(Ikcd) Q(cikd), Q = -<lc||ie> t(klde)
  {
    Tensor Q = tnew(cx, {I.v, o, o, I.v}, false);
    ctr(cx, CR(-1), I.ovov, "lcie", false, t, "klde", false, C0(), Q, "cikd");
    ctr(cx, CR(-0.5), t, "Ikcd", true, Q, "cikd", false, C1(), f3, "iI");
    tfree(cx, Q);
  }
  // -1/4 t*(Ikcd) Ht(ikcd)
  ctr(cx, CR(-0.25), t, "Ikcd", true, P.Ht, "ikcd", false, C1(), f3, "iI");
  // +1/4 <Ic||ie> rv_ce ; -1/4 <Im||ik> ro_km
  Tensor rv = tnew(cx, {I.v, I.v}, false), ro = tnew(cx, {o, o}, false);
  ctr(cx, C1(), t, "klcd", true, t, "klde", false, C0(), rv, "ce");
  ctr(cx, C1(), t, "klcd", true, t, "lmcd", false, C0(), ro, "km");
  ctr(cx, CR(0.25), I.ovov, "Icie", false, rv, "ce", false, C1(), f3, "iI");
  ctr(cx, CR(-0.25), I.oooo, "Imik", false, ro, "km", false, C1(), f3, "iI");
  tfree(cx, rv);
  tfree(cx, ro);
}

void m11_fv(adc_handle* h, Inst& I, Pre& P, Tensor& f2, Tensor& f3) {
  Ctx& cx = *I.cx;
  const int o = I.o, v = I.v, N = I.N;
  const Tensor& t = I.t1;
  f2 = tnew(cx, {v, v});
  f3 = tnew(cx, {v, v});
  // -1/4 t(klac) <kl||Ac>
  ctr(cx, CR(-0.25), t, "klac", false, I.oovv, "klAc", false, C0(), f2, "aA");
  ctr(cx, CR(-0.25), P.t2, "klac", false, I.oovv, "klAc", false, C1(), f3, "aA");
  // +ts(kc) <ak||Ac>, <ak||Ac> = -ovvv[k,a,A,c]
  ctr(cx, CR(-1), P.ts, "kc", false, I.ovvv, "kaAc", false, C1(), f3, "aA");
  // -1/4 t*(klAc) Lt(klac)
  ctr(cx, CR(-0.25), t, "klAc", true, P.Lt, "klac", false, C1(), f3, "aA");
  // -1/2 t*(klAc) P2(aklc), P2 = -<ma||kd> t(lmcd)
  {
    Tensor P2 = tnew(cx, {v, o, o, v}, false);
    ctr(cx, CR(-1), I.ovov, "makd", false, t, "lmcd", false, C0(), P2, "aklc");
    ctr(cx, CR(-0.5), t, "klAc", true, P2, "aklc", false, C1(), f3, "aA");
    tfree(cx, P2);
  }
  // -1/4 rv_ce <ac||Ae>,  <ac||Ae> = (aA|ce) - (ae|cA), through the Cholesky vectors
  Tensor rv = tnew(cx, {v, v}, false), ro = tnew(cx, {o, o}, false);
  ctr(cx, C1(), t, "klcd", true, t, "klde", false, C0(), rv, "ce");
  ctr(cx, C1(), t, "klcd", true, t, "lmcd", false, C0(), ro, "km");
  {
    Tensor s1 = tnew(cx, {N, 1}, false);
    Tensor rv1 = tensor_view(rv.p, {v, v, 1}, {});
    ctr(cx, C1(), I.Lvv, "Qce", false, rv1, "cex", false, C0(), s1, "Qx");
    Tensor f31 = tensor_view(f3.p, {v, v, 1}, {});
    ctr(cx, CR(-0.25), I.Lvv, "QaA", false, s1, "Qx", false, C1(), f31, "aAx");
    Tensor Z = tnew(cx, {N, v, v}, false);
    ctr(cx, C1(), rv, "ce", false, I.Lvv, "QcA", false, C0(), Z, "QeA");
    ctr(cx, CR(0.25), I.Lvv, "Qae", false, Z, "QeA", false, C1(), f3, "aA");
    tfree(cx, s1);
    tfree(cx, Z);
  }
  // +1/4 <am||Ak> ro_km,  <am||Ak> = ovov[m,a,k,A]
  ctr(cx, CR(0.25), I.ovov, "makA", false, ro, "km", false, C1(), f3, "aA");
  tfree(cx, rv);
  tfree(cx, ro);
}

// dense n x n block: herm(f) + diag(d) for IP / EA
void small_m11(adc_handle* h, Inst& I, Tensor& f2, Tensor& f3, const std::vector<double>& d) {
  Ctx& cx = *I.cx;
  const int64_t n1 = I.n1;
  Tensor MA = tnew(cx, {n1, n1}, false), MB = tnew(cx, {n1, n1}, false);
  rec_herm_add(cx, f2, MA, n1);
  rec_herm_add(cx, f3, MB, n1);
  double* dd = (double*)cx.pool.get(n1);
  hipcheck(hipMemcpyAsync(dd, d.data(), sizeof(double) * n1, hipMemcpyHostToDevice, cx.stream), "d1");
  launch_add_diag(MA.p, dd, n1, cx.stream);
  I.M11x = tnew(cx, {n1, n1}, false);
  perm(cx, C1(), MA, "pq", false, C0(), I.M11x, "pq");
  perm(cx, CR(I.x), MB, "pq", false, C1(), I.M11x, "pq");
  hipcheck(hipStreamSynchronize(cx.stream), "m11 sync");
  cx.pool.put((double2*)dd);
  tfree(cx, MA);
  I.M11b = MB;
}

// ============================================================================
// EE
// ============================================================================
void build_sx(Ctx& cx, const Inst& I, double x, Tensor& X1, Tensor& X2, Tensor* X1h, Tensor* X2h);

void ee_init(adc_handle* h, Inst& I, Pre& P, const std::vector<double>& eps_h) {
  Ctx& cx = *I.cx;
  const int o = I.o, v = I.v, N = I.N;
  const int64_t n1 = I.n1;
  const Tensor& t = I.t1;
  Tensor fo2, fo3, fv2, fv3;
  m11_fo(h, I, P, fo2, fo3);
  m11_fv(h, I, P, fv2, fv3);
  // order <= 2: X2 = 1/2 t(ikac) <Ik||Ac> + delta parts; M11 = herm(X) + M11(1) + M11(0)
  Tensor X2 = tnew(cx, {o, v, o, v});
  ctr(cx, CR(0.5), t, "ikac", false, I.oovv, "IkAc", false, C1(), X2, "iaIA");
  rec_m11_add_delta(cx, X2, fv2, o, v, 0);
  rec_m11_add_delta(cx, X2, fo2, o, v, 1);
  Tensor MA = tnew(cx, {n1, n1}, false);
  rec_herm_add(cx, X2, MA, n1);
  {
    Tensor MAv = tensor_view(MA.p, {o, v, o, v}, {});
    perm(cx, CR(-1), I.ovov, "jaib", false, C1(), MAv, "iajb");   // <aj||ib> = -<ja||ib>
    std::vector<double> d1(n1);
    for (int i = 0; i < o; ++i)
      for (int a = 0; a < v; ++a) d1[(int64_t)i * v + a] = eps_h[o + a] - eps_h[i];
    double* dd = (double*)cx.pool.get(n1);
    hipcheck(hipMemcpyAsync(dd, d1.data(), sizeof(double) * n1, hipMemcpyHostToDevice, cx.stream), "d1");
    launch_add_diag(MA.p, dd, n1, cx.stream);
    hipcheck(hipStreamSynchronize(cx.stream), "sync");
    cx.pool.put((double2*)dd);
  }
  // third order
  Tensor X = tnew(cx, {o, v, o, v});
  const Tensor& ov4 = I.ovov;
  ctr(cx, CR(0.5), P.t2, "ikac", false, I.oovv, "IkAc", false, C1(), X, "iaIA");
  // -ts(ic)<aI||Ac>, <aI||Ac> = -ovvv[I,a,A,c] ; +ts(ka)<Ik||iA>
  ctr(cx, C1(), P.ts, "ic", false, I.ovvv, "IaAc", false, C1(), X, "iaIA");
  ctr(cx, C1(), P.ts, "ka", false, I.ooov, "IkiA", false, C1(), X, "iaIA");
  // 1/2 t*(IkAc) (Lt + Ht)(ikac)
  ctr(cx, CR(0.5), t, "IkAc", true, P.Lt, "ikac", false, C1(), X, "iaIA");
  ctr(cx, CR(0.5), t, "IkAc", true, P.Ht, "ikac", false, C1(), X, "iaIA");
  {
    // -1/2 t*(IkAc) P(iakc), P = -<la||kd> t(ilcd)
    Tensor Pq = tnew(cx, {o, v, o, v}, false);
    ctr(cx, CR(-1), ov4, "lakd", false, t, "ilcd", false, C0(), Pq, "iakc");
    ctr(cx, CR(-0.5), t, "IkAc", true, Pq, "iakc", false, C1(), X, "iaIA");
    // -1/2 t*(IkAc) P2(ikca), P2 = -<lc||id> t(klad)
    Tensor P2 = tnew(cx, {o, o, v, v}, false);
    ctr(cx, CR(-1), ov4, "lcid", false, t, "klad", false, C0(), P2, "ikca");
    ctr(cx, CR(-0.5), t, "IkAc", true, P2, "ikca", false, C1(), X, "iaIA");
    tfree(cx, Pq);
    tfree(cx, P2);
  }
  {
    // +1/2 t*(Ikcd) <ac||Ae> t(ikde), <ac||Ae> = (aA|ce) - (ae|cA);  R_Iice = t*(Ikcd) t(ikde)
    Tensor Rr = tnew(cx, {o, o, v, v}, false);
    ctr(cx, C1(), t, "Ikcd", true, t, "ikde", false, C0(), Rr, "Iice");
    Tensor sQ = tnew(cx, {N, o, o}, false);
    ctr(cx, C1(), I.Lvv, "Qce", false, Rr, "Iice", false, C0(), sQ, "QIi");
    ctr(cx, CR(0.5), I.Lvv, "QaA", false, sQ, "QIi", false, C1(), X, "iaIA");
    tfree(cx, sQ);
    const size_t budget = h->opt.mem_budget ? h->opt.mem_budget : (size_t)4 << 30;
    int64_t na = std::max<int64_t>(1, (int64_t)(budget / 4 / sizeof(double2)) / ((int64_t)v * v * v));
    na = std::min<int64_t>(na, v);
    // under a tape every block gets its own buffer (the reverse sweep reads them all)
    const bool taped = cx.tape && cx.tape->recording;
    Tensor G = taped ? Tensor{} : tnew(cx, {na, v, v, v}, false);
    for (int64_t a0 = 0; a0 < v; a0 += na) {
      const int64_t a1 = std::min<int64_t>(v, a0 + na);
      Tensor Gb = taped ? tnew(cx, {a1 - a0, v, v, v}, false) : Tensor{};
      Tensor Gs = taped ? Gb : tslice(G, 0, 0, a1 - a0);
      Tensor Ls = tslice(I.Lvv, 1, a0, a1);
      ctr(cx, C1(), Ls, "Qae", false, I.Lvv, "QcA", false, C0(), Gs, "aecA");
      Tensor Xs = tslice(X, 1, a0, a1);
      ctr(cx, CR(-0.5), Gs, "aecA", false, Rr, "Iice", false, C1(), Xs, "iaIA");
      if (taped) tfree(cx, Gb);
    }
    if (!taped) tfree(cx, G);
    tfree(cx, Rr);
  }
  {
    // +1/4 <al||iA> A_Il, A = t*(Ikcd) t(klcd); <al||iA> = -ovov[l,a,i,A]
    Tensor Ao = tnew(cx, {o, o}, false);
    ctr(cx, C1(), t, "Ikcd", true, t, "klcd", false, C0(), Ao, "Il");
    ctr(cx, CR(-0.25), ov4, "laiA", false, Ao, "Il", false, C1(), X, "iaIA");
    tfree(cx, Ao);
    // +1/4 <al||Ak> B_Iikl, B = t*(Ikcd) t(ilcd); <al||Ak> = ovov[l,a,k,A]
    Tensor Bo = tnew(cx, {o, o, o, o}, false);
    ctr(cx, C1(), t, "Ikcd", true, t, "ilcd", false, C0(), Bo, "Iikl");
    ctr(cx, CR(0.25), ov4, "lakA", false, Bo, "Iikl", false, C1(), X, "iaIA");
    tfree(cx, Bo);
    // -t*(Ikcd) <cl||iA> t(klad); <cl||iA> = -ovov[l,c,i,A]
    Tensor Eo = tnew(cx, {o, v, o, v}, false);
    ctr(cx, C1(), t, "Ikcd", true, t, "klad", false, C0(), Eo, "Icla");
    ctr(cx, C1(), ov4, "lciA", false, Eo, "Icla", false, C1(), X, "iaIA");
    tfree(cx, Eo);
    // +1/4 <aI||id> F_Ad, F = t*(klAc) t(klcd); <aI||id> = -ovov[I,a,i,d]
    Tensor F = tnew(cx, {v, v}, false);
    ctr(cx, C1(), t, "klAc", true, t, "klcd", false, C0(), F, "Ad");
    ctr(cx, CR(-0.25), ov4, "Iaid", false, F, "Ad", false, C1(), X, "iaIA");
    tfree(cx, F);
  }
  {
    // +1/4 <Ic||id> G_Acad, G = t*(klAc) t(klad), in chunks of A
    const size_t budget = h->opt.mem_budget ? h->opt.mem_budget : (size_t)4 << 30;
    int64_t nA = std::max<int64_t>(1, (int64_t)(budget / 4 / sizeof(double2)) / ((int64_t)v * v * v));
    nA = std::min<int64_t>(nA, v);
    const bool taped = cx.tape && cx.tape->recording;
    Tensor G = taped ? Tensor{} : tnew(cx, {nA, v, v, v}, false);
    for (int64_t A0 = 0; A0 < v; A0 += nA) {
      const int64_t A1 = std::min<int64_t>(v, A0 + nA);
      Tensor Gb = taped ? tnew(cx, {A1 - A0, v, v, v}, false) : Tensor{};
      Tensor Gs = taped ? Gb : tslice(G, 0, 0, A1 - A0);
      Tensor ts_ = tslice(t, 2, A0, A1);
      ctr(cx, C1(), ts_, "klAc", true, t, "klad", false, C0(), Gs, "Acad");
      Tensor Xs = tslice(X, 3, A0, A1);
      ctr(cx, CR(0.25), ov4, "Icid", false, Gs, "Acad", false, C1(), Xs, "iaIA");
      if (taped) tfree(cx, Gb);
    }
    if (!taped) tfree(cx, G);
  }
  {
    // +1/2 <Im||ik> N_kAma, N = t*(klAc) t(lmac)
    Tensor Nn = tnew(cx, {o, v, o, v}, false);
    ctr(cx, C1(), t, "klAc", true, t, "lmac", false, C0(), Nn, "kAma");
    ctr(cx, CR(0.5), I.oooo, "Imik", false, Nn, "kAma", false, C1(), X, "iaIA");
    tfree(cx, Nn);
  }
  rec_m11_add_delta(cx, X, fv3, o, v, 0);
  rec_m11_add_delta(cx, X, fo3, o, v, 1);
  Tensor MB = tnew(cx, {n1, n1}, false);
  rec_herm_add(cx, X, MB, n1);
  I.M11x = tnew(cx, {n1, n1}, false);
  perm(cx, C1(), MA, "pq", false, C0(), I.M11x, "pq");
  perm(cx, CR(I.x), MB, "pq", false, C1(), I.M11x, "pq");
  I.M11b = MB;
  for (Tensor* p : {&X2, &MA, &X, &fo2, &fo3, &fv2, &fv3}) tfree(cx, *p);
  // coupling intermediates, independent of the trial vectors:
  // W[I,J,i,B]  = sum_cd conj(t[I,J,c,d]) conj(<iB||cd>)
  // W5[J,A,a,B] = sum_kc conj(t[J,k,A,c]) conj(<kB||ac>)
  // W6[I,B,J,i] = sum_kc conj(t[I,k,B,c]) conj(<ik||Jc>)
  I.W = tnew(cx, {o, o, o, v}, false);
  ctr(cx, C1(), t, "IJcd", true, I.ovvv, "iBcd", true, C0(), I.W, "IJiB");
  I.W5 = tnew(cx, {o, v, v, v}, false);
  ctr(cx, C1(), t, "JkAc", true, I.ovvv, "kBac", true, C0(), I.W5, "JAaB");
  I.W6 = tnew(cx, {o, v, o, o}, false);
  ctr(cx, C1(), t, "IkBc", true, I.ooov, "ikJc", true, C0(), I.W6, "IBJi");
  I.E0 = tnew(cx, {o, v, v, v + o}, false);
  {
    Tensor e = tslice(I.E0, 3, 0, v);
    perm(cx, C1(), I.ovvv, "icab", true, C0(), e, "iabc");
    Tensor f = tslice(I.E0, 3, v, v + o);
    perm(cx, C1(), t, "ikab", false, C0(), f, "iabk");
  }
  I.E1 = tnew(cx, {o, o, v, 2 * o + v}, false);
  {
    Tensor e = tslice(I.E1, 3, 0, o);
    perm(cx, C1(), I.ooov, "ijka", true, C0(), e, "ijak");
    Tensor f = tslice(I.E1, 3, o, o + v);
    perm(cx, C1(), t, "IJAc", false, C0(), f, "IJAc");
    Tensor g = tslice(I.E1, 3, o + v, 2 * o + v);
    perm(cx, C1(), I.W, "IJiA", true, C0(), g, "IJAi");
  }
  if (!cx.tape) {
    // A0 is antisymmetric in (a,b) and A1 in (I,J) (so are all their terms):
    // their factors are kept with that pair packed
    const int64_t Pv = I.Pv, Po = I.Po;
    // E0h [i][P_v][2v+o]: E0 packed in (a<b), and a third block that carries
    // the x W5 term of the doubles output into the A0 product: after
    // P(IJ)P(AB), x sum_a conj(W5_JAaB) y_Ia equals P(IJ) of
    // -x sum_a conj(W5_IAaB - W5_IBaA) y_Ja over A<B, i.e. the factor
    // -conj(W5_iAaB - W5_iBaA) against x y_ja on the trial side
    const int64_t q0 = (int64_t)v + o, qw = 2 * (int64_t)v + o;
    I.E0h = tnew(cx, {o, Pv, qw}, false);
    if (Pv > 0) {
      Tensor tmp = tnew(cx, {Pv, q0}, false);
      Tensor w5t = tnew(cx, {v, v, v}, false);
      Tensor w5h = tnew(cx, {Pv, v}, false);
      for (int i = 0; i < o; ++i) {
        launch_pack_pairs(I.E0.p + (int64_t)i * v * v * q0, tmp.p, 1, v, q0, I.pair_v, cx.stream);
        Tensor d0 = tensor_view(I.E0h.p + (int64_t)i * Pv * qw, {Pv, q0}, {qw, 1});
        perm(cx, C1(), tmp, "Pq", false, C0(), d0, "Pq");
        Tensor w5i = tensor_view(I.W5.p + (int64_t)i * v * v * v, {v, v, v}, {});
        perm(cx, C1(), w5i, "AaB", false, C0(), w5t, "ABa");
        launch_pack_pairs(w5t.p, w5h.p, 1, v, v, I.pair_v, cx.stream, 1);
        Tensor d1 = tensor_view(I.E0h.p + (int64_t)i * Pv * qw + q0, {Pv, v}, {qw, 1});
        perm(cx, CR(-1.0), w5h, "Pa", true, C0(), d1, "Pa");
      }
      tfree(cx, w5h);
      tfree(cx, w5t);
      tfree(cx, tmp);
    }
    I.E1h = tnew(cx, {Po, v, 2 * o + v}, false);
    launch_pack_pairs(I.E1.p, I.E1h.p, 1, o, (int64_t)v * (2 * o + v), I.pair_o, cx.stream);
    if (Po > 0) {
      // the x W6 term of the doubles output joins the A1 product: after
      // P(IJ)P(AB), x sum_i conj(W6_IBJi) y_iA equals P(AB) of
      // -x sum_i conj(W6_IAJi - W6_JAIi) y_iB over I<J, i.e. the factor
      // -2 conj(W6_IAJi - W6_JAIi) against the x/2 y_iB already on the trial
      // side of the third block
      Tensor w6t = tnew(cx, {v, o, o, o}, false);
      perm(cx, C1(), I.W6, "IAJi", false, C0(), w6t, "AIJi");
      Tensor w6h = tnew(cx, {v, Po, o}, false);
      launch_pack_pairs(w6t.p, w6h.p, v, o, o, I.pair_o, cx.stream, 1);
      tfree(cx, w6t);
      Tensor e3 = tslice(I.E1h, 2, o + v, 2 * o + v);
      perm(cx, CR(-2.0), w6h, "APi", true, C1(), e3, "PAi");
      tfree(cx, w6h);
    }
    I.th = tnew(cx, {o, o, Pv}, false);
    launch_pack_pairs(t.p, I.th.p, (int64_t)o * o, v, 1, I.pair_v, cx.stream);
    I.tIJ = tnew(cx, {Po, v, v}, false);
    launch_pack_pairs(t.p, I.tIJ.p, 1, o, (int64_t)v * v, I.pair_o, cx.stream);
    I.oooo_p = tnew(cx, {Po, o, o}, false);
    launch_pack_pairs(I.oooo.p, I.oooo_p.p, 1, o, (int64_t)o * o, I.pair_o, cx.stream);
    I.oooo_pp = tnew(cx, {Po, Po}, false);
    launch_pack_pairs(I.oooo_p.p, I.oooo_pp.p, Po, o, 1, I.pair_o, cx.stream);
    I.ooov_p = tnew(cx, {Po, o, v}, false);
    launch_pack_pairs(I.ooov.p, I.ooov_p.p, 1, o, (int64_t)o * v, I.pair_o, cx.stream);
    I.tpp = tnew(cx, {Po, Pv}, false);
    launch_pack_pairs(I.th.p, I.tpp.p, 1, o, Pv, I.pair_o, cx.stream);
    if (Po > 0 && Pv > 0) {
      // the x t.Z4 term of the doubles output, -x sum_{k<l} t_klAB Z4_klJI
      // with Z4_klJI = sum_a <kl||Ja> y_Ia, is -x sum_a U_JaP y_Ia with the
      // trial-independent U_JaP = sum_{k<l} <kl||Ja> t_klP; under P(IJ) it
      // equals +x sum_a U_iaP y_ja, so U joins the third block of E0h
      // (already met by x y_ja)
      Tensor U = tnew(cx, {o, v, Pv}, false);
      ctr(cx, C1(), I.ooov_p, "KJa", false, I.tpp, "KP", false, C0(), U, "JaP");
      const int64_t q0 = (int64_t)v + o, qw = 2 * (int64_t)v + o;
      Tensor e3 = tensor_view(I.E0h.p + q0, {o, Pv, v}, {Pv * qw, qw, 1});
      perm(cx, C1(), U, "iaP", false, C1(), e3, "iPa");
      tfree(cx, U);
    }
    // planes of the ring matrix [k][c][j][b]: rows (j,b), columns (k,c)
    const int64_t ov = (int64_t)o * v;
    I.ringKp = pad32(ov);
    I.ringq = (unsigned short*)dmalloc(h, (size_t)ov * I.ringKp * 8);
    SplitNd sp{};
    sp.src = I.ring.p; sp.dst = I.ringq; sp.rows = ov; sp.K = ov; sp.Kp = I.ringKp; sp.conj = 0;
    sp.nm = 2; sp.md[0] = o; sp.md[1] = v; sp.ms[0] = v; sp.ms[1] = 1;
    sp.nk = 2; sp.kd[0] = o; sp.kd[1] = v; sp.ks[0] = (int64_t)v * o * v; sp.ks[1] = ov;
    launch_split_nd(sp, 1, cx.stream);
    tfree(cx, I.E0);
    tfree(cx, I.E1);
  }
  // after the pair-packed factors: X1h takes the V2 term through U
  build_sx(cx, I, I.x, I.X1, I.X2, cx.tape ? nullptr : &I.X1h, cx.tape ? nullptr : &I.X2h);
}

// ============================================================================
// IP and EA one-off work
// ============================================================================
// Trial-independent factors of the singles output that share the layout in
// which they read the unpacked doubles Y (one contraction each):
//   EE: X1_jabc = -1/2 <ja||bc> + x W5_jbac
//       X2_jkib = -1/2 <jk||ib> - x/4 W_jkib + x W6_jbki
//   IP: X1_IJiA = 1/2 <IJ||iA> + x/4 W_IJiA - x W6_IAJi
//   EA: X1_IaAB = -1/2 ovvv_IaAB + x W5_IAaB
// (the M12(1) terms and the M12(2) terms in W, W5, W6).  x enters here, so a
// change of x needs new factors.
void build_sx(Ctx& cx, const Inst& I, double x, Tensor& X1, Tensor& X2, Tensor* X1h, Tensor* X2h) {
  const int o = I.o, v = I.v;
  if (I.kind == ADC_EE) {
    X1 = tnew(cx, {o, v, v, v}, false);
    perm(cx, CR(-0.5), I.ovvv, "jabc", false, C0(), X1, "jabc");
    perm(cx, CR(x), I.W5, "jbac", false, C1(), X1, "jabc");
    if (X1h) {
      // sum_bc X1_bc Y_bc = sum_{b<c} (X1_bc - X1_cb) Y_bc for antisymmetric Y
      *X1h = tnew(cx, {o, v, I.Pv}, false);
      launch_pack_pairs(X1.p, X1h->p, (int64_t)o * v, v, 1, I.pair_v, cx.stream, 1);
      tfree(cx, X1);
      if (I.ooov_p.p && I.tpp.p && I.Po > 0) {
        // the x V2 term of the singles output, -x/4 sum_{Jkl} conj(<kl||Ja>)
        // V2_iJkl with V2_iJkl = sum_AB conj(t_klAB) Y_iJAB, equals
        // -x sum_{J,A<B} conj(U_JaAB) Y_iJAB with the trial-independent
        // U_JaP = sum_{k<l} <kl||Ja> t_klP: it joins X1h
        Tensor U = tnew(cx, {o, v, I.Pv}, false);
        ctr(cx, C1(), I.ooov_p, "KJa", false, I.tpp, "KP", false, C0(), U, "JaP");
        perm(cx, CR(-x), U, "jaP", true, C1(), *X1h, "jaP");
        tfree(cx, U);
      }
    }
    X2 = tnew(cx, {o, o, o, v}, false);
    perm(cx, CR(-0.5), I.ooov, "jkib", false, C0(), X2, "jkib");
    perm(cx, CR(-0.25 * x), I.W, "jkib", false, C1(), X2, "jkib");
    perm(cx, CR(x), I.W6, "jbki", false, C1(), X2, "jkib");
    if (X2h) {
      // likewise sum_jk X2_jk Y_jk = sum_{j<k} (X2_jk - X2_kj) Y_jk
      *X2h = tnew(cx, {I.Po, o, v}, false);
      launch_pack_pairs(X2.p, X2h->p, 1, o, (int64_t)o * v, I.pair_o, cx.stream, 1);
      tfree(cx, X2);
    }
  } else if (I.kind == ADC_IP) {
    X1 = tnew(cx, {o, o, o, v}, false);
    perm(cx, CR(0.5), I.ooov, "IJiA", false, C0(), X1, "IJiA");
    perm(cx, CR(0.25 * x), I.W, "IJiA", false, C1(), X1, "IJiA");
    perm(cx, CR(-x), I.W6, "IAJi", false, C1(), X1, "IJiA");
  } else {
    X1 = tnew(cx, {o, v, v, v}, false);
    perm(cx, CR(-0.5), I.ovvv, "IaAB", false, C0(), X1, "IaAB");
    perm(cx, CR(x), I.W5, "IAaB", false, C1(), X1, "IaAB");
  }
}

void ip_init(adc_handle* h, Inst& I, Pre& P, const std::vector<double>& eps_h) {
  Ctx& cx = *I.cx;
  const int o = I.o;
  Tensor f2, f3;
  m11_fo(h, I, P, f2, f3);
  std::vector<double> d(o);
  for (int i = 0; i < o; ++i) d[i] = -eps_h[i];
  small_m11(h, I, f2, f3, d);
  tfree(cx, f2);
  tfree(cx, f3);
  const Tensor& t = I.t1;
  I.W = tnew(cx, {o, o, o, I.v}, false);
  ctr(cx, C1(), t, "IJcd", true, I.ovvv, "iBcd", true, C0(), I.W, "IJiB");
  I.W6 = tnew(cx, {o, I.v, o, o}, false);
  ctr(cx, C1(), t, "IkBc", true, I.ooov, "ikJc", true, C0(), I.W6, "IBJi");
  build_sx(cx, I, I.x, I.X1, I.X2, nullptr, nullptr);
  // the sigma build of IP needs no three-external integrals
  tfree(cx, I.ovvv);
}

void ea_init(adc_handle* h, Inst& I, Pre& P, const std::vector<double>& eps_h) {
  Ctx& cx = *I.cx;
  const int o = I.o, v = I.v;
  Tensor f2, f3;
  m11_fv(h, I, P, f2, f3);
  std::vector<double> d(v);
  for (int a = 0; a < v; ++a) d[a] = eps_h[o + a];
  small_m11(h, I, f2, f3, d);
  tfree(cx, f2);
  tfree(cx, f3);
  const Tensor& t = I.t1;
  I.W5 = tnew(cx, {o, v, v, v}, false);
  ctr(cx, C1(), t, "JkAc", true, I.ovvv, "kBac", true, C0(), I.W5, "JAaB");
  build_sx(cx, I, I.x, I.X1, I.X2, nullptr, nullptr);
}

void ee_sigma(adc_handle* h, Inst& I, const double2* Y, double2* S, int k, int prec) {
  Ctx& cx = *I.cx;
  const int o = I.o, v = I.v;
  const int64_t n1 = I.n1, dim = I.dim, Po = I.Po;
  const double x = I.x;
  const int saved = cx.prec;
  cx.prec = prec;
  Tensor ys = tnew(cx, {k, o, v}, false);
  rows_in(cx, Y, dim, 0, ys, k, n1);
  // outside a tape the terms that sum over an antisymmetric pair of Y take it
  // once (pairs packed, factors antisymmetrised at init): see E0h, th, X1h;
  // there the fully unpacked Y is needed only by the ring term outside
  // split-bf16 (which forms its planes from Yij below)
  const bool half = I.E0h.p && !cx.tape;
  const int64_t Pv = I.Pv;
  const bool ring_planes = half && prec == ADC_SPLIT_BF16 && I.ringq;
  const bool need_Ya = !half || (x != 0.0 && !ring_planes);
  Tensor Ya = need_Ya ? tnew(cx, {k, o, o, v, v}, false) : Tensor{};
  SplitScope scope(cx, {{Ya.p, Ya.size()}, {ys.p, ys.size()}});
  // split-bf16: the unpack also writes the planes of Y in its own order (the
  // layout of the contractions summing over (j,b,c) or (a,b) with rows
  // (z,i[,j])), when that layout needs no K padding
  unsigned short* yq = nullptr;
  if (!half && prec == ADC_SPLIT_BF16 && scope.id > 0 && ((int64_t)v * v) % 32 == 0)
    yq = (unsigned short*)cx.pool.get(Ya.size() / 2);
  if (need_Ya) launch_unpack_doubles(0, Y, dim, n1, k, o, v, Ya.p, nullptr, cx.stream, yq);
  if (yq) split_cache_put(cx, scope.id, Ya.p, Ya.size(), yq);
  // the doubles unpacked in the occupied pair only (virtual pairs a<b kept,
  // [k][o][o][P_v]), and in the virtual pair only (occupied pairs i<j kept,
  // [k][v][P_o][v]); every contraction reads each of them with rows (z, first
  // index) and the rest summed, so in split-bf16 the unpack also writes those
  // planes into the build's cache
  Tensor Yh, Yij;
  if (half) {
    Yh = tnew(cx, {k, o, o, Pv}, false);
    Yij = tnew(cx, {k, v, Po, v}, false);
  }
  SplitScope hscope(cx, {{Yh.p, Yh.size()}, {Yij.p, Yij.size()}});
  // ring-layout planes of Y (split-bf16 with the ring term)
  unsigned short* Rq = nullptr;
  if (half) {
    const bool fuse = prec == ADC_SPLIT_BF16 && hscope.id > 0;
    const int64_t Kh = (int64_t)o * Pv, Kij = Po * v;
    // with K >= 32 every contraction reading Yh or Yij takes their planes, so
    // the complex copies are never written: the planes of Yij (and the ring
    // planes) come straight from the packed vectors
    const bool only = fuse && Kh >= 32 && Kij >= 32;
    unsigned short* hq = fuse ? (unsigned short*)cx.pool.get(((int64_t)k * o * pad32(Kh) * 8 + 15) / 16) : nullptr;
    unsigned short* iq = fuse ? (unsigned short*)cx.pool.get(((int64_t)k * v * pad32(Kij) * 8 + 15) / 16) : nullptr;
    launch_unpack_doubles(1, Y, dim, n1, k, o, (int)Pv, only ? nullptr : Yh.p, nullptr, cx.stream, hq, Kh, pad32(Kh));
    if (only) {
      if (ring_planes && x != 0.0) Rq = (unsigned short*)cx.pool.get(((int64_t)k * o * v * I.ringKp * 8 + 15) / 16);
      launch_ee_pair_planes(Y, dim, n1, k, o, v, iq, pad32(Kij), Rq, I.ringKp, cx.stream);
    } else {
      launch_unpack_doubles(3, Y, dim, n1, k, o, v, Yij.p, nullptr, cx.stream, iq, Kij, pad32(Kij));
    }
    if (fuse) {
      split_cache_put_rows(cx, hscope.id, Yh.p, (int64_t)k * o, Kh, pad32(Kh), hq);
      split_cache_put_rows(cx, hscope.id, Yij.p, (int64_t)k * v, Kij, pad32(Kij), iq);
    }
    if (only) {
      split_cache_planes_only(cx, hscope.id, Yh.p, Yh.size());
      split_cache_planes_only(cx, hscope.id, Yij.p, Yij.size());
    }
  }
  const Tensor& t = I.t1;

  // ---------------- singles output
  Tensor s1 = tnew(cx, {k, o, v}, false);
  {
    // M11 stays FP64
    cx.prec = 0;
    Tensor M = tensor_view(I.M11x.p, {n1, n1}, {});
    Tensor ysf = tensor_view(ys.p, {k, n1}, {});
    Tensor s1f = tensor_view(s1.p, {k, n1}, {});
    ctr(cx, C1(), M, "PQ", false, ysf, "zQ", false, C0(), s1f, "zP");
    cx.prec = prec;
  }
  // M12(1) -1/2 <ja||bc> Y_ijbc - 1/2 <jk||ib> Y_jkab with the M12(2) terms
  // x W5_JAaB Y_iJAB - x/4 W_IJiB Y_IJaB + x W6_IBJi Y_IJaB, one contraction
  // per layout of Y through the factors X1, X2
  if (half) {
    ctr(cx, C1(), I.X1h, "jaP", false, Yh, "zijP", false, C1(), s1, "zia");
    ctr(cx, C1(), I.X2h, "Pib", false, Yij, "zaPb", false, C1(), s1, "zia");
  } else {
    ctr(cx, C1(), I.X1, "jabc", false, Ya, "zijbc", false, C1(), s1, "zia");
    ctr(cx, C1(), I.X2, "jkib", false, Ya, "zjkab", false, C1(), s1, "zia");
  }
  if (x != 0.0) {
    // M12(2), grouped with the antisymmetric Y
    Tensor rY = tnew(cx, {k, v, v}, false);
    // Y is antisymmetric in its virtual pair: read it as Y_IJBA = -Y_IJAB so
    // that it shares the layout (kept virtual first) of the M12(1) term above
    if (half) ctr(cx, CR(-2.0), I.tIJ, "PAc", true, Yij, "zBPA", false, C0(), rY, "zcB");
    else ctr(cx, CR(-1.0), t, "IJAc", true, Ya, "zIJBA", false, C0(), rY, "zcB");
    ctr(cx, CR(0.5 * x), I.ovvv, "iBac", true, rY, "zcB", false, C1(), s1, "zia");
    tfree(cx, rY);
    Tensor r2 = tnew(cx, {k, o, o}, false);
    // likewise Y_JIAB = -Y_IJAB (kept occupied first); t and Y are both
    // antisymmetric in (A,B), so the half form sums the pairs A<B twice
    if (half) ctr(cx, CR(-2.0), I.th, "IkP", true, Yh, "zJIP", false, C0(), r2, "zkJ");
    else ctr(cx, CR(-1.0), t, "IkAB", true, Ya, "zJIAB", false, C0(), r2, "zkJ");
    ctr(cx, CR(0.5 * x), I.ooov, "ikJa", true, r2, "zkJ", false, C1(), s1, "zia");
    tfree(cx, r2);
    // (outside a tape the V2 term is part of the X1h product above)
    if (!half) {
      Tensor V2 = tnew(cx, {k, o, o, o, o}, false);
      ctr(cx, C1(), t, "klAB", true, Ya, "ziJAB", false, C0(), V2, "ziJkl");
      ctr(cx, CR(-0.25 * x), I.ooov, "klJa", true, V2, "ziJkl", false, C1(), s1, "zia");
      tfree(cx, V2);
    }
  }
  // ---------------- doubles output: every term goes, with its coefficient,
  // into the accumulator of the antisymmetriser it needs (P(ij): A0, P(ab):
  // A1, P(ij)P(ab): A2); one pass then antisymmetrises, packs and adds D Y
  // in reduced precision the accumulators hold complex64: every term reaching
  // them is computed to FP32 accuracy, and it halves their traffic
  const bool acc32 = prec != ADC_FP64 && !cx.tape;
  // outside a tape A0 keeps only the pairs a<b and A1 only I<J (each is
  // antisymmetric there; the pack reads them accordingly)
  auto acc = [&](std::vector<int64_t> d) { return acc32 ? tnew32(cx, d) : tnew(cx, d, false); };
  Tensor A0 = half ? acc({k, o, o, Pv}) : acc({k, o, o, v, v});
  Tensor A1 = half ? acc({k, Po, v, v}) : acc({k, o, o, v, v});
  Tensor A2 = x != 0.0 ? acc({k, o, o, v, v}) : Tensor{};
  // M21(1) and the M21(2) terms with the same output roles, one GEMM per
  // accumulator over the concatenated summed index (the factors E0, E1 are
  // built once; x goes on the trial-vector side):
  //   A0 = sum_c conj(<ic||ab>) y_jc + x sum_k t_ikab Z2_kj,  Z2_kj = sum_ia <ik||ja> y_ia
  //   A1 = sum_k conj(<ij||ka>) y_kb + x sum_c t_ijac Z1_bc + x/2 sum_i conj(W_IJiA) y_iB,
  //        Z1_bc = sum_ia <ib||ac> y_ia; the last term is -x/2 conj(W_IJiB) y_iA
  //        relabelled a <-> b, which P(ab) leaves unchanged up to the sign taken here
  {
    // at x = 0 the x parts of B0, B1 stay zero; outside a tape B0 has a third
    // block, x y_ja, for the W5 term folded into E0h
    Tensor B0 = tnew(cx, {k, o, half ? 2 * v + o : v + o}, x == 0.0);
    Tensor B1 = tnew(cx, {k, v, 2 * o + v}, x == 0.0);
    Tensor b0c = tslice(B0, 2, 0, v), b0k = tslice(B0, 2, v, v + o);
    Tensor b1k = tslice(B1, 2, 0, o), b1c = tslice(B1, 2, o, o + v), b1i = tslice(B1, 2, o + v, 2 * o + v);
    perm(cx, C1(), ys, "zjc", false, C0(), b0c, "zjc");
    perm(cx, C1(), ys, "zkb", false, C0(), b1k, "zbk");
    if (x != 0.0) {
      Tensor Z2 = tnew(cx, {k, o, o}, false);
      ctr(cx, C1(), I.ooov, "ikJa", false, ys, "zia", false, C0(), Z2, "zkJ");
      perm(cx, CR(x), Z2, "zkJ", false, C0(), b0k, "zJk");
      tfree(cx, Z2);
      Tensor Z1 = tnew(cx, {k, v, v}, false);
      ctr(cx, C1(), I.ovvv, "iBac", false, ys, "zia", false, C0(), Z1, "zBc");
      perm(cx, CR(x), Z1, "zBc", false, C0(), b1c, "zBc");
      tfree(cx, Z1);
      perm(cx, CR(0.5 * x), ys, "ziB", false, C0(), b1i, "zBi");
      if (half) {
        Tensor b0w = tslice(B0, 2, v + o, 2 * v + o);
        perm(cx, CR(x), ys, "zja", false, C0(), b0w, "zja");
      }
    }
    if (half) {
      ctr(cx, C1(), I.E0h, "iPq", false, B0, "zjq", false, C0(), A0, "zijP");
      ctr(cx, C1(), I.E1h, "PAq", false, B1, "zBq", false, C0(), A1, "zPAB");
    } else {
      ctr(cx, C1(), I.E0, "iabq", false, B0, "zjq", false, C0(), A0, "zijab");
      ctr(cx, C1(), I.E1, "IJAq", false, B1, "zBq", false, C0(), A1, "zIJAB");
    }
    tfree(cx, B0);
    tfree(cx, B1);
  }
  if (x != 0.0) {
    // (outside a tape the t.Z4 term is part of the E0h product into A0)
    if (!half) {
      Tensor Z4 = tnew(cx, {k, o, o, o, o}, false);
      ctr(cx, C1(), I.ooov, "klJa", false, ys, "zIa", false, C0(), Z4, "zklJI");
      ctr(cx, CR(-0.5 * x), t, "klAB", false, Z4, "zklJI", false, C1(), A0, "zIJAB");
      tfree(cx, Z4);
    }
    // (outside a tape the W5 and W6 terms are part of the E0h and E1h
    // products into A0 and A1, and the ring term below is the first to
    // write A2)
    if (!half) {
      ctr(cx, CR(x), I.W5, "JAaB", true, ys, "zIa", false, C0(), A2, "zIJAB");
      ctr(cx, CR(x), I.W6, "IBJi", true, ys, "ziA", false, C1(), A2, "zIJAB");
    }
    // M22(1): hole ladder (already antisymmetric in ij, so half of it goes
    // through P(ij)) and ring; the particle ladder runs packed below.  Outside
    // a tape the hole ladder is antisymmetric in both pairs and goes straight
    // into the packed sigma after the pack (below)
    if (!half) {
      ctr(cx, CR(0.25 * x), I.oooo, "klij", false, Ya, "zklab", false, C1(), A0, "zijab");
    }
    if (ring_planes) {
      // A2[z][i][j][a][b] -= x sum_kc Y_ikac ring[k][c][j][b] on the planes
      const int64_t ov = (int64_t)o * v, rows = (int64_t)k * ov;
      if (!Rq) {
        Rq = (unsigned short*)cx.pool.get((rows * I.ringKp * 8 + 15) / 16);
        launch_ee_ring_planes(Yij.p, k, o, v, Rq, I.ringKp, cx.stream);
      }
      BfGemm g{};
      g.M = rows; g.N = ov; g.Kp = I.ringKp;
      g.A = Rq; g.lda = rows;
      g.B = I.ringq; g.ldb = ov;
      g.C = A2.p; g.c32 = A2.f32 ? 1 : 0;
      g.om.nm = 3; g.om.md[0] = k; g.om.md[1] = o; g.om.md[2] = v;
      g.om.ms[0] = (int64_t)o * o * v * v; g.om.ms[1] = (int64_t)o * v * v; g.om.ms[2] = v;
      g.om.nn = 2; g.om.nd[0] = o; g.om.nd[1] = v; g.om.ns[0] = (int64_t)v * v; g.om.ns[1] = 1;
      g.alpha = CR(-x); g.beta = half ? C0() : C1(); g.tag = 0;
      gemm_bf16p(cx, g);
      cx.pool.put((double2*)Rq);
      Rq = nullptr;
    } else {
      ctr(cx, CR(-x), Ya, "zikac", false, I.ring, "kcjb", false, half ? C0() : C1(), A2, "zijab");
    }
  }
  if (half) {
    launch_pack_ee_half(A0.p, A1.p, A2.p, S, Y, dim, n1, k, o, v, I.eps, I.pair_o, I.pair_v, cx.stream,
                        acc32 ? 1 : 0);
    if (x != 0.0 && Po > 0) {
      // hole ladder: sigma_ijab += x sum_{k<l} <kl||ij> Y_klab for i<j, a<b,
      // both factors read pair-packed (P(ij) of the half sum over ordered
      // (i,j) gives the same)
      Tensor Yp = tensor_view(const_cast<double2*>(Y) + n1, {k, Po, Pv}, {dim, Pv, 1});
      Tensor Sp = tensor_view(S + n1, {k, Po, Pv}, {dim, Pv, 1});
      ctr(cx, CR(x), I.oooo_pp, "KI", false, Yp, "zKP", false, C1(), Sp, "zIP");
    }
  } else {
    rec_pack_ee(cx, A0, A1, A2, S, Y, dim, n1, k, o, v, I.eps, I.pair_o, I.pair_v);
  }
  tfree(cx, A0);
  tfree(cx, A1);
  if (A2.p) tfree(cx, A2);
  rows_out(cx, s1, S, dim, 0, k, n1, C0());
  for (Tensor* p : {&ys, &s1}) tfree(cx, *p);
  for (Tensor* p : {&Ya, &Yh, &Yij})
    if (p->p) tfree(cx, *p);
  cx.prec = saved;
}

// ============================================================================
// IP:  singles i, doubles (i<j, a)
// ============================================================================
void ip_sigma(adc_handle* h, Inst& I, const double2* Y, double2* S, int k, int prec) {
  Ctx& cx = *I.cx;
  const int o = I.o, v = I.v;
  const int64_t n1 = I.n1, dim = I.dim;
  const double x = I.x;
  const int saved = cx.prec;
  Tensor ys = tnew(cx, {k, o}, false);
  rows_in(cx, Y, dim, 0, ys, k, n1);
  Tensor Ya = tnew(cx, {k, o, o, v}, false);
  launch_unpack_doubles(1, Y, dim, n1, k, o, v, Ya.p, nullptr, cx.stream);
  SplitScope scope(cx, {{Ya.p, Ya.size()}, {ys.p, ys.size()}});
  Tensor s1 = tnew(cx, {k, o}, false);
  cx.prec = 0;
  ctr(cx, C1(), I.M11x, "PQ", false, ys, "zQ", false, C0(), s1, "zP");
  cx.prec = prec;
  // M12(1): 1/2 <IJ||iA> Y_IJA ;  M12(2): x/4 W_IJiA Y_IJA - x W6_IAJi Y_IJA,
  // summed into the factor X1
  ctr(cx, C1(), I.X1, "IJiA", false, Ya, "zIJA", false, C1(), s1, "zi");
  Tensor s2 = tnew(cx, {k, o, o, v});
  // M21(1): conj(<IJ||iA>) y_i
  ctr(cx, C1(), I.ooov, "IJiA", true, ys, "zi", false, C1(), s2, "zIJA");
  if (x != 0.0) {
    ctr(cx, CR(0.5 * x), I.W, "IJiA", true, ys, "zi", false, C1(), s2, "zIJA");
    Tensor T = tnew(cx, {k, o, o, v}, false);
    ctr(cx, CR(-1), I.W6, "IAJi", true, ys, "zi", false, C0(), T, "zIJA");
    rec_antisym_add(cx, T, s2, k, o, o, v, 1, 0, CR(x));
    // M22(1): hole ladder and ring
    ctr(cx, CR(0.5 * x), I.oooo, "klij", false, Ya, "zkla", false, C1(), s2, "zija");
    ctr(cx, C1(), Ya, "zikc", false, I.ring, "kcja", false, C0(), T, "zija");
    rec_antisym_add(cx, T, s2, k, o, o, v, 1, 0, CR(-x));
    tfree(cx, T);
  }
  rec_pack_doubles(cx, 1, s2, S, Y, dim, n1, k, o, v, I.eps, C1(), 0, I.pair_o, I.pair_v);
  rows_out(cx, s1, S, dim, 0, k, n1, C0());
  for (Tensor* p : {&ys, &Ya, &s1, &s2}) tfree(cx, *p);
  cx.prec = saved;
}

// ============================================================================
// EA:  singles a, doubles (i, a<b)
// ============================================================================
void ea_sigma(adc_handle* h, Inst& I, const double2* Y, double2* S, int k, int prec) {
  Ctx& cx = *I.cx;
  const int o = I.o, v = I.v;
  const int64_t n1 = I.n1, dim = I.dim;
  const double x = I.x;
  const int saved = cx.prec;
  const Tensor& t = I.t1;
  Tensor ys = tnew(cx, {k, v}, false);
  rows_in(cx, Y, dim, 0, ys, k, n1);
  Tensor Ya = tnew(cx, {k, o, v, v}, false);
  launch_unpack_doubles(2, Y, dim, n1, k, o, v, Ya.p, nullptr, cx.stream);
  SplitScope scope(cx, {{Ya.p, Ya.size()}, {ys.p, ys.size()}});
  Tensor s1 = tnew(cx, {k, v}, false);
  cx.prec = 0;
  ctr(cx, C1(), I.M11x, "PQ", false, ys, "zQ", false, C0(), s1, "zP");
  cx.prec = prec;
  // M12(1): 1/2 <aI||AB> Y_IAB,  <aI||AB> = -ovvv[I,a,A,B], and the M12(2)
  // term x W5_IAaB Y_IAB, summed into the factor X1
  ctr(cx, C1(), I.X1, "IaAB", false, Ya, "zIAB", false, C1(), s1, "za");
  if (x != 0.0) {
    // M12(2): the 1/4 conj(<kl||Ia>)-term
    Tensor Vk = tnew(cx, {k, o, o, o}, false);
    ctr(cx, C1(), t, "klAB", true, Ya, "zIAB", false, C0(), Vk, "zIkl");
    ctr(cx, CR(-0.25 * x), I.ooov, "klIa", true, Vk, "zIkl", false, C1(), s1, "za");
    tfree(cx, Vk);
  }
  Tensor s2 = tnew(cx, {k, o, v, v});
  // M21(1): -conj(ovvv[I,a,A,B]) y_a
  ctr(cx, CR(-1), I.ovvv, "IaAB", true, ys, "za", false, C1(), s2, "zIAB");
  if (x != 0.0) {
    Tensor T = tnew(cx, {k, o, v, v}, false);
    ctr(cx, C1(), I.W5, "IAaB", true, ys, "za", false, C0(), T, "zIAB");
    rec_antisym_add(cx, T, s2, k, o, 1, v, v, 1, CR(x));
    Tensor Z = tnew(cx, {k, o, o, o}, false);
    ctr(cx, C1(), I.ooov, "klIa", false, ys, "za", false, C0(), Z, "zklI");
    ctr(cx, CR(-0.5 * x), t, "klAB", false, Z, "zklI", false, C1(), s2, "zIAB");
    tfree(cx, Z);
    // M22(1) ring (the particle ladder runs packed below)
    ctr(cx, C1(), Ya, "zjac", false, I.ring, "jcib", false, C0(), T, "ziab");
    rec_antisym_add(cx, T, s2, k, o, 1, v, v, 1, CR(-x));
    tfree(cx, T);
  }
  rec_pack_doubles(cx, 2, s2, S, Y, dim, n1, k, o, v, I.eps, C1(), 0, I.pair_o, I.pair_v);
  rows_out(cx, s1, S, dim, 0, k, n1, C0());
  for (Tensor* p : {&ys, &Ya, &s1, &s2}) tfree(cx, *p);
  cx.prec = saved;
}

// ============================================================================
// validation (host only)
// ============================================================================
int validate(const adc_problem* p) {
  if (!p) return ADC_ERR_INVALID_ARG;
  if (p->kind < 0 || p->kind > 2) return ADC_ERR_INVALID_ARG;
  if (p->n_occ < 1 || p->n_vir < 2 || p->n_chol < 1 || p->n_roots < 1) return ADC_ERR_INVALID_ARG;
  if (!p->eps || !p->L) return ADC_ERR_INVALID_ARG;
  if (!std::isfinite(p->x)) return ADC_ERR_NONFINITE_INPUT;
  const int n = p->n_occ + p->n_vir;
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(p->eps[i])) return ADC_ERR_NONFINITE_INPUT;
  return ADC_OK;
}

int validate_L_host(const double* L, int N, int n) {
  for (int q = 0; q < N; ++q) {
    const double* Lq = L + (int64_t)q * n * n * 2;
    double mx = 0.0, dev = 0.0;
    for (int64_t i = 0; i < (int64_t)n * n * 2; ++i) {
      if (!std::isfinite(Lq[i])) return ADC_ERR_NONFINITE_INPUT;
      mx = std::max(mx, std::fabs(Lq[i]));
    }
    for (int p = 0; p < n; ++p)
      for (int r = 0; r < n; ++r) {
        const double* a = Lq + ((int64_t)p * n + r) * 2;
        const double* b = Lq + ((int64_t)r * n + p) * 2;
        dev = std::max(dev, std::fabs(a[0] - b[0]) + std::fabs(a[1] + b[1]));
      }
    if (dev > 1e-12 * mx) return ADC_ERR_NOT_HERMITIAN;
  }
  return ADC_OK;
}

int dims_of(int kind, int64_t o, int64_t v, int64_t* n1, int64_t* n2) {
  const int64_t Po = npair(o), Pv = npair(v);
  if (kind == ADC_EE) { *n1 = o * v; *n2 = Po * Pv; }
  else if (kind == ADC_IP) { *n1 = o; *n2 = Po * v; }
  else { *n1 = v; *n2 = o * Pv; }
  return 0;
}

void inst_init(adc_handle* h, const adc_problem* p, Inst& I) {
  Ctx& cx = *I.cx;
  I.kind = p->kind;
  I.o = p->n_occ;
  I.v = p->n_vir;
  I.N = p->n_chol;
  I.k = p->n_roots;
  I.x = p->x;
  I.Po = npair(I.o);
  I.Pv = npair(I.v);
  dims_of(I.kind, I.o, I.v, &I.n1, &I.n2);
  I.dim = I.n1 + I.n2;
  const int o = I.o, v = I.v, n = o + v, N = I.N;
  I.eps = (double*)dmalloc(h, sizeof(double) * n);
  hipcheck(hipMemcpy(I.eps, p->eps, sizeof(double) * n, hipMemcpyHostToDevice), "eps");
  {
    auto po = pair_table(o), pv = pair_table(v);
    I.pair_o = (int2*)dmalloc(h, sizeof(int2) * std::max<size_t>(1, po.size()));
    I.pair_v = (int2*)dmalloc(h, sizeof(int2) * std::max<size_t>(1, pv.size()));
    if (!po.empty()) hipcheck(hipMemcpy(I.pair_o, po.data(), sizeof(int2) * po.size(), hipMemcpyHostToDevice), "po");
    if (!pv.empty()) hipcheck(hipMemcpy(I.pair_v, pv.data(), sizeof(int2) * pv.size(), hipMemcpyHostToDevice), "pv");
  }
  // L on the device (borrowed or copied), then the class blocks [Q][.][.]
  double2* Ld = nullptr;
  Tensor Lown;
  if (p->L_on_device) {
    Ld = (double2*)p->L;
    // the checks adc_init makes on a host L, made on the device: finite
    // values and Hermitian L^Q (max |L^Q - L^Q^H| <= 1e-12 max |L^Q|)
    double* chk = (double*)cx.pool.get((3 * (int64_t)N + 1) / 2);
    launch_check_L(Ld, N, n, chk, cx.stream);
    std::vector<double> hc(3 * (size_t)N);
    hipcheck(hipMemcpyAsync(hc.data(), chk, sizeof(double) * hc.size(), hipMemcpyDeviceToHost, cx.stream), "check L");
    hipcheck(hipStreamSynchronize(cx.stream), "check L sync");
    cx.pool.put((double2*)chk);
    for (int q = 0; q < N; ++q)
      if (hc[3 * (size_t)q + 2] > 0.0) throw Status{ADC_ERR_NONFINITE_INPUT, "non-finite L"};
    for (int q = 0; q < N; ++q)
      if (hc[3 * (size_t)q] > 1e-12 * hc[3 * (size_t)q + 1]) throw Status{ADC_ERR_NOT_HERMITIAN, "L not Hermitian"};
  } else {
    Lown = tnew(cx, {N, n, n}, false);
    hipcheck(hipMemcpyAsync(Lown.p, p->L, sizeof(double2) * (size_t)N * n * n, hipMemcpyHostToDevice, cx.stream),
             "L");
    Ld = Lown.p;
  }
  Tensor Lfull = tensor_view(Ld, {N, n, n}, {});
  auto block = [&](int r0, int nr, int c0, int nc) {
    Tensor dst = tnew(cx, {N, nr, nc}, false);
    Tensor src = tensor_view(Ld + (int64_t)r0 * n + c0, {N, nr, nc}, {(int64_t)n * n, n, 1});
    perm(cx, C1(), src, "Qpq", false, C0(), dst, "Qpq");
    return dst;
  };
  I.Loo = block(0, o, 0, o);
  I.Lov = block(0, o, o, v);
  I.Lvo = block(o, v, 0, o);
  I.Lvv = block(o, v, o, v);
  if (Lown.p) tfree(cx, Lown);
  // zeroth-order diagonal of the packed basis
  {
    std::vector<double> d(I.dim);
    const double* e = p->eps;
    if (I.kind == ADC_EE) {
      for (int i = 0; i < o; ++i)
        for (int a = 0; a < v; ++a) d[(int64_t)i * v + a] = e[o + a] - e[i];
      int64_t q = I.n1;
      for (int i = 0; i < o; ++i)
        for (int j = i + 1; j < o; ++j)
          for (int a = 0; a < v; ++a)
            for (int b = a + 1; b < v; ++b) d[q++] = e[o + a] + e[o + b] - e[i] - e[j];
    } else if (I.kind == ADC_IP) {
      for (int i = 0; i < o; ++i) d[i] = -e[i];
      int64_t q = I.n1;
      for (int i = 0; i < o; ++i)
        for (int j = i + 1; j < o; ++j)
          for (int a = 0; a < v; ++a) d[q++] = e[o + a] - e[i] - e[j];
    } else {
      for (int a = 0; a < v; ++a) d[a] = e[o + a];
      int64_t q = I.n1;
      for (int i = 0; i < o; ++i)
        for (int a = 0; a < v; ++a)
          for (int b = a + 1; b < v; ++b) d[q++] = e[o + a] + e[o + b] - e[i];
    }
    I.diag = (double*)dmalloc(h, sizeof(double) * I.dim);
    hipcheck(hipMemcpy(I.diag, d.data(), sizeof(double) * I.dim, hipMemcpyHostToDevice), "diag");
  }
  {
    std::vector<double> eps_h(p->eps, p->eps + n);
    init_integrals(h, I);
    Pre P;
    init_amplitudes(h, I, P);
    if (I.kind == ADC_EE) ee_init(h, I, P, eps_h);
    else if (I.kind == ADC_IP) ip_init(h, I, P, eps_h);
    else ea_init(h, I, P, eps_h);
    I.ts = P.ts;  // kept for the ground-state density of the properties
    P.ts = Tensor{};
    for (Tensor* q : {&P.Lt, &P.Ht, &P.t2}) tfree(cx, *q);
  }
  // the trial-independent operands are frozen from here on: their split-bf16
  // planes are kept per layout (at most their own size in bytes) and reused
  // by every sigma build
  for (Tensor* t : {&I.oooo, &I.ooov, &I.oovv, &I.ovov, &I.ovvv, &I.ring, &I.t1, &I.W, &I.W5, &I.W6, &I.E0, &I.E1,
                    &I.X1, &I.X2, &I.E0h, &I.E1h, &I.th, &I.X1h, &I.X2h, &I.tIJ, &I.oooo_p, &I.oooo_pp, &I.ooov_p, &I.tpp})
    if (t->p) split_freeze(cx, t->p, t->size(), t->size() * (int64_t)sizeof(double2));
  // host copy of diag(M11x) for the Davidson guesses
  {
    std::vector<double2> m(I.n1 * I.n1);
    hipcheck(hipStreamSynchronize(cx.stream), "sync");
    hipcheck(hipMemcpy(m.data(), I.M11x.p, sizeof(double2) * m.size(), hipMemcpyDeviceToHost), "m11");
    I.m11diag.resize(I.n1);
    for (int64_t i = 0; i < I.n1; ++i) I.m11diag[i] = m[i * I.n1 + i].x;
  }
}

// ============================================================================
// small Hermitian eigensolver (cyclic complex Jacobi), host
// ============================================================================
void heevj(int n, std::vector<zc>& A, std::vector<double>& w, std::vector<zc>& V) {
  // a non-finite entry (a trial vector or sigma result gone bad) ends the
  // solve with an error; the rotations and the ordering below need numbers
  for (size_t i = 0; i < (size_t)n * n; ++i)
    if (!std::isfinite(A[i].real()) || !std::isfinite(A[i].imag()))
      throw Status{ADC_ERR_NONFINITE_INPUT, "non-finite subspace matrix"};
  V.assign((size_t)n * n, zc(0, 0));
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> zc& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double m = std::norm(a(i, j));
        tot += m;
        if (i != j) off += m;
      }
    if (off <= 1e-30 * std::max(tot, 1e-300)) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const zc apq = a(p, q);
        const double mag = std::abs(apq);
        if (mag < 1e-300) continue;
        const zc ph = apq / mag;  // a_pq = |a_pq| e^{i phi}
        const double app = a(p, p).real(), aqq = a(q, q).real();
        const double theta = 0.5 * std::atan2(2.0 * mag, aqq - app);
        const double c = std::cos(theta), s = std::sin(theta);
        // columns: new_p = c*col_p - s*conj(ph)*col_q ; new_q = s*ph*col_p + c*col_q
        for (int i = 0; i < n; ++i) {
          const zc xp = a(i, p), xq = a(i, q);
          a(i, p) = c * xp - s * std::conj(ph) * xq;
          a(i, q) = s * ph * xp + c * xq;
        }
        for (int j = 0; j < n; ++j) {
          const zc xp = a(p, j), xq = a(q, j);
          a(p, j) = c * xp - s * ph * xq;
          a(q, j) = s * std::conj(ph) * xp + c * xq;
        }
        for (int i = 0; i < n; ++i) {
          const zc xp = V[(size_t)i * n + p], xq = V[(size_t)i * n + q];
          V[(size_t)i * n + p] = c * xp - s * std::conj(ph) * xq;
          V[(size_t)i * n + q] = s * ph * xp + c * xq;
        }
        a(p, q) = 0.0;
        a(q, p) = 0.0;
      }
  }
  // sort ascending
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return a(x, x).real() < a(y, y).real(); });
  w.resize(n);
  std::vector<zc> V2((size_t)n * n);
  for (int c = 0; c < n; ++c) {
    w[c] = a(idx[c], idx[c]).real();
    for (int r = 0; r < n; ++r) V2[(size_t)r * n + c] = V[(size_t)r * n + idx[c]];
  }
  V.swap(V2);
}

// ============================================================================
// Davidson on device vectors
// ============================================================================
// The terms other than the particle-particle ladder work on unpacked doubles
// ([k][o][o][v][v] for EE): their workspace grows with the number of trial
// vectors, so they take the vectors in groups that fit the workspace budget.
// The ladder, whose <ab||cd> assembly does not depend on the vectors, then
// runs once over all of them (it adds into the packed output).
// workspace bytes a build plans for: the allocation-free call's scratch, the
// handle's budget, or the default
size_t cx_ws(const adc_handle* h, const Ctx& cx, size_t dflt) {
  if (cx.ws_override) return cx.ws_override;
  return h->opt.mem_budget ? h->opt.mem_budget : dflt;
}

void sigma_dispatch(adc_handle* h, Inst& I, const double2* Y, double2* S, int k, int prec) {
  if (k <= 0) return;
  // Y stays unchanged during the build: splits of it are shared by the
  // contractions (and the ladder) that read it in the same layout
  SplitScope yscope(*I.cx, {{Y, (int64_t)k * I.dim}});
  const int64_t o = I.o, v = I.v;
  const int64_t unp = I.kind == ADC_EE ? o * o * v * v : (I.kind == ADC_IP ? o * o * v : o * v * v);
  const size_t ws = cx_ws(h, *I.cx, (size_t)16 << 30);
  // unpacked vectors, three accumulators, operand planes and temporaries
  const int64_t per_row = std::max<int64_t>(1, 6 * unp * (int64_t)sizeof(double2));
  const int rows = (int)std::max<int64_t>(1, std::min<int64_t>(k, (int64_t)ws / per_row));
  for (int r0 = 0; r0 < k; r0 += rows) {
    const int nr = std::min(rows, k - r0);
    const double2* Yr = Y + (int64_t)r0 * I.dim;
    double2* Sr = S + (int64_t)r0 * I.dim;
    if (I.kind == ADC_EE) ee_sigma(h, I, Yr, Sr, nr, prec);
    else if (I.kind == ADC_IP) ip_sigma(h, I, Yr, Sr, nr, prec);
    else ea_sigma(h, I, Yr, Sr, nr, prec);
  }
  if (I.x != 0.0 && I.kind != ADC_IP) {
    const int64_t nrow = I.kind == ADC_EE ? I.Po : I.o;
    ladder(h, I, Y, I.dim, I.n1, S, I.dim, I.n1, nrow, k, CR(I.x), prec);
  }
}

// Sigma build of a small instance replayed from a captured hipGraph: the
// launch sequence of one build is fixed for given rows and precision, so it is
// captured once (after an eager warm-up that creates every workspace block and
// precision plane) and replayed on staging buffers.  Worth it where kernel
// launches, not arithmetic, dominate.
constexpr double kGraphMaxCost = 5e9;  // complex MACs of one build

double inst_cost(const Inst& I) {
  const double o = I.o, v = I.v, N = I.N, k = I.k;
  const double Po = o * (o - 1) / 2, Pv = v * (v - 1) / 2;
  if (I.kind == ADC_EE) return 2 * N * Pv * Pv + k * (Po * Pv * Pv + std::pow(o * v, 3) + o * o * v * v * v);
  if (I.kind == ADC_IP) return k * (o * std::pow(o * v, 2) + Po * Po * v) + N * o * o * v * v;
  return 2 * N * Pv * Pv + k * (o * Pv * Pv + v * std::pow(o * v, 2));
}

// After a capture that failed: make sure the stream has left capture mode
// (an invalidated capture can survive a failed end) and clear the error.
void end_failed_capture(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(s, &g);
    if (g) (void)hipGraphDestroy(g);
  }
  (void)hipGetLastError();
}

void sigma_call(adc_handle* h, Inst& I, const double2* Y, double2* S, int rows, int prec) {
  Ctx& cx = *I.cx;
  if (rows <= 0) return;
  if (h->opt.graphs != 1 || inst_cost(I) > kGraphMaxCost || I.graphs_off) {
    sigma_dispatch(h, I, Y, S, rows, prec);
    return;
  }
  Inst::Graph* G = nullptr;
  for (auto& g : I.graphs)
    if (g.rows == rows && g.prec == prec) G = &g;
  const size_t bytes = sizeof(double2) * (size_t)rows * I.dim;
  if (!G) {
    Inst::Graph ng;
    ng.rows = rows;
    ng.prec = prec;
    ng.Yin = (double2*)dmalloc(h, bytes);
    ng.Sout = (double2*)dmalloc(h, bytes);
    hipcheck(hipMemcpyAsync(ng.Yin, Y, bytes, hipMemcpyDeviceToDevice, cx.stream), "graph in");
    sigma_dispatch(h, I, ng.Yin, ng.Sout, rows, prec);  // warm-up: workspace, planes, tuning
    hipcheck(hipStreamSynchronize(cx.stream), "graph warm");
    cx.pool.begin_hold();
    hipError_t e;
    {
      std::shared_lock<std::shared_mutex> gate(capture_gate());
      e = hipStreamBeginCapture(cx.stream, hipStreamCaptureModeRelaxed);
      if (e == hipSuccess) {
        try {
          sigma_dispatch(h, I, ng.Yin, ng.Sout, rows, prec);
        } catch (const HipError& err) {
          e = err.e;
        } catch (...) {
          hipGraph_t dead = nullptr;
          (void)hipStreamEndCapture(cx.stream, &dead);
          if (dead) (void)hipGraphDestroy(dead);
          for (double2* p : cx.pool.end_hold()) cx.pool.put(p);
          throw;
        }
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(cx.stream, &g);
        if (e == hipSuccess) e = ee;
        if (e == hipSuccess) ng.g = g;
        else if (g) (void)hipGraphDestroy(g);
      }
    }
    ng.held = cx.pool.end_hold();
    if (e == hipSuccess) e = hipGraphInstantiate(&ng.ex, ng.g, nullptr, nullptr, 0);
    // the warm-up already holds this call's result
    if (e != hipSuccess) {
      // no graph (e.g. no memory for the capture's own blocks): this
      // instance's sigma builds run eagerly from now on
      end_failed_capture(cx.stream);
      if (ng.g) (void)hipGraphDestroy(ng.g);
      for (double2* p : ng.held) cx.pool.put(p);
      I.graphs_off = true;
      hipcheck(hipMemcpyAsync(S, ng.Sout, bytes, hipMemcpyDeviceToDevice, cx.stream), "graph out");
      return;
    }
    I.graphs.push_back(std::move(ng));
    G = &I.graphs.back();
    hipcheck(hipMemcpyAsync(S, G->Sout, bytes, hipMemcpyDeviceToDevice, cx.stream), "graph out");
    return;
  }
  hipcheck(hipMemcpyAsync(G->Yin, Y, bytes, hipMemcpyDeviceToDevice, cx.stream), "graph in");
  hipcheck(hipGraphLaunch(G->ex, cx.stream), "graph launch");
  hipcheck(hipMemcpyAsync(S, G->Sout, bytes, hipMemcpyDeviceToDevice, cx.stream), "graph out");
}

void release_graphs(Inst& I) {
  for (auto& g : I.graphs) {
    if (g.ex) (void)hipGraphExecDestroy(g.ex);
    if (g.g) (void)hipGraphDestroy(g.g);
    for (double2* p : g.held) I.cx->pool.put(p);
  }
  I.graphs.clear();
}

// G[a][b] = sum_i conj(X[a][i]) Y[b][i]  (ra x rb, host result)
std::vector<zc> gram(Ctx& cx, const double2* X, int ra, const double2* Y, int rb, int64_t dim) {
  std::vector<zc> G((size_t)ra * rb, zc(0, 0));
  if (ra == 0 || rb == 0) return G;
  const int64_t chunk = 1 << 16;
  const int64_t nsplit = dim / chunk;
  const int64_t rem = dim - nsplit * chunk;
  const int64_t nparts = nsplit + (rem ? 1 : 0);
  double2* part = cx.pool.get(nparts * ra * rb);
  if (nsplit) {
    GemmDesc g{};
    g.M = ra; g.N = rb; g.K = chunk; g.batch = nsplit;
    g.A = X; g.sam = dim; g.sak = 1; g.sab = chunk; g.conjA = 1;
    g.B = Y; g.sbk = 1; g.sbn = dim; g.sbb = chunk;
    g.C = part; g.scm = rb; g.scn = 1; g.scb = (int64_t)ra * rb;
    g.alpha = C1(); g.beta = C0();
    { const int sp = cx.prec; cx.prec = 0; gemm(cx, g); cx.prec = sp; }
  }
  if (rem) {
    GemmDesc g{};
    g.M = ra; g.N = rb; g.K = rem; g.batch = 1;
    g.A = X + nsplit * chunk; g.sam = dim; g.sak = 1; g.sab = 0; g.conjA = 1;
    g.B = Y + nsplit * chunk; g.sbk = 1; g.sbn = dim; g.sbb = 0;
    g.C = part + nsplit * ra * rb; g.scm = rb; g.scn = 1; g.scb = 0;
    g.alpha = C1(); g.beta = C0();
    { const int sp = cx.prec; cx.prec = 0; gemm(cx, g); cx.prec = sp; }
  }
  std::vector<double2> hp((size_t)nparts * ra * rb);
  hipcheck(hipMemcpyAsync(hp.data(), part, sizeof(double2) * hp.size(), hipMemcpyDeviceToHost, cx.stream), "gram");
  hipcheck(hipStreamSynchronize(cx.stream), "gram sync");
  cx.pool.put(part);
  for (int64_t s = 0; s < nparts; ++s)
    for (int64_t e = 0; e < (int64_t)ra * rb; ++e) G[e] += zc(hp[s * ra * rb + e].x, hp[s * ra * rb + e].y);
  return G;
}

// Out[r][i] = sum_a C[a][r] In[a][i]  (C is m x r host matrix), beta accumulate
void combine(Ctx& cx, const std::vector<zc>& Cm, int m, int r, const double2* In, double2* Out, int64_t dim,
             cplx alpha, cplx beta) {
  if (m == 0 || r == 0) return;
  double2* c = cx.pool.get((int64_t)m * r);
  std::vector<double2> hc((size_t)m * r);
  for (size_t i = 0; i < hc.size(); ++i) hc[i] = make_double2(Cm[i].real(), Cm[i].imag());
  hipcheck(hipMemcpyAsync(c, hc.data(), sizeof(double2) * hc.size(), hipMemcpyHostToDevice, cx.stream), "comb");
  GemmDesc g{};
  g.M = r; g.N = dim; g.K = m; g.batch = 1;
  g.A = c; g.sam = 1; g.sak = r; g.sab = 0;        // A(r', a) = C[a][r']
  g.B = In; g.sbk = dim; g.sbn = 1; g.sbb = 0;
  g.C = Out; g.scm = dim; g.scn = 1; g.scb = 0;
  g.alpha = alpha; g.beta = beta;
  { const int sp = cx.prec; cx.prec = 0; gemm(cx, g); cx.prec = sp; }
  hipcheck(hipStreamSynchronize(cx.stream), "comb sync");
  cx.pool.put(c);
}

// orthonormalise rows of N (nn x dim) against V (m x dim) and among themselves;
// returns the number of kept rows (compacted to the front of N)
int orthonormalize(Ctx& cx, double2* V, int m, double2* N, int nn, int64_t dim) {
  for (int pass = 0; pass < 2; ++pass) {
    if (m > 0) {
      auto C = gram(cx, V, m, N, nn, dim);  // m x nn
      combine(cx, C, m, nn, V, N, dim, CR(-1), C1());
    }
    auto G = gram(cx, N, nn, N, nn, dim);
    std::vector<double> w;
    std::vector<zc> U;
    heevj(nn, G, w, U);
    const double wmax = w.empty() ? 0.0 : w.back();
    std::vector<int> keep;
    for (int j = 0; j < nn; ++j)
      if (w[j] > 1e-12 * std::max(wmax, 1e-300) && w[j] > 1e-20) keep.push_back(j);
    // new rows r = sum_a U[a][j]/sqrt(w_j) N[a]
    const int nk = (int)keep.size();
    // G = U diag(w) U^H with G[a][b] = <N_a|N_b>: q_j = sum_a U[a][j] N_a / sqrt(w_j)
    std::vector<zc> Cm((size_t)nn * nk);
    for (int a = 0; a < nn; ++a)
      for (int c = 0; c < nk; ++c) Cm[(size_t)a * nk + c] = U[(size_t)a * nn + keep[c]] / std::sqrt(w[keep[c]]);
    double2* tmp = cx.pool.get((int64_t)std::max(1, nk) * dim);
    combine(cx, Cm, nn, nk, N, tmp, dim, C1(), C0());
    if (nk) hipcheck(hipMemcpyAsync(N, tmp, sizeof(double2) * nk * dim, hipMemcpyDeviceToDevice, cx.stream), "on");
    hipcheck(hipStreamSynchronize(cx.stream), "on sync");
    cx.pool.put(tmp);
    nn = nk;
    if (nn == 0) break;
  }
  return nn;
}

// out[r] = sum_i conj(X[r][i]) Y[r][i] for contiguous rows
std::vector<zc> row_dots(Ctx& cx, const double2* X, const double2* Y, int rows, int64_t dim) {
  const int nb = row_dot_blocks(dim);
  double2* part = cx.pool.get((int64_t)rows * nb);
  launch_row_dots(X, dim, Y, dim, rows, dim, part, nb, cx.stream);
  std::vector<double2> hp((size_t)rows * nb);
  hipcheck(hipMemcpyAsync(hp.data(), part, sizeof(double2) * hp.size(), hipMemcpyDeviceToHost, cx.stream), "rd");
  hipcheck(hipStreamSynchronize(cx.stream), "rd sync");
  cx.pool.put(part);
  std::vector<zc> out(rows, zc(0, 0));
  for (int r = 0; r < rows; ++r)
    for (int b = 0; b < nb; ++b) out[r] += zc(hp[(size_t)r * nb + b].x, hp[(size_t)r * nb + b].y);
  return out;
}

std::vector<double> row_norms2(Ctx& cx, const double2* X, int rows, int64_t dim) {
  const int nb = row_dot_blocks(dim);
  double2* part = cx.pool.get((int64_t)rows * nb);
  launch_row_dots(X, dim, X, dim, rows, dim, part, nb, cx.stream);
  std::vector<double2> hp((size_t)rows * nb);
  hipcheck(hipMemcpyAsync(hp.data(), part, sizeof(double2) * hp.size(), hipMemcpyDeviceToHost, cx.stream), "rn");
  hipcheck(hipStreamSynchronize(cx.stream), "rn sync");
  cx.pool.put(part);
  std::vector<double> out(rows, 0.0);
  for (int r = 0; r < rows; ++r)
    for (int b = 0; b < nb; ++b) out[r] += hp[(size_t)r * nb + b].x;
  return out;
}

// ---------------------------------------------------------------------------
// Davidson preconditioner on the singles block.  The step P r of the new
// directions takes (w_r - M11)^-1 exactly on the singles part, from
// M11 = U diag(lam) U^H (one FP64 eigendecomposition per solve), and the
// zeroth-order diagonal on the doubles.  Strongly coupled singles spectra
// need far fewer iterations with it (an EE instance with o = 29, v = 231:
// 40 instead of 77 to |r| < 1e-4), and the coupling of the singles to the
// doubles stays with Olsen's correction.
// ---------------------------------------------------------------------------
constexpr int64_t kPrecondMaxN1 = 12288;

struct SinglesPrecond {
  int64_t n1 = 0;
  int kmax = 0;
  double2* E = nullptr;   // [n1][n1] row-major: row j = conj of eigenvector j (U^H)
  double* lam = nullptr;  // [n1] eigenvalues
  double2* C = nullptr;   // [n1][kmax] coefficients of the residuals in the eigenbasis
  bool on() const { return E != nullptr; }
};

void precond_release(Ctx& cx, SinglesPrecond& P) {
  for (double2* q : {P.E, (double2*)P.lam, P.C}) cx.pool.put(q);
  P = SinglesPrecond{};
}

// The eigendecomposition of M11x for a solve with up to kmax new directions
// per iteration (nothing when the option asks for the diagonal or n1 is
// outside 2 .. kPrecondMaxN1; a failed decomposition leaves the diagonal).
void precond_setup(adc_handle* h, Inst& I, SinglesPrecond& P, int kmax) {
  Ctx& cx = *I.cx;
  // deterministic solves keep the diagonal: the solver library's own
  // reduction order is not part of the library's bitwise guarantee
  if (h->opt.precond != 0 || h->opt.deterministic || I.n1 < 2 || I.n1 > kPrecondMaxN1 || !I.M11x.p) return;
  const int64_t n1 = I.n1;
  auto t0 = std::chrono::steady_clock::now();
  P.n1 = n1;
  P.kmax = kmax;
  P.E = cx.pool.get(n1 * n1);
  P.lam = (double*)cx.pool.get((n1 + 1) / 2);
  P.C = cx.pool.get(n1 * kmax);
  double* offd = (double*)cx.pool.get((n1 + 1) / 2);
  int* info = (int*)cx.pool.get(1);
  hipcheck(hipMemcpyAsync(P.E, I.M11x.p, sizeof(double2) * n1 * n1, hipMemcpyDeviceToDevice, cx.stream), "m11 copy");
  // M11x is Hermitian and row-major; read column-major it is conj(M11x),
  // with the same eigenvalues and conjugated eigenvectors, so the
  // column-major eigenvectors the solver returns, read row-major, are U^H.
  // The solver may allocate and free device memory: no other lane may be
  // recording a graph meanwhile.
  rocblas_status st = rocblas_status_internal_error;
  int info_h = -1;
  {
    std::unique_lock<std::shared_mutex> gate(capture_gate());
    rocblas_handle rb = nullptr;
    if (rocblas_create_handle(&rb) == rocblas_status_success) {
      rocblas_set_stream(rb, cx.stream);
      st = rocsolver_zheevd(rb, rocblas_evect_original, rocblas_fill_upper, (rocblas_int)n1,
                            (rocblas_double_complex*)P.E, (rocblas_int)n1, P.lam, offd, info);
      (void)hipStreamSynchronize(cx.stream);
      (void)rocblas_destroy_handle(rb);
    }
  }
  if (st == rocblas_status_success) {
    hipcheck(hipMemcpyAsync(&info_h, info, sizeof(int), hipMemcpyDeviceToHost, cx.stream), "eig info");
    hipcheck(hipStreamSynchronize(cx.stream), "eig info sync");
  }
  cx.pool.put((double2*)offd);
  cx.pool.put((double2*)info);
  if (st != rocblas_status_success || info_h != 0) {
    (void)hipGetLastError();
    precond_release(cx, P);
  }
  if (h->opt.verbose)
    std::fprintf(stderr, "[adc] singles preconditioner: n1 %lld, %s in %.0f ms\n", (long long)n1,
                 P.on() ? "eigendecomposition" : "eigendecomposition failed, diagonal",
                 std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
}

// P.C = (U^H R_singles) scaled by 1 / (w_r - lam_j): before the diagonal step
// overwrites R (rows of length dim, rows <= kmax)
void precond_coeffs(Ctx& cx, const SinglesPrecond& P, const double2* R, const double* w, int rows, int64_t dim) {
  if (!P.on() || rows <= 0) return;
  const int sp = cx.prec;
  cx.prec = 0;
  GemmDesc g{};
  g.M = P.n1; g.N = rows; g.K = P.n1; g.batch = 1;
  g.A = P.E; g.sam = P.n1; g.sak = 1;
  g.B = R; g.sbk = 1; g.sbn = dim;
  g.C = P.C; g.scm = rows; g.scn = 1;
  g.alpha = C1(); g.beta = C0();
  gemm(cx, g);
  cx.prec = sp;
  launch_shift_scale(P.C, P.lam, w, P.n1, rows, cx.stream);
}

// singles part of N = U P.C (after the diagonal step wrote all of N)
void precond_store(Ctx& cx, const SinglesPrecond& P, double2* N, int rows, int64_t dim) {
  if (!P.on() || rows <= 0) return;
  const int sp = cx.prec;
  cx.prec = 0;
  GemmDesc g{};
  g.M = rows; g.N = P.n1; g.K = P.n1; g.batch = 1;
  g.A = P.C; g.sam = 1; g.sak = rows;
  g.B = P.E; g.sbk = P.n1; g.sbn = 1; g.conjB = 1;
  g.C = N; g.scm = dim; g.scn = 1;
  g.alpha = C1(); g.beta = C0();
  gemm(cx, g);
  cx.prec = sp;
}

// ---------------------------------------------------------------------------
// device-side iteration (options.graphs): everything from the Gram matrix of
// the subspace to the orthonormalised new directions runs on the device, in
// FP64, and is captured once per subspace size as a hipGraph; the host reads
// one small report per iteration and then enqueues the sigma build of the
// directions it keeps.
// ---------------------------------------------------------------------------
// K-chunks of a device Gram matrix over a vector length dim.  The products
// are short (a few dozen rows) and long (dim), so one workgroup per chunk
// walks its chunk with little in flight: about 2048 chunks keep ~6 of them on
// every compute unit.  What is left after the whole chunks is cut again into
// at most 64 pieces, and the last few elements make one more part, so no
// single workgroup walks a long remainder.
struct GramSplit {
  int64_t chunk = 0, n1 = 0, chunk2 = 0, n2 = 0, tail = 0;
  int64_t parts() const { return n1 + n2 + (tail ? 1 : 0); }
};
GramSplit gram_split(int64_t dim) {
  GramSplit g;
  g.chunk = std::max<int64_t>(256, ((dim + 2047) / 2048 + 15) / 16 * 16);
  g.n1 = dim / g.chunk;
  const int64_t rem = dim - g.n1 * g.chunk;
  g.chunk2 = std::max<int64_t>(16, ((rem + 63) / 64 + 15) / 16 * 16);
  g.n2 = rem / g.chunk2;
  g.tail = rem - g.n2 * g.chunk2;
  return g;
}
int64_t gram_parts(int64_t dim) { return gram_split(dim).parts(); }

// out[a][b] (row stride ldo) = sum_i conj(X[a][i]) Y[b][i] (ra x rb) on the
// device, in FP64: per-chunk products into part, then their sum (through
// stage when there are many parts)
void gram_dev(Ctx& cx, const double2* X, int ra, const double2* Y, int rb, int64_t dim, double2* part,
              double2* stage, double2* out, int ldo) {
  const GramSplit sp = gram_split(dim);
  // a few columns: the 32-wide tiles
  const int tile = rb <= 32 ? (ra <= 64 ? 4 : 3) : 0;
  int64_t at = 0, p0 = 0;
  auto launch = [&](int64_t len, int64_t nb) {
    if (nb <= 0 || len <= 0) return;
    GemmDesc g{};
    g.M = ra; g.N = rb; g.K = len; g.batch = nb;
    g.A = X + at; g.sam = dim; g.sak = 1; g.sab = len; g.conjA = 1;
    g.B = Y + at; g.sbk = 1; g.sbn = dim; g.sbb = len;
    g.C = part + p0 * ra * rb; g.scm = rb; g.scn = 1; g.scb = (int64_t)ra * rb;
    g.alpha = C1(); g.beta = C0();
    g.tile = tile;
    launch_zgemm(g, 0, cx.stream);
    at += len * nb;
    p0 += nb;
  };
  launch(sp.chunk, sp.n1);
  launch(sp.chunk2, sp.n2);
  launch(sp.tail, sp.tail ? 1 : 0);
  launch_sum_parts(part, (int)p0, ra, rb, stage, out, ldo, cx.stream);
}

// Out[r][i] = alpha sum_a C[a][r] In[a][i] + beta Out[r][i], C a device matrix
// with row stride ldc (a < m, r < nr)
void combine_dev(Ctx& cx, const double2* C, int ldc, int m, int nr, const double2* In, double2* Out, int64_t dim,
                 cplx alpha, cplx beta) {
  launch_combine_cols(nullptr, C, ldc, m, nr, In, Out, dim, alpha, beta, cx.stream);
}

struct DevDav {
  int k = 0, mmax = 0, nb = 1;
  int64_t dim = 0;
  double2 *N = nullptr, *T = nullptr;                  // new directions [k][dim], temporary [2k][dim]
  double2 *G = nullptr, *U = nullptr, *Aw = nullptr, *Vw = nullptr;  // [mmax][mmax]
  double2 *gpart = nullptr, *gstage = nullptr, *rpart = nullptr;  // Gram partial sums, their first-stage sums, row dots
  double2 *rn2 = nullptr, *ra = nullptr, *rb = nullptr;  // row sums [k]
  double2 *Cc = nullptr, *Gn = nullptr, *Un = nullptr;   // [mmax][k], [k][k], [k][k]
  double *w = nullptr, *wn = nullptr, *wold = nullptr, *par = nullptr, *rep = nullptr;
  double* rep_host = nullptr;  // the lane's page-locked buffer
  int lds_max = 0;             // dynamic LDS bytes the eigensolver may take
  bool capture_off = false;    // a capture failed: iterate launch by launch
  const SinglesPrecond* sp = nullptr;  // the singles-block preconditioner (or off)
  struct Graph {
    int m = 0;
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    std::vector<double2*> held;
  };
  std::vector<Graph> graphs;
  std::vector<double2*> blocks;
  int rep_len() const { return 4 + 3 * k; }
  int mode(int n) const {
    if (heev_lds_bytes(n, 2) <= (size_t)lds_max) return 2;
    if (heev_lds_bytes(n, 1) <= (size_t)lds_max) return 1;
    return 0;
  }
};

void devdav_setup(Ctx& cx, DevDav& D, int k, int mmax, int64_t dim) {
  D.k = k;
  D.mmax = mmax;
  D.dim = dim;
  D.nb = row_dot_blocks(dim);
  auto take = [&](int64_t n) {
    double2* p = cx.pool.get(std::max<int64_t>(n, 1));
    D.blocks.push_back(p);
    return p;
  };
  const int64_t nparts = gram_parts(dim);
  const int64_t mm = (int64_t)mmax * mmax;
  D.N = take((int64_t)k * dim);
  D.T = take((int64_t)2 * k * dim);
  D.G = take(mm);  // the subspace Gram matrix, kept across iterations, row stride mmax
  D.U = take(mm);
  D.Aw = take(mm);
  D.Vw = take(mm);
  // every Gram product here has at most mmax rows and k columns
  D.gpart = take(nparts * mmax * k);
  D.gstage = take((int64_t)sum_parts_slices((int)nparts) * mmax * k);
  D.rpart = take((int64_t)3 * k * D.nb);
  D.rn2 = take(k);
  D.ra = take(k);
  D.rb = take(k);
  D.Cc = take((int64_t)mmax * k);
  D.Gn = take((int64_t)k * k);
  D.Un = take((int64_t)k * k);
  D.w = (double*)take(mmax);
  D.wn = (double*)take(k);
  D.wold = (double*)take(k);
  D.par = (double*)take(2);
  D.rep = (double*)take(D.rep_len());
  // the report, then the two convergence thresholds sent with each step
  D.rep_host = cx.pinned((size_t)D.rep_len() + 2);
  int dev = 0, lds = 0;
  hipcheck(hipGetDevice(&dev), "device");
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
    (void)hipGetLastError();
    lds = 0;
  }
  const int64_t avail = (int64_t)lds - (int64_t)heev_static_lds() - 1024;
  D.lds_max = (int)std::max<int64_t>(0, avail);
  if (D.lds_max > 0) heev_allow_lds((size_t)D.lds_max);
}

void devdav_release(Ctx& cx, DevDav& D) {
  if (!D.graphs.empty() || !D.blocks.empty()) {
    (void)hipStreamSynchronize(cx.stream);
    (void)hipGetLastError();
  }
  for (auto& g : D.graphs) {
    if (g.ex) (void)hipGraphExecDestroy(g.ex);
    if (g.g) (void)hipGraphDestroy(g.g);
    for (double2* p : g.held) cx.pool.put(p);
  }
  D.graphs.clear();
  for (double2* p : D.blocks) cx.pool.put(p);
  D.blocks.clear();
  D.rep_host = nullptr;
}

// Columns c0 .. m of the kept Gram matrix G = V^H S (rows 0 .. m), and the
// rows they mirror to (G is Hermitian up to the rounding of S, and only its
// Hermitian part is diagonalised): after the sigma build of rows c0 .. m.
void devdav_gram_cols(Ctx& cx, DevDav& D, const double2* V, const double2* S, int c0, int m) {
  if (m <= c0) return;
  gram_dev(cx, V, m, S + (int64_t)c0 * D.dim, m - c0, D.dim, D.gpart, D.gstage, D.G + c0, D.mmax);
  launch_gram_mirror(D.G, D.mmax, c0, m, cx.stream);
}

// One iteration from the subspace V, S (m rows, Gram matrix G) to the new
// directions in N:
//  eigenpairs of G; Ritz vectors X = U_k^T V, AX = U_k^T S;
//  residuals R = AX - w X, their norms and the convergence test (report);
//  N = Olsen-corrected preconditioned residuals, zero for converged roots;
//  collapse of V, S onto the 2k lowest Ritz vectors when the subspace cannot
//  take one direction per unconverged root (the host-driven rule);
//  N orthonormalised against V and among themselves (two passes of
//  projection and canonical orthonormalisation; kept directions first, their
//  count in the report).
void devdav_body(Ctx& cx, const Inst& I, DevDav& D, double2* V, double2* S, double2* X, double2* AX, double2* R,
                 int m) {
  const int k = D.k;
  const int64_t dim = D.dim;
  hipStream_t s = cx.stream;
  launch_heev_jacobi(D.G, D.mmax, m, D.Aw, D.Vw, D.mode(m), D.U, m, D.w, s);
  combine_dev(cx, D.U, m, m, k, V, X, dim, C1(), C0());
  combine_dev(cx, D.U, m, m, k, S, AX, dim, C1(), C0());
  launch_resid(AX, X, D.w, R, k, dim, s);
  launch_row_dots(R, dim, R, dim, k, dim, D.rpart, D.nb, s);
  launch_row_sums(D.rpart, D.nb, k, D.rn2, s);
  launch_dav_converge(D.w, D.rn2, D.wold, k, m, D.mmax, D.par, D.rep, s);
  // Olsen's correction t = P (r - e x), e = <x|P r> / <x|P x>, P = (w - D)^-1
  const SinglesPrecond& SP = *D.sp;
  precond_coeffs(cx, SP, R, D.w, k, dim);
  launch_precondition(R, D.N, I.diag, D.w, k, dim, s);
  precond_store(cx, SP, D.N, k, dim);
  precond_coeffs(cx, SP, X, D.w, k, dim);
  launch_precondition(X, D.T, I.diag, D.w, k, dim, s);
  precond_store(cx, SP, D.T, k, dim);
  launch_row_dots(X, dim, D.N, dim, k, dim, D.rpart, D.nb, s);
  launch_row_sums(D.rpart, D.nb, k, D.ra, s);
  launch_row_dots(X, dim, D.T, dim, k, dim, D.rpart, D.nb, s);
  launch_row_sums(D.rpart, D.nb, k, D.rb, s);
  launch_olsen(D.N, D.T, D.ra, D.rb, D.rep + 1 + 2 * k, k, dim, s);
  // collapse (decided on the device): rows past the kept 2k become zero, so
  // the projection below may run over all m rows either way
  const double* collapse = D.rep + 3 + 3 * k;
  const int mc = std::min(2 * k, m);
  launch_collapse(collapse, D.U, m, m, mc, V, D.T, V, dim, s);
  launch_collapse(collapse, D.U, m, m, mc, S, D.T, S, dim, s);
  launch_gram_diag(collapse, D.w, mc, D.G, D.mmax, s);
  // the first pass projects N and writes its orthonormal rows to T, the
  // second projects T and writes them back to N
  for (int pass = 0; pass < 2; ++pass) {
    double2* A = pass == 0 ? D.N : D.T;
    double2* B = pass == 0 ? D.T : D.N;
    gram_dev(cx, V, m, A, k, dim, D.gpart, D.gstage, D.Cc, k);  // Cc[a][b] = <V_a|A_b>
    combine_dev(cx, D.Cc, k, m, k, V, A, dim, CR(-1), C1());
    gram_dev(cx, A, k, A, k, dim, D.gpart, D.gstage, D.Gn, k);
    launch_heev_jacobi(D.Gn, k, k, D.Aw, D.Vw, D.mode(k), D.Un, k, D.wn, s);
    launch_canon(D.wn, D.Un, k, k, D.Cc, D.rep + 1 + 3 * k + pass, s);
    combine_dev(cx, D.Cc, k, k, k, A, B, dim, C1(), C0());
  }
}

// Runs the iteration for subspace size m (from its captured graph when
// capture is on, capturing it on first use) and reads the report.
void devdav_step(Ctx& cx, const Inst& I, DevDav& D, bool capture, double2* V, double2* S, double2* X, double2* AX,
                 double2* R, int m) {
  if (!capture || D.capture_off) {
    devdav_body(cx, I, D, V, S, X, AX, R, m);
  } else {
    DevDav::Graph* G = nullptr;
    for (auto& g : D.graphs)
      if (g.m == m) G = &g;
    if (!G) {
      DevDav::Graph ng;
      ng.m = m;
      cx.pool.begin_hold();
      hipError_t e;
      {
        std::shared_lock<std::shared_mutex> gate(capture_gate());
        e = hipStreamBeginCapture(cx.stream, hipStreamCaptureModeRelaxed);
        if (e == hipSuccess) {
          try {
            devdav_body(cx, I, D, V, S, X, AX, R, m);
          } catch (const HipError& err) {
            e = err.e;
          } catch (...) {
            hipGraph_t dead = nullptr;
            (void)hipStreamEndCapture(cx.stream, &dead);
            if (dead) (void)hipGraphDestroy(dead);
            for (double2* p : cx.pool.end_hold()) cx.pool.put(p);
            throw;
          }
          hipGraph_t g = nullptr;
          const hipError_t ee = hipStreamEndCapture(cx.stream, &g);
          if (e == hipSuccess) e = ee;
          if (e == hipSuccess) ng.g = g;
          else if (g) (void)hipGraphDestroy(g);
        }
      }
      ng.held = cx.pool.end_hold();
      if (e == hipSuccess) e = hipGraphInstantiate(&ng.ex, ng.g, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        // no graph: this solve's iterations run launch by launch from now on
        end_failed_capture(cx.stream);
        if (ng.g) (void)hipGraphDestroy(ng.g);
        for (double2* p : ng.held) cx.pool.put(p);
        D.capture_off = true;
        devdav_body(cx, I, D, V, S, X, AX, R, m);
      } else {
        D.graphs.push_back(std::move(ng));
        G = &D.graphs.back();
      }
    }
    if (G) hipcheck(hipGraphLaunch(G->ex, cx.stream), "iteration graph");
  }
  hipcheck(hipMemcpyAsync(D.rep_host, D.rep, sizeof(double) * D.rep_len(), hipMemcpyDeviceToHost, cx.stream),
           "report");
  hipcheck(hipStreamSynchronize(cx.stream), "report sync");
}

int davidson_one(adc_handle* h, Inst& I, const double2* guess, double* omega, double2* vecs, double* resnorm,
                 int* iters, int* conv_out) {
  Ctx& cx = *I.cx;
  const int k = I.k;
  const int64_t dim = I.dim;
  const double tol = h->opt.conv_tol > 0 ? h->opt.conv_tol : 1e-7;
  const int max_iter = h->opt.max_iter > 0 ? h->opt.max_iter : 200;
  int mmax = h->opt.max_subspace > 0 ? h->opt.max_subspace : 6 * k;
  // a collapse keeps 2k vectors and the next iteration adds up to k
  mmax = std::max(mmax, 3 * k);
  if ((int64_t)mmax > dim) mmax = (int)dim;
  if (k > dim) throw Status{ADC_ERR_INVALID_ARG, "n_roots > dim"};
  const int prec_mixed = h->opt.precision;
  int prec = prec_mixed;
  const double tol_mixed = 1e-4;
  // The reduced-precision sweep hands over at 1e-4, or when its largest
  // residual, once below ten times its rounding floor, has not come down by
  // 10% for 15 iterations: the sweep's own rounding puts a floor of about
  // 1e-7 |omega| under the residual (the rounding of M y, |M y| ~ |omega|
  // for a Ritz pair), above 1e-4 for roots beyond ~1000 Eh.  Above 1e-6
  // |omega| a slow stretch is the iteration's own (strongly coupled roots),
  // which the reduced precision still serves, so the window is not armed
  double best_res = 1e300;
  int best_it = 0;
  auto mixed_stalled = [&](const std::vector<double>& rv, const std::vector<double>& wv, int itn) {
    double mx = 0.0, wmax = 0.0;
    for (double x : rv) mx = std::max(mx, x);
    for (double x : wv) wmax = std::max(wmax, std::fabs(x));
    if (mx < 0.9 * best_res || mx > 1e-6 * wmax) {
      best_res = mx;
      best_it = itn;
    }
    const bool st = itn - best_it >= 15;
    if (st && h->opt.verbose)
      std::fprintf(stderr, "[adc] it %3d: residual %.1e stalled near the reduced-precision floor, FP64 from here\n",
                   itn, mx);
    return st;
  };
  double2* V = cx.pool.get((int64_t)mmax * dim);
  double2* S = cx.pool.get((int64_t)mmax * dim);
  double2* X = cx.pool.get((int64_t)k * dim);
  double2* AX = cx.pool.get((int64_t)k * dim);
  double2* R = cx.pool.get((int64_t)k * dim);
  double* wd = (double*)cx.pool.get(k);
  int m = 0;
  // default guesses: unit vectors on the lowest diagonal entries of M11, then
  // (more roots than singles) of the doubles' zeroth-order diagonal; the
  // positions in that order, as many as asked for
  auto unit_positions = [&](int want) {
    std::vector<int64_t> pos;
    std::vector<int> idx(I.n1);
    for (int i = 0; i < (int)I.n1; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return I.m11diag[a] < I.m11diag[b]; });
    for (int i = 0; i < (int)I.n1 && (int)pos.size() < want; ++i) pos.push_back(idx[i]);
    if ((int)pos.size() < want) {
      std::vector<double> dd(dim);
      hipcheck(hipMemcpyAsync(dd.data(), I.diag, sizeof(double) * dim, hipMemcpyDeviceToHost, cx.stream), "dd");
      hipcheck(hipStreamSynchronize(cx.stream), "dd sync");
      std::vector<int64_t> id2(dim - I.n1);
      for (int64_t i = 0; i < (int64_t)id2.size(); ++i) id2[i] = I.n1 + i;
      std::stable_sort(id2.begin(), id2.end(), [&](int64_t a, int64_t b) { return dd[a] < dd[b]; });
      for (size_t i = 0; i < id2.size() && (int)pos.size() < want; ++i) pos.push_back(id2[i]);
    }
    return pos;
  };
  auto put_units = [&](double2* dst, const std::vector<int64_t>& pos) {
    launch_fill(dst, (int64_t)pos.size() * dim, C0(), cx.stream);
    const double2 one = make_double2(1.0, 0.0);
    for (size_t r = 0; r < pos.size(); ++r)
      hipcheck(hipMemcpyAsync(dst + (int64_t)r * dim + pos[r], &one, sizeof(double2), hipMemcpyHostToDevice,
                              cx.stream), "unit");
    hipcheck(hipStreamSynchronize(cx.stream), "unit sync");
  };
  if (guess) {
    hipcheck(hipMemcpyAsync(V, guess, sizeof(double2) * k * dim, hipMemcpyDeviceToDevice, cx.stream), "guess");
    m = orthonormalize(cx, V, 0, V, k, dim);
    // a guess of lower rank (repeated or zero rows) is topped up with the
    // default unit vectors that are not in its span, lowest diagonal first
    if (m < k) {
      const auto pos = unit_positions((int)std::min<int64_t>(dim, 3 * (int64_t)k + 8));
      double2* T = cx.pool.get((int64_t)pos.size() * dim);
      put_units(T, pos);
      const int nt = orthonormalize(cx, V, m, T, (int)pos.size(), dim);
      const int take = std::min(k - m, nt);
      if (take > 0)
        hipcheck(hipMemcpyAsync(V + (int64_t)m * dim, T, sizeof(double2) * take * dim, hipMemcpyDeviceToDevice,
                                cx.stream), "top up");
      hipcheck(hipStreamSynchronize(cx.stream), "top up sync");
      cx.pool.put(T);
      m += take;
      if (m < k) throw Status{ADC_ERR_INVALID_ARG, "guess spans fewer than n_roots directions"};
    }
  } else {
    put_units(V, unit_positions(k));
    m = k;
  }
  auto now = []() { return std::chrono::steady_clock::now(); };
  auto ms_since = [](std::chrono::steady_clock::time_point t) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
  };
  double t_sigma = 0.0, t_sub = 0.0, t_orth = 0.0;
  {
    auto t0 = now();
    sigma_call(h, I, V, S, m, prec);
    hipcheck(hipStreamSynchronize(cx.stream), "sigma sync");
    t_sigma += ms_since(t0);
  }
  std::vector<double> w_old(k, 1e300), w(k), rn(k);
  std::vector<int> conv(k, 0);
  std::vector<int> sel(k);
  // root following (a given start block, root_follow set): the start vectors
  // are the references every iteration's Ritz vectors are matched against
  double2* Gref = nullptr;
  if (guess && h->opt.root_follow) {
    Gref = cx.pool.get((int64_t)k * dim);
    hipcheck(hipMemcpyAsync(Gref, V, sizeof(double2) * k * dim, hipMemcpyDeviceToDevice, cx.stream), "ref");
  }
  int it = 0;
  // refine_fp64 < 0: a mixed-precision solve iterates to conv_tol in its own
  // precision and reports its own residuals (no FP64 restart)
  const bool refine = h->opt.refine_fp64 >= 0;
  bool refined_phase = (prec == 0) || !refine;
  // device-side iteration (graphs on, no root following); graphs = 2 runs
  // it launch by launch instead of from captured graphs
  const bool dev_iter = h->opt.graphs && !Gref && mmax <= heev_device_max();
  // the singles-block preconditioner, declared before the device iteration so
  // that the graphs which use its buffers are released first; without memory
  // for it the solve keeps the diagonal
  SinglesPrecond SP;
  struct SPGuard {
    Ctx& cx;
    SinglesPrecond& P;
    ~SPGuard() {
      (void)hipStreamSynchronize(cx.stream);
      precond_release(cx, P);
    }
  } sp_guard{cx, SP};
  try {
    precond_setup(h, I, SP, k);
  } catch (const HipError&) {
    (void)hipGetLastError();
    precond_release(cx, SP);
  }
  DevDav D;
  D.sp = &SP;
  struct DevGuard {
    Ctx& cx;
    DevDav& D;
    ~DevGuard() { devdav_release(cx, D); }
  } dev_guard{cx, D};
  auto reset_wold = [&]() { launch_fill((double2*)D.wold, k, {1e300, 1e300}, cx.stream); };
  if (dev_iter) {
    devdav_setup(cx, D, k, mmax, dim);
    reset_wold();
    devdav_gram_cols(cx, D, V, S, 0, m);
  }
  for (it = 1; it <= max_iter && dev_iter; ++it) {
    auto t_it = now();
    const double tol_now = refined_phase ? tol : std::max(tol, tol_mixed);
    const double dw_tol = refined_phase ? std::max(1e-10, tol * tol) : 1e-7;
    double* par_host = D.rep_host + D.rep_len();
    par_host[0] = tol_now;
    par_host[1] = dw_tol;
    hipcheck(hipMemcpyAsync(D.par, par_host, sizeof(double) * 2, hipMemcpyHostToDevice, cx.stream), "par");
    devdav_step(cx, I, D, h->opt.graphs == 1, V, S, X, AX, R, m);
    const double* rp = D.rep_host;
    if (rp[0] < 0 || rp[1 + 3 * k] < 0 || rp[2 + 3 * k] < 0)
      throw Status{ADC_ERR_NONFINITE_INPUT, "non-finite subspace matrix"};
    const bool all = rp[0] == 1.0;
    for (int r = 0; r < k; ++r) {
      w[r] = rp[1 + r];
      rn[r] = rp[1 + k + r];
      conv[r] = rp[1 + 2 * k + r] != 0.0 ? 1 : 0;
    }
    const int nk = (int)rp[2 + 3 * k];
    if (rp[3 + 3 * k] != 0.0) m = std::min(2 * k, m);  // the step collapsed the subspace
    t_sub += ms_since(t_it);
    if (h->opt.verbose) {
      std::fprintf(stderr, "[adc] it %3d m %3d prec %d dev (sigma %.0f sub %.0f ms)", it, m, prec, t_sigma, t_sub);
      for (int r = 0; r < k; ++r) std::fprintf(stderr, "  %.10f (%.1e)", w[r], rn[r]);
      std::fprintf(stderr, "\n");
    }
    const bool stalled = !refined_phase && mixed_stalled(rn, w, it);
    if (all || nk == 0 || stalled) {
      if (!refined_phase) {
        // mixed precision converged (or out of directions, or stalled):
        // restart from the Ritz vectors in FP64
        refined_phase = true;
        prec = 0;
        hipcheck(hipMemcpyAsync(V, X, sizeof(double2) * k * dim, hipMemcpyDeviceToDevice, cx.stream), "restart");
        m = orthonormalize(cx, V, 0, V, k, dim);
        sigma_call(h, I, V, S, m, prec);
        devdav_gram_cols(cx, D, V, S, 0, m);
        reset_wold();
        continue;
      }
      if (!all)
        for (int r = 0; r < k; ++r) conv[r] = rn[r] <= tol_now ? 1 : 0;
      break;
    }
    hipcheck(hipMemcpyAsync(V + (int64_t)m * dim, D.N, sizeof(double2) * nk * dim, hipMemcpyDeviceToDevice,
                            cx.stream), "append");
    auto t_s = now();
    sigma_call(h, I, V + (int64_t)m * dim, S + (int64_t)m * dim, nk, prec);
    if (h->opt.verbose) hipcheck(hipStreamSynchronize(cx.stream), "sigma sync");
    t_sigma += ms_since(t_s);
    devdav_gram_cols(cx, D, V, S, m, m + nk);
    m += nk;
  }
  for (it = dev_iter ? it : 1; it <= max_iter && !dev_iter; ++it) {
    auto t_it = now();
    auto G = gram(cx, V, m, S, m, dim);
    for (int a = 0; a < m; ++a)
      for (int b = a; b < m; ++b) {
        const zc x = 0.5 * (G[(size_t)a * m + b] + std::conj(G[(size_t)b * m + a]));
        G[(size_t)a * m + b] = x;
        G[(size_t)b * m + a] = std::conj(x);
      }
    std::vector<double> wall;
    std::vector<zc> U;
    heevj(m, G, wall, U);
    // root r: the r-th lowest Ritz pair, or (root following) the one with the
    // largest overlap with start vector r among those not yet taken
    for (int r = 0; r < k; ++r) sel[r] = r;
    if (Gref) {
      const auto O = gram(cx, V, m, Gref, k, dim);  // O[a][r] = <V_a|g_r>
      std::vector<char> used(m, 0);
      for (int r = 0; r < k; ++r) {
        int best = -1;
        double bo = -1.0;
        for (int j = 0; j < m; ++j) {
          if (used[j]) continue;
          zc s = 0.0;
          for (int a = 0; a < m; ++a) s += std::conj(U[(size_t)a * m + j]) * O[(size_t)a * k + r];
          if (std::norm(s) > bo) {
            bo = std::norm(s);
            best = j;
          }
        }
        sel[r] = best;
        used[best] = 1;
      }
    }
    std::vector<zc> Uk((size_t)m * k);
    for (int a = 0; a < m; ++a)
      for (int r = 0; r < k; ++r) Uk[(size_t)a * k + r] = U[(size_t)a * m + sel[r]];
    combine(cx, Uk, m, k, V, X, dim, C1(), C0());
    combine(cx, Uk, m, k, S, AX, dim, C1(), C0());
    for (int r = 0; r < k; ++r) w[r] = wall[sel[r]];
    hipcheck(hipMemcpyAsync(wd, w.data(), sizeof(double) * k, hipMemcpyHostToDevice, cx.stream), "w");
    launch_resid(AX, X, wd, R, k, dim, cx.stream);
    auto r2 = row_norms2(cx, R, k, dim);
    bool all = true;
    // |d omega| between iterations: 1e-10 Eh, or tol^2 when that is looser
    // (the eigenvalue error of a residual r is at most |r|^2 / gap)
    const double tol_now = refined_phase ? tol : std::max(tol, tol_mixed);
    const double dw_tol = refined_phase ? std::max(1e-10, tol * tol) : 1e-7;
    for (int r = 0; r < k; ++r) {
      rn[r] = std::sqrt(std::max(0.0, r2[r]));
      conv[r] = (rn[r] <= tol_now && std::fabs(w[r] - w_old[r]) <= dw_tol) ? 1 : 0;
      all = all && conv[r];
    }
    t_sub += ms_since(t_it);
    if (h->opt.verbose) {
      std::fprintf(stderr, "[adc] it %3d m %3d prec %d (sigma %.0f sub %.0f orth %.0f ms)", it, m, prec, t_sigma,
                   t_sub, t_orth);
      for (int r = 0; r < k; ++r) std::fprintf(stderr, "  %.10f (%.1e)", w[r], rn[r]);
      std::fprintf(stderr, "\n");
    }
    w_old = w;
    const bool stalled = !refined_phase && mixed_stalled(rn, w, it);
    if (all || stalled) {
      if (refined_phase) break;
      // mixed precision converged (or stalled): restart from the Ritz
      // vectors in FP64
      refined_phase = true;
      prec = 0;
      hipcheck(hipMemcpyAsync(V, X, sizeof(double2) * k * dim, hipMemcpyDeviceToDevice, cx.stream), "restart");
      m = orthonormalize(cx, V, 0, V, k, dim);
      sigma_call(h, I, V, S, m, prec);
      std::fill(w_old.begin(), w_old.end(), 1e300);
      continue;
    }
    // new directions
    std::vector<int> un;
    for (int r = 0; r < k; ++r)
      if (!conv[r]) un.push_back(r);
    const int nn = (int)un.size();
    double2* Nd = cx.pool.get((int64_t)nn * dim);
    double* wn = (double*)cx.pool.get(nn);
    std::vector<double> wv(nn);
    for (int j = 0; j < nn; ++j) {
      wv[j] = w[un[j]];
      hipcheck(hipMemcpyAsync(Nd + (int64_t)j * dim, R + (int64_t)un[j] * dim, sizeof(double2) * dim,
                              hipMemcpyDeviceToDevice, cx.stream), "N");
    }
    hipcheck(hipMemcpyAsync(wn, wv.data(), sizeof(double) * nn, hipMemcpyHostToDevice, cx.stream), "wn");
    precond_coeffs(cx, SP, Nd, wn, nn, dim);
    launch_precondition(Nd, Nd, I.diag, wn, nn, dim, cx.stream);
    precond_store(cx, SP, Nd, nn, dim);
    {
      // Olsen's correction t = P (r - e x), e = <x|P r> / <x|P x>, P = (w - D)^-1:
      // keeps the new direction out of the span of the Ritz vector x when
      // M is close to its diagonal
      double2* Xu = cx.pool.get((int64_t)nn * dim);
      double2* Xp = cx.pool.get((int64_t)nn * dim);
      for (int j = 0; j < nn; ++j)
        hipcheck(hipMemcpyAsync(Xu + (int64_t)j * dim, X + (int64_t)un[j] * dim, sizeof(double2) * dim,
                                hipMemcpyDeviceToDevice, cx.stream), "Xu");
      precond_coeffs(cx, SP, Xu, wn, nn, dim);
      launch_precondition(Xu, Xp, I.diag, wn, nn, dim, cx.stream);
      precond_store(cx, SP, Xp, nn, dim);
      const auto a = row_dots(cx, Xu, Nd, nn, dim);
      const auto b = row_dots(cx, Xu, Xp, nn, dim);
      for (int j = 0; j < nn; ++j) {
        if (std::abs(b[j]) < 1e-300) continue;
        const zc e = a[j] / b[j];
        const int64_t od[1] = {dim}, st[1] = {1};
        launch_permute(1, od, st, st, Xp + (int64_t)j * dim, Nd + (int64_t)j * dim, {-e.real(), -e.imag()}, C1(), 0,
                       cx.stream);
      }
      cx.pool.put(Xu);
      cx.pool.put(Xp);
    }
    if (m + nn > mmax) {
      // collapse onto the 2k lowest Ritz vectors of the current subspace
      // (with root following: the followed ones first, then the lowest)
      const int mc = std::min(2 * k, m);
      std::vector<int> keep(sel.begin(), sel.end());
      for (int j = 0; j < m && (int)keep.size() < mc; ++j)
        if (std::find(keep.begin(), keep.end(), j) == keep.end()) keep.push_back(j);
      std::vector<zc> Uc((size_t)m * mc);
      for (int a = 0; a < m; ++a)
        for (int r = 0; r < mc; ++r) Uc[(size_t)a * mc + r] = U[(size_t)a * m + keep[r]];
      double2* T = cx.pool.get((int64_t)mc * dim);
      combine(cx, Uc, m, mc, V, T, dim, C1(), C0());
      hipcheck(hipMemcpyAsync(V, T, sizeof(double2) * mc * dim, hipMemcpyDeviceToDevice, cx.stream), "col");
      combine(cx, Uc, m, mc, S, T, dim, C1(), C0());
      hipcheck(hipMemcpyAsync(S, T, sizeof(double2) * mc * dim, hipMemcpyDeviceToDevice, cx.stream), "col");
      hipcheck(hipStreamSynchronize(cx.stream), "col sync");
      cx.pool.put(T);
      m = mc;
    }
    auto t_o = now();
    const int nk = orthonormalize(cx, V, m, Nd, nn, dim);
    t_orth += ms_since(t_o);
    if (nk > 0) {
      hipcheck(hipMemcpyAsync(V + (int64_t)m * dim, Nd, sizeof(double2) * nk * dim, hipMemcpyDeviceToDevice,
                              cx.stream), "app");
      auto t_s = now();
      sigma_call(h, I, V + (int64_t)m * dim, S + (int64_t)m * dim, nk, prec);
      hipcheck(hipStreamSynchronize(cx.stream), "sigma sync");
      t_sigma += ms_since(t_s);
      m += nk;
    }
    cx.pool.put(Nd);
    cx.pool.put((double2*)wn);
    if (nk == 0) {
      // no direction is left outside the subspace (it is invariant, e.g. the
      // whole space of a tiny instance): the Ritz pairs are final, after an
      // FP64 pass when the sweep ran in mixed precision
      if (!refined_phase) {
        refined_phase = true;
        prec = 0;
        hipcheck(hipMemcpyAsync(V, X, sizeof(double2) * k * dim, hipMemcpyDeviceToDevice, cx.stream), "restart");
        m = orthonormalize(cx, V, 0, V, k, dim);
        sigma_call(h, I, V, S, m, prec);
        std::fill(w_old.begin(), w_old.end(), 1e300);
        continue;
      }
      for (int r = 0; r < k; ++r) conv[r] = rn[r] <= tol_now ? 1 : 0;
      break;
    }
  }
  for (int r = 0; r < k; ++r) {
    omega[r] = w[r];
    resnorm[r] = rn[r];
    conv_out[r] = conv[r];
  }
  *iters = std::min(it, max_iter);
  if (vecs) hipcheck(hipMemcpyAsync(vecs, X, sizeof(double2) * k * dim, hipMemcpyDeviceToDevice, cx.stream), "vecs");
  hipcheck(hipStreamSynchronize(cx.stream), "dav end");
  for (double2* p : {V, S, X, AX, R}) cx.pool.put(p);
  if (Gref) cx.pool.put(Gref);
  cx.pool.put((double2*)wd);
  for (int r = 0; r < k; ++r)
    if (!conv[r]) return ADC_NOT_CONVERGED;
  return ADC_OK;
}

// ============================================================================
// adjoint of the sigma build
// ============================================================================
// Reverse rule of the particle-particle ladder S[z][r][ab] += alpha sum_{c<d}
// <ab||cd> Y[z][r][cd], with <ab||cd> = sum_Q (L_ac L_bd - L_ad L_bc):
//  * Y: the packed <ab||cd> matrix is Hermitian, so G_Y += conj(alpha) ladder(G_S);
//  * L_vv: with Gamma[ab][cd] = alpha sum_{z,r} conj(G_S[z][r][ab]) Y[z][r][cd]
//    and its extension G4[a][b][c][d] = sign(b-a) sign(d-c) Gamma[pair(a,b)][pair(c,d)]
//    (zero on a==b or c==d), G_L[Q][a][c] += sum_{b,d} conj(G4[a][b][c][d] L[Q][b][d]).
//    G4 is formed per block of a from Gamma and contracted at once (never stored whole).
void ladder_backward(Ctx& cx, const TapeOp& op, const double2* gS, double2* gY) {
  adc_handle* h = (adc_handle*)op.owner;
  Inst& I = *(Inst*)op.inst;
  const int v = I.v;
  const int64_t Pv = I.Pv, N = I.N;
  const int64_t ldY = op.n[0], offY = op.n[1], ldS = op.n[2], offS = op.n[3], nrow = op.n[4];
  const int k = (int)op.n[5];
  if (Pv == 0 || nrow == 0 || k == 0) return;
  if (gY) ladder(h, I, gS, ldS, offS, gY, ldY, offY, nrow, k, {op.alpha.re, -op.alpha.im}, op.prec);
  Tensor Gam = tnew(cx, {Pv, Pv}, false);
  {
    Tensor gSv = tensor_view(const_cast<double2*>(gS) + offS, {k, nrow, Pv}, {ldS, Pv, 1});
    Tensor Yv = tensor_view(op.A.p + offY, {k, nrow, Pv}, {ldY, Pv, 1});
    ctr(cx, op.alpha, gSv, "zrp", true, Yv, "zrq", false, C0(), Gam, "pq");
  }
  Tensor GL = grad_view(cx, I.Lvv);
  const size_t budget = h->opt.mem_budget ? h->opt.mem_budget : (size_t)4 << 30;
  int64_t nx = std::max<int64_t>(1, (int64_t)(budget / 2 / sizeof(double2)) / ((int64_t)v * v * v));
  nx = std::min<int64_t>(nx, v);
  Tensor G4 = tnew(cx, {nx, v, v, v}, false);
  for (int64_t x0 = 0; x0 < v; x0 += nx) {
    const int64_t x1 = std::min<int64_t>(v, x0 + nx);
    launch_expand_gamma(Gam.p, Pv, (int)x0, (int)x1, v, G4.p, cx.stream);
    Tensor Gs = tslice(G4, 0, 0, x1 - x0);
    Tensor GLs = tslice(GL, 1, x0, x1);
    ctr(cx, C1(), Gs, "xybd", true, I.Lvv, "Qbd", true, C1(), GLs, "Qxy");
  }
  tfree(cx, G4);
  tfree(cx, Gam);
  (void)N;
}

void inst_release_derived(Ctx& cx, Inst& J) {
  for (Tensor* t : {&J.oooo, &J.ooov, &J.oovv, &J.ovov, &J.ovvv, &J.ring, &J.t1, &J.M11x, &J.M11b, &J.W, &J.W5,
                    &J.W6, &J.E0, &J.E1, &J.X1, &J.X2})
    if (t->p) tfree(cx, *t);
}

// f = Re sum_z Sbar_z^H M(L, x) Y_z.  dL (device, [N][n][n]) receives the
// Hermitian-projected G_L; *dx = f(x + 1) - f(x) (M is affine in x).
void sigma_backward(adc_handle* h, Inst& I, const double2* Sbar, const double2* Y, int k, double2* dL, double* dx) {
  Ctx& cx = *I.cx;
  const int o = I.o, v = I.v, n = o + v, N = I.N;
  const int64_t dim = I.dim;
  const int saved_prec = cx.prec;
  cx.prec = 0;
  hipcheck(hipStreamSynchronize(cx.stream), "bw sync");
  if (dx) {
    Tensor S0 = tnew(cx, {k, dim}, false), S1 = tnew(cx, {k, dim}, false);
    sigma_dispatch(h, I, Y, S0.p, k, 0);
    Tensor Mx = tnew(cx, {I.n1, I.n1}, false);
    perm(cx, C1(), I.M11x, "pq", false, C0(), Mx, "pq");
    perm(cx, C1(), I.M11b, "pq", false, C1(), Mx, "pq");
    std::swap(I.M11x, Mx);
    const double x0 = I.x;
    // the singles-coupling factors at x + 1 (the frozen ones stay untouched)
    Tensor X1b, X2b, X1hb, X2hb;
    build_sx(cx, I, x0 + 1.0, X1b, X2b, I.X1h.p ? &X1hb : nullptr, I.X2h.p ? &X2hb : nullptr);
    auto swap_all = [&]() {
      std::swap(I.X1, X1b);
      std::swap(I.X2, X2b);
      std::swap(I.X1h, X1hb);
      std::swap(I.X2h, X2hb);
    };
    swap_all();
    auto restore = [&]() {
      I.x = x0;
      std::swap(I.M11x, Mx);
      swap_all();
    };
    I.x = x0 + 1.0;
    try {
      sigma_dispatch(h, I, Y, S1.p, k, 0);
    } catch (...) {
      restore();
      throw;
    }
    restore();
    tfree(cx, Mx);
    for (Tensor* t : {&X1b, &X2b, &X1hb, &X2hb})
      if (t->p) tfree(cx, *t);
    perm(cx, CR(-1), S0, "zp", false, C1(), S1, "zp");
    Tensor Sb = tensor_view(const_cast<double2*>(Sbar), {1, (int64_t)k * dim}, {});
    Tensor D = tensor_view(S1.p, {(int64_t)k * dim, 1}, {});
    Tensor r = tnew(cx, {1, 1}, false);
    ctr(cx, C1(), Sb, "yp", true, D, "px", false, C0(), r, "yx");
    double2 hv;
    hipcheck(hipMemcpyAsync(&hv, r.p, sizeof(double2), hipMemcpyDeviceToHost, cx.stream), "dx");
    hipcheck(hipStreamSynchronize(cx.stream), "dx sync");
    *dx = hv.x;
    for (Tensor* t : {&S0, &S1, &r}) tfree(cx, *t);
  }
  if (dL) {
    // the one-off part is recorded by the first call and kept (with every
    // buffer it wrote) for the later ones
    const bool fresh = !I.bw;
    if (fresh) I.bw = std::make_shared<BwCache>();
    BwCache& B = *I.bw;
    Tape& T = B.T;
    Inst& J = B.J;
    bool done = false;
    struct Cleanup {
      Ctx& cx;
      Inst& I;
      BwCache& B;
      int prec;
      bool& done;
      ~Cleanup() {
        if (done) {
          // cut the tape back to the one-off part: the sigma part's ops,
          // buffers and postponed frees go, every gradient is dropped
          for (auto& a : B.T.allocs)
            if (a.grad) {
              cx.pool.put(a.grad);
              a.grad = nullptr;
            }
          for (size_t i = B.n_deferred; i < B.T.deferred.size(); ++i) cx.pool.put(B.T.deferred[i]);
          B.T.deferred.resize(B.n_deferred);
          B.T.allocs.resize(B.n_allocs);
          B.T.ops.resize(B.n_ops);
          B.T.recording = false;
          cx.pool.tape = nullptr;
          cx.tape = nullptr;
        } else {
          cx.tape = &B.T;
          tape_release(cx);
          inst_release_derived(cx, B.J);
          I.bw.reset();
        }
        cx.pool.trim();
        cx.prec = prec;
      }
    } cleanup{cx, I, B, saved_prec, done};
    cx.tape = &T;
    cx.pool.tape = &T;
    // a split-bf16 ladder reads the instance's planes of L_vv (the same L_vv)
    if (h->opt.precision == ADC_SPLIT_BF16 && I.kind != ADC_IP) ensure_planes(h, I);
    if (fresh) {
      for (Tensor* leaf : {&I.Loo, &I.Lov, &I.Lvo, &I.Lvv}) {
        T.add(leaf->p, sizeof(double2) * (size_t)leaf->size(), true);
        T.allocs.back().ref = true;
      }
      J.cx = I.cx;
      J.kind = I.kind; J.o = o; J.v = v; J.N = N; J.k = I.k; J.x = I.x;
      J.n1 = I.n1; J.n2 = I.n2; J.dim = dim; J.Po = I.Po; J.Pv = I.Pv;
      J.eps = I.eps; J.Loo = I.Loo; J.Lov = I.Lov; J.Lvo = I.Lvo; J.Lvv = I.Lvv;
      J.pair_o = I.pair_o; J.pair_v = I.pair_v; J.diag = I.diag;
      std::vector<double> eps_h(n);
      hipcheck(hipMemcpy(eps_h.data(), I.eps, sizeof(double) * n, hipMemcpyDeviceToHost), "bw eps");
      T.recording = true;
      init_integrals(h, J);
      {
        Pre P;
        init_amplitudes(h, J, P);
        if (J.kind == ADC_EE) ee_init(h, J, P, eps_h);
        else if (J.kind == ADC_IP) ip_init(h, J, P, eps_h);
        else ea_init(h, J, P, eps_h);
        for (Tensor* q : {&P.Lt, &P.Ht, &P.t2, &P.ts}) tfree(cx, *q);
      }
      T.recording = false;
      B.n_ops = T.ops.size();
      B.n_allocs = T.allocs.size();
      B.n_deferred = T.deferred.size();
    }
    J.Lq = I.Lq;
    J.Kq = I.Kq;
    // fresh copies of the constant operands, so every recorded pointer is tracked
    Tensor Yc = tnew(cx, {k, dim}, false), Sg = tnew(cx, {k, dim}, false);
    hipcheck(hipMemcpyAsync(Yc.p, Y, sizeof(double2) * k * dim, hipMemcpyDeviceToDevice, cx.stream), "bw Y");
    // the sigma part in the handle's arithmetic (its reverse rules follow
    // it); the one-off part above stays FP64, as in adc_init
    T.recording = true;
    sigma_dispatch(h, J, Yc.p, Sg.p, k, h->opt.precision);
    T.recording = false;
    {
      Tensor gS = grad_view(cx, Sg);
      hipcheck(hipMemcpyAsync(gS.p, Sbar, sizeof(double2) * k * dim, hipMemcpyDeviceToDevice, cx.stream), "bw seed");
    }
    tape_backward(cx);
    // gather the four class blocks into [N][n][n], then project onto Hermitian L^Q
    Tensor G = tnew(cx, {N, n, n}, true);
    auto put = [&](Tensor& leaf, int r0, int c0) {
      const int i = T.find(leaf.p);
      if (i < 0 || !T.allocs[i].grad) return;
      Tensor g = grad_view(cx, leaf);
      Tensor dst = tensor_view(G.p + (int64_t)r0 * n + c0, leaf.d, {(int64_t)n * n, n, 1});
      perm(cx, C1(), g, "Qpq", false, C0(), dst, "Qpq");
    };
    put(I.Loo, 0, 0);
    put(I.Lov, 0, o);
    put(I.Lvo, o, 0);
    put(I.Lvv, o, o);
    launch_herm_project(G.p, dL, N, n, cx.stream);
    tfree(cx, G);
    tfree(cx, Yc);
    tfree(cx, Sg);
    hipcheck(hipStreamSynchronize(cx.stream), "bw end");
    done = true;
  }
  cx.prec = saved_prec;
}

// detail of the calling thread's last failed call (adc_last_error)
thread_local std::string g_last_error;

// an early rejection, with its detail for adc_last_error
int reject(int code, const char* msg) {
  g_last_error = msg;
  return code;
}

template <class F>
int guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const Status& s) {
    g_last_error = s.msg ? s.msg : "";
    return s.code;
  } catch (const HipError& e) {
    (void)hipGetLastError();
    g_last_error = std::string(e.where ? e.where : "") + ": " + hipGetErrorString(e.e);
    return e.e == hipErrorOutOfMemory ? ADC_ERR_OUT_OF_MEMORY : ADC_ERR_HIP;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return ADC_ERR_OUT_OF_MEMORY;
  } catch (const std::invalid_argument& e) {
    g_last_error = e.what();
    return ADC_ERR_INVALID_ARG;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return ADC_ERR_HIP;
  } catch (...) {
    g_last_error = "unknown exception";
    return ADC_ERR_HIP;
  }
}

// ============================================================================
// frozen natural spinors (Section 2.4, eqs. 25-31)
// ============================================================================
// The virtual density, its natural spinors and the truncated semicanonical
// basis B; the problem (orbital energies, Cholesky vectors) and optionally a
// vector of the instance's kind carried into that basis.
void fns_build(adc_handle* h, Inst& I, const double2* X, double eta_crit, int* n_vir, double* eps_out,
               double2* L_out, double* eta_out, double2* B_out, double2* X_out) {
  Ctx& cx = *I.cx;
  const int o = I.o, v = I.v, N = I.N;
  const int saved = cx.prec;
  cx.prec = 0;
  // eq. 25: D_ab = 1/2 sum_{ijc} t_ij^ac conj(t_ij^bc)
  Tensor D = tnew(cx, {v, v}, false);
  ctr(cx, CR(0.5), I.t1, "ijac", false, I.t1, "ijbc", true, C0(), D, "ab");
  if (X) {
    // eq. 31: the state's virtual density through the zeroth-order
    // intermediate states, D_ab += <Psi| a+_b a_a |Psi>
    if (I.kind == ADC_EE) {
      Tensor Xs = tensor_view(const_cast<double2*>(X), {o, v}, {});
      ctr(cx, C1(), Xs, "ia", false, Xs, "ib", true, C1(), D, "ab");
      Tensor Ya = tnew(cx, {1, o, o, v, v}, false);
      launch_unpack_doubles(0, X, I.dim, I.n1, 1, o, v, Ya.p, nullptr, cx.stream);
      ctr(cx, CR(0.5), Ya, "zijac", false, Ya, "zijbc", true, C1(), D, "ab");
      tfree(cx, Ya);
    } else {
      Tensor Xs = tensor_view(const_cast<double2*>(X), {1, v}, {});
      ctr(cx, C1(), Xs, "za", false, Xs, "zb", true, C1(), D, "ab");
      Tensor Ya = tnew(cx, {1, o, v, v}, false);
      launch_unpack_doubles(2, X, I.dim, I.n1, 1, o, v, Ya.p, nullptr, cx.stream);
      ctr(cx, C1(), Ya, "zjac", false, Ya, "zjbc", true, C1(), D, "ab");
      tfree(cx, Ya);
    }
  }
  std::vector<double2> hD((size_t)v * v);
  hipcheck(hipMemcpyAsync(hD.data(), D.p, sizeof(double2) * hD.size(), hipMemcpyDeviceToHost, cx.stream), "fns D");
  hipcheck(hipStreamSynchronize(cx.stream), "fns D sync");
  tfree(cx, D);
  // eq. 26: natural spinors (the small Hermitian eigenproblem on the host)
  std::vector<zc> A((size_t)v * v), U;
  for (int a = 0; a < v; ++a)
    for (int b = 0; b < v; ++b) {
      const zc x(hD[(size_t)a * v + b].x, hD[(size_t)a * v + b].y), y(hD[(size_t)b * v + a].x, -hD[(size_t)b * v + a].y);
      A[(size_t)a * v + b] = 0.5 * (x + y);
    }
  std::vector<double> w;
  heevj(v, A, w, U);  // ascending
  // occupations descending; eq. 27: keep eta >= eta_crit
  std::vector<int> kept;
  for (int c = v - 1; c >= 0; --c)
    if (w[c] >= eta_crit) kept.push_back(c);
  if (eta_out)
    for (int c = 0; c < v; ++c) eta_out[c] = w[v - 1 - c];
  const int v2 = (int)kept.size();
  if (v2 < 2) throw Status{ADC_ERR_INVALID_ARG, "eta_crit keeps fewer than two virtual spinors"};
  // eq. 28: F~ = V~^H diag(e_vir) V~
  std::vector<double> ev(v);
  {
    std::vector<double> e(o + v);
    hipcheck(hipMemcpy(e.data(), I.eps, sizeof(double) * (o + v), hipMemcpyDeviceToHost), "fns eps");
    for (int a = 0; a < v; ++a) ev[a] = e[o + a];
    for (int i = 0; i < o; ++i) eps_out[i] = e[i];
  }
  std::vector<zc> F((size_t)v2 * v2);
  for (int p = 0; p < v2; ++p)
    for (int q = 0; q < v2; ++q) {
      zc s = 0.0;
      for (int a = 0; a < v; ++a) s += std::conj(U[(size_t)a * v + kept[p]]) * ev[a] * U[(size_t)a * v + kept[q]];
      F[(size_t)p * v2 + q] = s;
    }
  for (int p = 0; p < v2; ++p)
    for (int q = p + 1; q < v2; ++q) {
      const zc x = 0.5 * (F[(size_t)p * v2 + q] + std::conj(F[(size_t)q * v2 + p]));
      F[(size_t)p * v2 + q] = x;
      F[(size_t)q * v2 + p] = std::conj(x);
    }
  std::vector<double> et;
  std::vector<zc> Z;
  heevj(v2, F, et, Z);  // eq. 29, ascending
  // eq. 30: B = V~ Z~
  std::vector<double2> hB((size_t)v * v2);
  for (int a = 0; a < v; ++a)
    for (int c = 0; c < v2; ++c) {
      zc s = 0.0;
      for (int p = 0; p < v2; ++p) s += U[(size_t)a * v + kept[p]] * Z[(size_t)p * v2 + c];
      hB[(size_t)a * v2 + c] = make_double2(s.real(), s.imag());
    }
  for (int c = 0; c < v2; ++c) eps_out[o + c] = et[c];
  *n_vir = v2;
  Tensor B = tnew(cx, {v, v2}, false);
  hipcheck(hipMemcpyAsync(B.p, hB.data(), sizeof(double2) * hB.size(), hipMemcpyHostToDevice, cx.stream), "fns B");
  if (B_out) hipcheck(hipMemcpyAsync(B_out, B.p, sizeof(double2) * hB.size(), hipMemcpyDeviceToDevice, cx.stream),
                      "fns B out");
  // the Cholesky vectors follow the spinors (eq. 42 with the coefficients C B)
  const int64_t n2 = o + v2;
  auto blk = [&](int r0, int nr, int c0, int nc) {
    return tensor_view(L_out + (int64_t)r0 * n2 + c0, {N, nr, nc}, {n2 * n2, n2, 1});
  };
  {
    Tensor oo = blk(0, o, 0, o), ov = blk(0, o, o, v2), vo = blk(o, v2, 0, o), vv = blk(o, v2, o, v2);
    perm(cx, C1(), I.Loo, "Qij", false, C0(), oo, "Qij");
    ctr(cx, C1(), I.Lov, "Qib", false, B, "bc", false, C0(), ov, "Qic");
    ctr(cx, C1(), B, "ac", true, I.Lvo, "Qaj", false, C0(), vo, "Qcj");
    Tensor T = tnew(cx, {N, v, v2}, false);
    ctr(cx, C1(), I.Lvv, "Qab", false, B, "bd", false, C0(), T, "Qad");
    ctr(cx, C1(), B, "ac", true, T, "Qad", false, C0(), vv, "Qcd");
    tfree(cx, T);
  }
  if (X && X_out) {
    // the vector in the new basis: every virtual index contracted with conj(B)
    int64_t n1b, n2b;
    dims_of(I.kind, o, v2, &n1b, &n2b);
    const int64_t dimb = n1b + n2b;
    if (I.kind == ADC_EE) {
      Tensor Xs = tensor_view(const_cast<double2*>(X), {o, v}, {});
      Tensor Os = tensor_view(X_out, {o, v2}, {});
      ctr(cx, C1(), B, "ac", true, Xs, "ia", false, C0(), Os, "ic");
      Tensor Ya = tnew(cx, {1, o, o, v, v}, false);
      launch_unpack_doubles(0, X, I.dim, I.n1, 1, o, v, Ya.p, nullptr, cx.stream);
      Tensor T1 = tnew(cx, {1, o, o, v, v2}, false), T2 = tnew(cx, {1, o, o, v2, v2}, false);
      ctr(cx, C1(), B, "bd", true, Ya, "zijab", false, C0(), T1, "zijad");
      ctr(cx, C1(), B, "ac", true, T1, "zijad", false, C0(), T2, "zijcd");
      // pack (i<j, c<d) of the antisymmetric result
      std::vector<int2> po = pair_table(o), pv = pair_table(v2);
      int2* dpo = (int2*)cx.pool.get(((int64_t)std::max<size_t>(1, po.size()) + 1) / 2);
      int2* dpv = (int2*)cx.pool.get(((int64_t)std::max<size_t>(1, pv.size()) + 1) / 2);
      if (!po.empty()) hipcheck(hipMemcpyAsync(dpo, po.data(), sizeof(int2) * po.size(), hipMemcpyHostToDevice, cx.stream), "po");
      if (!pv.empty()) hipcheck(hipMemcpyAsync(dpv, pv.data(), sizeof(int2) * pv.size(), hipMemcpyHostToDevice, cx.stream), "pv");
      // (the kernel reads eps even without a diagonal term: the instance's
      // energies cover the indices below o + v2 <= o + v)
      launch_pack_doubles(0, T2.p, X_out, nullptr, dimb, n1b, 1, o, v2, I.eps, C1(), 0, dpo, dpv, cx.stream);
      hipcheck(hipStreamSynchronize(cx.stream), "fns pack sync");
      cx.pool.put((double2*)dpo);
      cx.pool.put((double2*)dpv);
      for (Tensor* t : {&Ya, &T1, &T2}) tfree(cx, *t);
    } else {
      Tensor Xs = tensor_view(const_cast<double2*>(X), {v}, {});
      Tensor Os = tensor_view(X_out, {v2}, {});
      ctr(cx, C1(), B, "ac", true, Xs, "a", false, C0(), Os, "c");
      Tensor Ya = tnew(cx, {1, o, v, v}, false);
      launch_unpack_doubles(2, X, I.dim, I.n1, 1, o, v, Ya.p, nullptr, cx.stream);
      Tensor T1 = tnew(cx, {1, o, v, v2}, false), T2 = tnew(cx, {1, o, v2, v2}, false);
      ctr(cx, C1(), B, "bd", true, Ya, "zjab", false, C0(), T1, "zjad");
      ctr(cx, C1(), B, "ac", true, T1, "zjad", false, C0(), T2, "zjcd");
      std::vector<int2> pv = pair_table(v2);
      int2* dpv = (int2*)cx.pool.get(((int64_t)pv.size() + 1) / 2);
      hipcheck(hipMemcpyAsync(dpv, pv.data(), sizeof(int2) * pv.size(), hipMemcpyHostToDevice, cx.stream), "pv");
      launch_pack_doubles(2, T2.p, X_out, nullptr, dimb, n1b, 1, o, v2, I.eps, C1(), 0, I.pair_o, dpv, cx.stream);
      hipcheck(hipStreamSynchronize(cx.stream), "fns pack sync");
      cx.pool.put((double2*)dpv);
      for (Tensor* t : {&Ya, &T1, &T2}) tfree(cx, *t);
    }
  }
  hipcheck(hipStreamSynchronize(cx.stream), "fns end");
  tfree(cx, B);
  cx.prec = saved;
}

// ============================================================================
// ISR one-particle properties of EE states (Section 2.2)
// ============================================================================
// rho^{0->K} = Y^* f through first order and rho^K = Y^* g(0) Y + rho_GS(2)
// for k normalised EE vectors (the rows of Y are normalised here first), as
// [k][n][n] blocks; optionally D_K = sum d_pq rho^K_pq and T_K = sum d_pq
// rho^{0->K}_pq for a one-particle operator d [n][n].
void props_build(adc_handle* h, Inst& I, const double2* Y, int k, double2* rho, double2* tdm, const double2* d,
                 double* dk, double* tk) {
  (void)h;
  Ctx& cx = *I.cx;
  const int o = I.o, v = I.v, n = o + v;
  const int64_t dim = I.dim, nn = (int64_t)n * n;
  const int saved = cx.prec;
  cx.prec = 0;
  // normalised copy of the vectors
  Tensor Yn = tnew(cx, {k, dim}, false);
  {
    const auto nr = row_norms2(cx, Y, k, dim);
    for (int z = 0; z < k; ++z) {
      const double s = nr[z] > 0.0 ? 1.0 / std::sqrt(nr[z]) : 0.0;
      const int64_t od[1] = {dim}, st[1] = {1};
      launch_permute(1, od, st, st, Y + (int64_t)z * dim, Yn.p + (int64_t)z * dim, CR(s), C0(), 0, cx.stream);
    }
  }
  Tensor Ys = tensor_view(Yn.p, {k, o, v}, {dim, v, 1});
  Tensor Ya = tnew(cx, {k, o, o, v, v}, false);
  launch_unpack_doubles(0, Yn.p, dim, I.n1, k, o, v, Ya.p, nullptr, cx.stream);
  auto blk = [&](double2* base, int r0, int nr, int c0, int nc) {
    return tensor_view(base + (int64_t)r0 * n + c0, {k, nr, nc}, {nn, n, 1});
  };
  Tensor tdm_t, rho_t;
  if (tdm || tk) {
    tdm_t = tnew(cx, {k, n, n}, true);
    Tensor vo = blk(tdm_t.p, o, v, 0, o), ov = blk(tdm_t.p, 0, o, o, v), vv = blk(tdm_t.p, o, v, o, v),
           oo = blk(tdm_t.p, 0, o, 0, o);
    perm(cx, C1(), Ys, "zia", true, C0(), vo, "zai");
    ctr(cx, C1(), Ys, "zia", true, I.t1, "ijab", false, C0(), ov, "zjb");
    ctr(cx, CR(0.5), Ya, "zijcb", true, I.t1, "ijdb", false, C0(), vv, "zcd");
    ctr(cx, CR(-0.5), Ya, "zljab", true, I.t1, "kjab", false, C0(), oo, "zkl");
  }
  if (rho || dk) {
    rho_t = tnew(cx, {k, n, n}, true);
    Tensor vo = blk(rho_t.p, o, v, 0, o), ov = blk(rho_t.p, 0, o, o, v), vv = blk(rho_t.p, o, v, o, v),
           oo = blk(rho_t.p, 0, o, 0, o);
    ctr(cx, C1(), Ys, "zic", true, Ys, "zid", false, C0(), vv, "zcd");
    ctr(cx, CR(0.5), Ya, "zijce", true, Ya, "zijde", false, C1(), vv, "zcd");
    ctr(cx, CR(-1.0), Ys, "zla", true, Ys, "zka", false, C0(), oo, "zkl");
    ctr(cx, CR(-0.5), Ya, "zljab", true, Ya, "zkjab", false, C1(), oo, "zkl");
    ctr(cx, C1(), Ys, "zia", true, Ya, "zikad", false, C0(), ov, "zkd");
    perm(cx, C1(), ov, "zkd", true, C0(), vo, "zdk");
    // the ground-state correlation density rho_GS(2), added to every state
    // together with the occupied identity (unit-norm vectors)
    Tensor G = tnew(cx, {n, n}, true);
    Tensor gvv = tensor_view(G.p + (int64_t)o * n + o, {v, v}, {n, 1});
    Tensor goo = tensor_view(G.p, {o, o}, {n, 1});
    Tensor gov = tensor_view(G.p + o, {o, v}, {n, 1});
    Tensor gvo = tensor_view(G.p + (int64_t)o * n, {v, o}, {n, 1});
    ctr(cx, CR(0.5), I.t1, "ijcb", true, I.t1, "ijdb", false, C0(), gvv, "cd");
    ctr(cx, CR(-0.5), I.t1, "ljab", true, I.t1, "kjab", false, C0(), goo, "kl");
    perm(cx, C1(), I.ts, "kd", false, C0(), gov, "kd");
    perm(cx, C1(), I.ts, "kd", true, C0(), gvo, "dk");
    std::vector<double> one(n, 0.0);
    for (int i = 0; i < o; ++i) one[i] = 1.0;
    double* dd = (double*)cx.pool.get((n + 1) / 2);
    hipcheck(hipMemcpyAsync(dd, one.data(), sizeof(double) * n, hipMemcpyHostToDevice, cx.stream), "props diag");
    launch_add_diag(G.p, dd, n, cx.stream);
    for (int z = 0; z < k; ++z) {
      Tensor Rz = tensor_view(rho_t.p + (int64_t)z * nn, {n, n}, {});
      perm(cx, C1(), G, "pq", false, C1(), Rz, "pq");
    }
    hipcheck(hipStreamSynchronize(cx.stream), "props diag sync");
    cx.pool.put((double2*)dd);
    tfree(cx, G);
  }
  auto contract_d = [&](const Tensor& R, double* out) {
    Tensor dv = tensor_view(const_cast<double2*>(d), {1, n, n}, {});
    Tensor r = tnew(cx, {1, k}, false);
    ctr(cx, C1(), dv, "ypq", false, R, "zpq", false, C0(), r, "yz");
    std::vector<double2> hv(k);
    hipcheck(hipMemcpyAsync(hv.data(), r.p, sizeof(double2) * k, hipMemcpyDeviceToHost, cx.stream), "props d");
    hipcheck(hipStreamSynchronize(cx.stream), "props d sync");
    for (int z = 0; z < k; ++z) {
      out[2 * z] = hv[z].x;
      out[2 * z + 1] = hv[z].y;
    }
    tfree(cx, r);
  };
  if (d && dk) contract_d(rho_t, dk);
  if (d && tk) contract_d(tdm_t, tk);
  if (rho) hipcheck(hipMemcpyAsync(rho, rho_t.p, sizeof(double2) * k * nn, hipMemcpyDeviceToDevice, cx.stream), "rho");
  if (tdm) hipcheck(hipMemcpyAsync(tdm, tdm_t.p, sizeof(double2) * k * nn, hipMemcpyDeviceToDevice, cx.stream), "tdm");
  hipcheck(hipStreamSynchronize(cx.stream), "props end");
  for (Tensor* t : {&Yn, &Ya, &tdm_t, &rho_t})
    if (t->p) tfree(cx, *t);
  cx.prec = saved;
}

// Bytes that an allocation-free sigma build of k vectors certainly takes from
// its scratch (a lower bound): the doubles accumulators of one vector and,
// when the particle-particle ladder runs, one (ac|bd) block of one a.
size_t noalloc_lower_bound(const Inst& I, int k, int prec) {
  (void)k;
  const double o = I.o, v = I.v, Po = (double)I.Po, Pv = (double)I.Pv;
  const double esz = prec == ADC_FP64 ? 16.0 : 8.0;
  double acc = 0.0;
  if (I.kind == ADC_EE) acc = esz * (o * o * Pv + Po * v * v + (I.x != 0.0 ? o * o * v * v : 0.0));
  else if (I.kind == ADC_IP) acc = 16.0 * o * o * v;
  else acc = 16.0 * o * v * v;
  const bool lad = I.x != 0.0 && I.kind != ADC_IP && Pv > 0 && (I.kind == ADC_EA || Po > 0);
  const double w = lad ? 16.0 * v * v * v : 0.0;
  return (size_t)std::max(acc, w);
}

// Rough cost of one sigma build (complex MACs), used to order instances
// longest first and to balance them over the lanes.
double sigma_cost(const adc_problem& p) {
  const double o = p.n_occ, v = p.n_vir, N = p.n_chol, k = p.n_roots;
  const double Po = o * (o - 1) / 2, Pv = v * (v - 1) / 2;
  if (p.kind == ADC_EE) return 2 * N * Pv * Pv + k * (Po * Pv * Pv + std::pow(o * v, 3) + o * o * v * v * v);
  if (p.kind == ADC_IP) return k * (o * std::pow(o * v, 2) + Po * Po * v) + N * o * o * v * v;
  return 2 * N * Pv * Pv + k * (o * Pv * Pv + v * std::pow(o * v, 2));
}

// Run f(lane) for every lane, lanes > 0 on worker threads (each with the
// handle's device current); returns the first error.
template <class F>
int for_lanes(adc_handle* h, F&& f) {
  const int L = h->n_lanes();
  std::vector<int> rc(L, ADC_OK);
  std::vector<std::thread> th;
  for (int l = 1; l < L; ++l)
    th.emplace_back([&, l]() {
      if (hipSetDevice(h->device) != hipSuccess) {
        rc[l] = ADC_ERR_HIP;
        return;
      }
      rc[l] = guarded([&]() { return f(l); });
    });
  rc[0] = guarded([&]() { return f(0); });
  for (auto& t : th) t.join();
  for (int l = 0; l < L; ++l)
    if (rc[l] < 0) return rc[l];
  for (int l = 0; l < L; ++l)
    if (rc[l] != ADC_OK) return rc[l];
  return ADC_OK;
}

// order a lane's stream after the handle's stream (before) or the handle's
// stream after the lane (after); no-op for lane 0
void lane_wait(adc_handle* h, Ctx& lane, bool before) {
  if (&lane == &h->cx) return;
  hipEvent_t e;
  hipcheck(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
  hipStream_t from = before ? h->cx.stream : lane.stream, to = before ? lane.stream : h->cx.stream;
  hipError_t r = hipEventRecord(e, from);
  if (r == hipSuccess) r = hipStreamWaitEvent(to, e, 0);
  (void)hipEventDestroy(e);
  hipcheck(r, "lane order");
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

int adc_init(const adc_problem* problems, int n_problems, const adc_options* opts, adc_handle** out) {
  g_last_error.clear();
  auto fail = [](int code, const char* msg) {
    g_last_error = msg;
    return code;
  };
  if (!out) return fail(ADC_ERR_INVALID_ARG, "no output handle");
  *out = nullptr;
  if (!problems || n_problems < 1) return fail(ADC_ERR_INVALID_ARG, "no problems");
  if (opts && (opts->precision < 0 || opts->precision > 2))
    return fail(ADC_ERR_INVALID_ARG, "precision must be ADC_FP64, ADC_FP32 or ADC_SPLIT_BF16");
  if (opts && opts->precision == ADC_SPLIT_BF16 && !kSplitBf16Built)
    return fail(ADC_ERR_UNSUPPORTED, "split-bf16 kernels not built");
  if (opts && opts->n_streams < 0) return fail(ADC_ERR_INVALID_ARG, "n_streams < 0");
  if (opts && (opts->graphs < 0 || opts->graphs > 2)) return fail(ADC_ERR_INVALID_ARG, "graphs must be 0, 1 or 2");
  if (opts && (opts->precond < 0 || opts->precond > 1)) return fail(ADC_ERR_INVALID_ARG, "precond must be 0 or 1");
  if (opts && !(opts->conv_tol >= 0.0 && std::isfinite(opts->conv_tol)))
    return fail(ADC_ERR_INVALID_ARG, "conv_tol must be finite and >= 0 (0 = default)");
  if (opts && (opts->max_iter < 0 || opts->max_subspace < 0))
    return fail(ADC_ERR_INVALID_ARG, "max_iter and max_subspace must be >= 0 (0 = default)");
  if (opts && (opts->refine_fp64 < -1 || opts->refine_fp64 > 1))
    return fail(ADC_ERR_INVALID_ARG, "refine_fp64 must be -1, 0 or 1");
  for (int i = 0; i < n_problems; ++i) {
    int rc = validate(&problems[i]);
    if (rc) return fail(rc, "problem description rejected (kind, sizes, eps, L or x)");
    if (!problems[i].L_on_device) {
      rc = validate_L_host((const double*)problems[i].L, problems[i].n_chol, problems[i].n_occ + problems[i].n_vir);
      if (rc) return fail(rc, "host L is non-finite or not Hermitian in (p,q)");
    }
  }
  adc_handle* h = nullptr;
  int rc = guarded([&]() {
    h = new adc_handle();
    if (opts) h->opt = *opts;
    hipcheck(hipGetDevice(&h->device), "device");
    // the allocation-free entry point's scratch on this device (its address
    // is taken once per device; nullptr leaves that entry point unavailable)
    h->scratch = scratch_address();
    if (h->opt.stream) {
      h->cx.stream = (hipStream_t)h->opt.stream;
    } else {
      hipcheck(hipStreamCreate(&h->cx.stream), "stream");
      h->own_stream = true;
    }
    int L = h->opt.n_streams > 0 ? h->opt.n_streams : 4;
    L = std::max(1, std::min(L, n_problems));
    for (int l = 1; l < L; ++l) {
      h->extra.emplace_back(new Ctx());
      hipcheck(hipStreamCreateWithFlags(&h->extra.back()->stream, hipStreamNonBlocking), "lane stream");
    }
    if (h->opt.deterministic) {
      h->opt.autotune = 0;
      h->opt.tune_cache = nullptr;
    }
    // the cache path is the caller's string: keep a copy for adc_free
    if (h->opt.tune_cache) {
      h->tune_path = h->opt.tune_cache;
      h->opt.tune_cache = nullptr;
      (void)tune_cache_load(h->tune_path.c_str());
    }
    for (int l = 0; l < L; ++l) {
      Ctx& c = h->lane(l);
      c.autotune = h->opt.autotune != 0;
      c.verbose = h->opt.verbose;
      if (h->opt.mem_budget)
        c.max_temp = std::min<int64_t>((int64_t)1 << 29, (int64_t)(h->opt.mem_budget / sizeof(double2)));
    }
    // longest processing time first: each instance to the least loaded lane
    std::vector<int> order(n_problems);
    for (int i = 0; i < n_problems; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return sigma_cost(problems[a]) > sigma_cost(problems[b]); });
    std::vector<double> load(L, 0.0);
    h->lane_inst.assign(L, {});
    h->inst.resize(n_problems);
    for (int i : order) {
      const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[l] += sigma_cost(problems[i]);
      h->lane_inst[l].push_back(i);
      h->inst[i].cx = &h->lane(l);
    }
    auto t0 = std::chrono::steady_clock::now();
    const int r = for_lanes(h, [&](int l) {
      for (int i : h->lane_inst[l]) inst_init(h, &problems[i], h->inst[i]);
      Ctx& c = h->lane(l);
      hipcheck(hipStreamSynchronize(c.stream), "init sync");
      c.pool.trim();
      return (int)ADC_OK;
    });
    if (r != ADC_OK) return r;
    h->init_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return (int)ADC_OK;
  });
  if (rc != ADC_OK) {
    adc_free(h);
    return rc;
  }
  *out = h;
  return ADC_OK;
}

int adc_dims(const adc_handle* h, int inst, long long* n1, long long* n2) {
  g_last_error.clear();
  if (!h || inst < 0 || inst >= (int)h->inst.size() || !n1 || !n2)
    return reject(ADC_ERR_INVALID_ARG, "adc_dims: NULL handle or output, or instance out of range");
  *n1 = h->inst[inst].n1;
  *n2 = h->inst[inst].n2;
  return ADC_OK;
}

int adc_sigma(adc_handle* h, int inst, const void* Y, void* S, int k, int precision) {
  g_last_error.clear();
  if (!h || inst < 0 || inst >= (int)h->inst.size() || !Y || !S || k < 0 || Y == S)
    return reject(ADC_ERR_INVALID_ARG, "adc_sigma: NULL handle, Y or S, instance out of range, k < 0 or Y == S");
  if (precision > 2) return reject(ADC_ERR_INVALID_ARG, "adc_sigma: unknown precision");
  const int prec = precision < 0 ? h->opt.precision : precision;
  if (prec == ADC_SPLIT_BF16 && !kSplitBf16Built) return reject(ADC_ERR_UNSUPPORTED, "split-bf16 kernels not built");
  return guarded([&]() {
    Inst& I = h->inst[inst];
    lane_wait(h, *I.cx, true);
    sigma_dispatch(h, I, (const double2*)Y, (double2*)S, k, prec);
    lane_wait(h, *I.cx, false);
    hipcheck(hipGetLastError(), "sigma launch");
    return ADC_OK;
  });
}

int adc_sigma_term(adc_handle* h, int inst, int term, const void* Y, void* S, int k, int precision) {
  g_last_error.clear();
  if (term == ADC_TERM_ALL) return adc_sigma(h, inst, Y, S, k, precision);
  if (!h || inst < 0 || inst >= (int)h->inst.size() || !Y || !S || k < 0 || Y == S)
    return reject(ADC_ERR_INVALID_ARG,
                  "adc_sigma_term: NULL handle, Y or S, instance out of range, k < 0 or Y == S");
  if (precision > 2 || term != ADC_TERM_LADDER)
    return reject(ADC_ERR_INVALID_ARG, "adc_sigma_term: unknown precision or term");
  Inst& I = h->inst[inst];
  if (I.kind == ADC_IP) return reject(ADC_ERR_UNSUPPORTED, "adc_sigma_term: IP has no particle-particle ladder");
  const int prec = precision < 0 ? h->opt.precision : precision;
  return guarded([&]() {
    lane_wait(h, *I.cx, true);
    launch_fill((double2*)S, (int64_t)k * I.dim, C0(), I.cx->stream);
    const int64_t nrow = I.kind == ADC_EE ? I.Po : I.o;
    ladder(h, I, (const double2*)Y, I.dim, I.n1, (double2*)S, I.dim, I.n1, nrow, k, CR(I.x), prec);
    lane_wait(h, *I.cx, false);
    hipcheck(hipGetLastError(), "term launch");
    return ADC_OK;
  });
}

int adc_sigma_noalloc(adc_handle* h, int inst, const void* Y, void* S, int k, int precision) {
  g_last_error.clear();
  if (!h || inst < 0 || inst >= (int)h->inst.size() || !Y || !S || k < 0 || Y == S)
    return reject(ADC_ERR_INVALID_ARG,
                  "adc_sigma_noalloc: NULL handle, Y or S, instance out of range, k < 0 or Y == S");
  if (precision > 2) return reject(ADC_ERR_INVALID_ARG, "adc_sigma_noalloc: unknown precision");
  const int prec = precision < 0 ? h->opt.precision : precision;
  if (prec == ADC_SPLIT_BF16 && !kSplitBf16Built) return reject(ADC_ERR_UNSUPPORTED, "split-bf16 kernels not built");
  if (!h->scratch) return reject(ADC_ERR_HIP, "adc_sigma_noalloc: the fixed device scratch is not available");
  Inst& I = h->inst[inst];
  if (k == 0) return ADC_OK;
  if (noalloc_lower_bound(I, k, prec) > kScratchBytes)
    return reject(ADC_ERR_SCRATCH, "adc_sigma_noalloc: the build needs more than the fixed device scratch");
  if (I.noalloc_too_big[prec] > 0 && k >= I.noalloc_too_big[prec])
    return reject(ADC_ERR_SCRATCH, "adc_sigma_noalloc: a build with this many vectors already exceeded the scratch");
  return guarded([&]() {
    Ctx& cx = *I.cx;
    // the build's temporaries come from the scratch; its passes, ladder
    // batches and temporary copies are planned for the scratch size, and no
    // GEMM is timed (the tuner would need extra buffers and host waits)
    struct Arena {
      Ctx& cx;
      bool tune;
      int64_t max_temp;
      Arena(Ctx& c, void* base) : cx(c), tune(c.autotune), max_temp(c.max_temp) {
        cx.pool.begin_arena(base, kScratchBytes);
        cx.autotune = false;
        cx.ws_override = kScratchBytes;
        cx.max_temp = std::min<int64_t>(cx.max_temp, (int64_t)(kScratchBytes / sizeof(double2) / 8));
      }
      ~Arena() {
        cx.pool.end_arena();
        cx.autotune = tune;
        cx.ws_override = 0;
        cx.max_temp = max_temp;
      }
    } arena(cx, h->scratch);
    lane_wait(h, cx, true);
    try {
      sigma_dispatch(h, I, (const double2*)Y, (double2*)S, k, prec);
    } catch (const ArenaFull&) {
      // kernels already enqueued use the scratch: let them finish (unless a
      // capture is recording them) before another call may reuse it
      I.noalloc_too_big[prec] = I.noalloc_too_big[prec] > 0 ? std::min(I.noalloc_too_big[prec], k) : k;
      hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing(cx.stream, &st) == hipSuccess && st == hipStreamCaptureStatusNone)
        (void)hipStreamSynchronize(cx.stream);
      (void)hipGetLastError();
      return (int)ADC_ERR_SCRATCH;
    }
    lane_wait(h, cx, false);
    hipcheck(hipGetLastError(), "sigma launch");
    return (int)ADC_OK;
  });
}

int adc_properties(adc_handle* h, int inst, const void* Y, int k, void* rho, void* tdm, const void* d, double* dk,
                   double* tk) {
  g_last_error.clear();
  if (!h || inst < 0 || inst >= (int)h->inst.size() || !Y || k < 1)
    return reject(ADC_ERR_INVALID_ARG, "adc_properties: NULL handle or Y, instance out of range or k < 1");
  if ((dk || tk) && !d) return reject(ADC_ERR_INVALID_ARG, "adc_properties: dk or tk needs the operator d");
  Inst& I = h->inst[inst];
  if (I.kind != ADC_EE) return reject(ADC_ERR_UNSUPPORTED, "adc_properties: EE instances only");
  return guarded([&]() {
    lane_wait(h, *I.cx, true);
    props_build(h, I, (const double2*)Y, k, (double2*)rho, (double2*)tdm, (const double2*)d, dk, tk);
    lane_wait(h, *I.cx, false);
    hipcheck(hipGetLastError(), "properties launch");
    return (int)ADC_OK;
  });
}

int adc_fns(adc_handle* h, int inst, const void* X, double eta_crit, int* n_vir, double* eps_out, void* L_out,
            double* eta_out, void* B_out, void* X_out) {
  g_last_error.clear();
  if (!h || inst < 0 || inst >= (int)h->inst.size() || !n_vir || !eps_out || !L_out || !std::isfinite(eta_crit))
    return reject(ADC_ERR_INVALID_ARG, "adc_fns: NULL handle or output, instance out of range or non-finite eta_crit");
  Inst& I = h->inst[inst];
  if (X && I.kind == ADC_IP) return reject(ADC_ERR_UNSUPPORTED, "adc_fns: no state-specific density for IP");
  if (X_out && !X) return reject(ADC_ERR_INVALID_ARG, "adc_fns: X_out needs X");
  return guarded([&]() {
    lane_wait(h, *I.cx, true);
    fns_build(h, I, (const double2*)X, eta_crit, n_vir, eps_out, (double2*)L_out, eta_out, (double2*)B_out,
              (double2*)X_out);
    lane_wait(h, *I.cx, false);
    hipcheck(hipGetLastError(), "fns launch");
    return (int)ADC_OK;
  });
}

int adc_davidson(adc_handle* h, const void* const* guess, double* omega, void* const* vecs, double* resnorm,
                 int* iters, int* converged) {
  g_last_error.clear();
  if (!h || !omega || !resnorm || !iters || !converged)
    return reject(ADC_ERR_INVALID_ARG, "adc_davidson: NULL handle or output array");
  // offsets of each instance's roots in the concatenated outputs
  std::vector<int64_t> off(h->inst.size() + 1, 0);
  for (size_t i = 0; i < h->inst.size(); ++i) off[i + 1] = off[i] + h->inst[i].k;
  return guarded([&]() {
    hipcheck(hipStreamSynchronize(h->cx.stream), "dav start");
    std::vector<int> st(h->inst.size(), ADC_OK);
    const int r = for_lanes(h, [&](int l) {
      for (int i : h->lane_inst[l]) {
        Inst& I = h->inst[i];
        const double2* g = guess ? (const double2*)guess[i] : nullptr;
        double2* vv = vecs ? (double2*)vecs[i] : nullptr;
        st[i] = davidson_one(h, I, g, omega + off[i], vv, resnorm + off[i], iters + i, converged + off[i]);
      }
      return (int)ADC_OK;
    });
    if (r != ADC_OK) return r;
    for (int s_ : st)
      if (s_ != ADC_OK) return s_;
    return (int)ADC_OK;
  });
}

int adc_sigma_backward(adc_handle* h, int inst, const void* Sbar, const void* Y, int k, void* dL, double* dx) {
  g_last_error.clear();
  if (!h || inst < 0 || inst >= (int)h->inst.size() || !Sbar || !Y || k < 0)
    return reject(ADC_ERR_INVALID_ARG, "adc_sigma_backward: NULL handle, Sbar or Y, instance out of range or k < 0");
  return guarded([&]() {
    Inst& I = h->inst[inst];
    hipcheck(hipStreamSynchronize(h->cx.stream), "bw start");
    if (k == 0) {
      if (dL) {
        const int64_t n = I.o + I.v;
        launch_fill((double2*)dL, (int64_t)I.N * n * n, C0(), I.cx->stream);
        hipcheck(hipStreamSynchronize(I.cx->stream), "bw zero");
      }
      if (dx) *dx = 0.0;
      return ADC_OK;
    }
    sigma_backward(h, I, (const double2*)Sbar, (const double2*)Y, k, (double2*)dL, dx);
    hipcheck(hipGetLastError(), "backward launch");
    return ADC_OK;
  });
}

double adc_init_ms(const adc_handle* h) { return h ? h->init_ms : 0.0; }

void adc_free(adc_handle* h) {
  if (!h) return;
  if (!h->tune_path.empty() && h->opt.autotune) (void)tune_cache_save(h->tune_path.c_str());
  if (h->cx.stream) (void)hipStreamSynchronize(h->cx.stream);
  for (auto& I : h->inst)
    if (I.cx) {
      (void)hipStreamSynchronize(I.cx->stream);
      release_graphs(I);
    }
  for (auto& c : h->extra) {
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    c->pool.release_all();
    if (c->stream) (void)hipStreamDestroy(c->stream);
  }
  h->cx.pool.release_all();
  if (!h->raw.empty()) {
    std::unique_lock<std::shared_mutex> gate(capture_gate());
    for (void* p : h->raw) (void)hipFree(p);
  }
  if (h->own_stream && h->cx.stream) (void)hipStreamDestroy(h->cx.stream);
  delete h;
}

const char* adc_last_error(void) { return g_last_error.c_str(); }

const char* adc_strerror(int code) {
  switch (code) {
    case ADC_OK: return "ok";
    case ADC_NOT_CONVERGED: return "Davidson did not converge for every root (outputs filled)";
    case ADC_ERR_INVALID_ARG: return "invalid argument";
    case ADC_ERR_NONFINITE_INPUT: return "non-finite value in eps, L or x, or in a Davidson subspace matrix";
    case ADC_ERR_NOT_HERMITIAN: return "a Cholesky vector L^Q is not Hermitian in (p,q)";
    case ADC_ERR_OUT_OF_MEMORY: return "out of device memory";
    case ADC_ERR_HIP: return "HIP runtime error";
    case ADC_ERR_UNSUPPORTED: return "unsupported request";
    case ADC_ERR_SCRATCH: return "the build does not fit the fixed scratch of the allocation-free entry point";
    default: return "unknown status";
  }
}

}  // extern "C"
