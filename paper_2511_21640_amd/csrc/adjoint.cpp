// Reverse-mode differentiation of the recorded device operations.
//
// The sigma build S = M(L, x) Y is a chain of linear maps in each tensor it
// touches: complex contractions, permutations, real diagonal scalings
// (the MP denominators), antisymmetrisers, Hermitian parts, packing and the
// particle-particle ladder.  For a real objective f the gradient of a complex
// tensor Z is G_Z = df/dRe Z + i df/dIm Z; for a linear op C = alpha op(A) B
// it propagates as
//     G_A += conj(alpha) G_C conj(B)^T         (A used as is)
//     G_A += alpha conj(G_C) B^T   (conjugated)  (A used conjugated)
// contracted over the labels of C and B that A lacks, which is again one
// ctr() call.  Ops that overwrite C (beta = 0) clear G_C once they have
// passed it on, so a buffer reused for several tensors receives each
// tensor's gradient in turn.
#include <stdexcept>
#include <string>

#include "internal.h"

namespace adc {

namespace {

int alloc_of(const Tape& T, const void* p) { return p ? T.find(p) : -1; }

bool has_grad(const Tape& T, const void* p) {
  const int i = alloc_of(T, p);
  return i >= 0 && T.allocs[i].grad != nullptr;
}

double2* grad_ptr(Ctx& cx, const void* p) {
  Tape& T = *cx.tape;
  const int i = alloc_of(T, p);
  if (i < 0) throw std::logic_error("gradient of an unrecorded buffer");
  Tape::Alloc& a = T.allocs[i];
  if (!a.grad) {
    const int64_t n = (int64_t)(a.bytes / sizeof(double2));
    a.grad = cx.pool.get(n);
    launch_fill(a.grad, n, C0(), cx.stream);
  }
  return a.grad + ((uintptr_t)p - a.base) / sizeof(double2);
}

std::string labels(size_t rank) { return std::string("abcdefgh").substr(0, rank); }

// G <- s * G over the view (s = 0 clears it)
void scale_view(Ctx& cx, Tensor G, cplx s) {
  if (s.re == 1.0 && s.im == 0.0) return;
  const std::string l = labels(G.d.size());
  perm(cx, s, G, l.c_str(), false, C0(), G, l.c_str());
}

// dst[0..n) += alpha * src[0..n)
void add_flat(Ctx& cx, double2* dst, const double2* src, int64_t n, cplx alpha) {
  if (n <= 0) return;
  const int64_t od[1] = {n}, st[1] = {1};
  launch_permute(1, od, st, st, src, dst, alpha, C1(), 0, cx.stream);
}

cplx conjc(cplx a) { return {a.re, -a.im}; }

void check_labels(const std::string& out, const std::string& a, const std::string& b) {
  for (char c : out)
    if (a.find(c) == std::string::npos && b.find(c) == std::string::npos)
      throw std::logic_error("adjoint needs a broadcast over label " + std::string(1, c));
}

void check_distinct(const Tape& T, const Tensor& x, const Tensor& c) {
  if (x.p && alloc_of(T, x.p) >= 0 && alloc_of(T, x.p) == alloc_of(T, c.p))
    throw std::logic_error("recorded op reads and writes one buffer");
}

// element count of an unpacked doubles tensor [k][...] of the given kind
int64_t unpacked_per(int kind, int64_t o, int64_t v) {
  return kind == 0 ? o * o * v * v : (kind == 1 ? o * o * v : o * v * v);
}
int64_t packed_n2(int kind, int64_t o, int64_t v) {
  const int64_t Po = o * (o - 1) / 2, Pv = v * (v - 1) / 2;
  return kind == 0 ? Po * Pv : (kind == 1 ? Po * v : o * Pv);
}

void bw_ctr(Ctx& cx, const TapeOp& op) {
  Tape& T = *cx.tape;
  if (!has_grad(T, op.C.p)) return;
  check_distinct(T, op.A, op.C);
  check_distinct(T, op.B, op.C);
  Tensor GC = grad_view(cx, op.C);
  if (T.rg(op.A.p)) {
    check_labels(op.la, op.lc, op.lb);
    Tensor GA = grad_view(cx, op.A);
    if (!op.cA)
      ctr(cx, conjc(op.alpha), GC, op.lc.c_str(), false, op.B, op.lb.c_str(), !op.cB, C1(), GA, op.la.c_str());
    else
      ctr(cx, op.alpha, GC, op.lc.c_str(), true, op.B, op.lb.c_str(), op.cB, C1(), GA, op.la.c_str());
  }
  if (T.rg(op.B.p)) {
    check_labels(op.lb, op.lc, op.la);
    Tensor GB = grad_view(cx, op.B);
    if (!op.cB)
      ctr(cx, conjc(op.alpha), GC, op.lc.c_str(), false, op.A, op.la.c_str(), !op.cA, C1(), GB, op.lb.c_str());
    else
      ctr(cx, op.alpha, GC, op.lc.c_str(), true, op.A, op.la.c_str(), op.cA, C1(), GB, op.lb.c_str());
  }
  scale_view(cx, GC, conjc(op.beta));
}

void bw_perm(Ctx& cx, const TapeOp& op) {
  Tape& T = *cx.tape;
  if (!has_grad(T, op.C.p)) return;
  check_distinct(T, op.A, op.C);
  Tensor GC = grad_view(cx, op.C);
  if (T.rg(op.A.p)) {
    Tensor GA = grad_view(cx, op.A);
    if (!op.cA) perm(cx, conjc(op.alpha), GC, op.lc.c_str(), false, C1(), GA, op.la.c_str());
    else perm(cx, op.alpha, GC, op.lc.c_str(), true, C1(), GA, op.la.c_str());
  }
  scale_view(cx, GC, conjc(op.beta));
}

void bw_op_in(Ctx& cx, const TapeOp& op);

// every reverse rule runs in the arithmetic of its forward op
void bw_op(Ctx& cx, const TapeOp& op) {
  const int saved = cx.prec;
  cx.prec = op.prec;
  try {
    bw_op_in(cx, op);
  } catch (...) {
    cx.prec = saved;
    throw;
  }
  cx.prec = saved;
}

void bw_op_in(Ctx& cx, const TapeOp& op) {
  Tape& T = *cx.tape;
  switch (op.kind) {
    case TapeOp::CTR: bw_ctr(cx, op); break;
    case TapeOp::PERM: bw_perm(cx, op); break;
    case TapeOp::DIV_D2:
    case TapeOp::DIV_D1: {
      // t <- t / D elementwise with real D: G_t <- G_t / D
      if (!has_grad(T, op.C.p)) break;
      double2* g = grad_ptr(cx, op.C.p);
      if (op.kind == TapeOp::DIV_D2) launch_div_d2(g, op.eps, (int)op.n[0], (int)op.n[1], cx.stream);
      else launch_div_d1(g, op.eps, (int)op.n[0], (int)op.n[1], cx.stream);
      break;
    }
    case TapeOp::ANTISYM: {
      // out += alpha (X - swap X): the antisymmetriser is self-adjoint
      if (!has_grad(T, op.C.p) || !T.rg(op.A.p)) break;
      check_distinct(T, op.A, op.C);
      launch_antisym_add(grad_ptr(cx, op.C.p), grad_ptr(cx, op.A.p), op.n[0], op.n[1], op.n[2], op.n[3], op.n[4],
                         (int)op.n[5], conjc(op.alpha), cx.stream);
      break;
    }
    case TapeOp::HERM_ADD: {
      // out = X + X^H (n x n): G_X += G_out + G_out^H, then G_out = 0
      if (!has_grad(T, op.C.p)) break;
      check_distinct(T, op.A, op.C);
      const int64_t n = op.n[0];
      double2* gout = grad_ptr(cx, op.C.p);
      if (T.rg(op.A.p)) {
        double2* tmp = cx.pool.get(n * n);
        launch_herm_add(gout, tmp, n, cx.stream);
        add_flat(cx, grad_ptr(cx, op.A.p), tmp, n * n, C1());
        cx.pool.put(tmp);
      }
      launch_fill(gout, n * n, C0(), cx.stream);
      break;
    }
    case TapeOp::M11_DELTA: {
      // M[(i,a),(i,A)] += f[a][A] (or the occupied twin): G_f += partial traces of G_M
      if (!has_grad(T, op.C.p) || !T.rg(op.A.p)) break;
      launch_m11_delta_adjoint(grad_ptr(cx, op.C.p), grad_ptr(cx, op.A.p), (int)op.n[0], (int)op.n[1],
                               (int)op.n[2], cx.stream);
      break;
    }
    case TapeOp::PACK: {
      // S[z][off + q] = alpha U[z][canonical(q)] + D_q Y (+ S): G_U at the canonical
      // positions += conj(alpha) G_S; the overwrite clears G_S
      if (!has_grad(T, op.C.p)) break;
      const int kind = (int)op.n[0];
      const int64_t ld = op.n[1], off = op.n[2], k = op.n[3], o = op.n[4], v = op.n[5];
      double2* gS = grad_ptr(cx, op.C.p);
      if (op.A.p && T.rg(op.A.p)) {
        const int64_t per = unpacked_per(kind, o, v);
        double2* tmp = cx.pool.get(k * per);
        launch_unpack_doubles(kind, gS, ld, off, (int)k, (int)o, (int)v, nullptr, tmp, cx.stream);
        add_flat(cx, grad_ptr(cx, op.A.p), tmp, k * per, conjc(op.alpha));
        cx.pool.put(tmp);
      }
      if (!op.n[6]) {
        Tensor g;
        g.p = gS + off;
        g.d = {k, packed_n2(kind, o, v)};
        g.st = {ld, 1};
        scale_view(cx, g, C0());
      }
      break;
    }
    case TapeOp::UNPACK: {
      // Ya = antisymmetric expansion of packed Y: G_Y += signed sum of G_Ya over
      // the images of each packed element; the overwrite clears G_Ya
      if (!has_grad(T, op.C.p)) break;
      const int kind = (int)op.n[0];
      const int64_t ld = op.n[1], off = op.n[2], k = op.n[3], o = op.n[4], v = op.n[5];
      const int64_t per = unpacked_per(kind, o, v);
      double2* gYa = grad_ptr(cx, op.C.p);
      if (T.rg(op.A.p)) {
        double2* tmp = cx.pool.get(k * per);
        launch_fill(tmp, k * per, C0(), cx.stream);
        if (kind == 0) launch_antisym_add(gYa, tmp, k, o, o, v, v, 2, C1(), cx.stream);
        else if (kind == 1) launch_antisym_add(gYa, tmp, k, o, o, v, 1, 0, C1(), cx.stream);
        else launch_antisym_add(gYa, tmp, k, o, 1, v, v, 1, C1(), cx.stream);
        launch_pack_doubles(kind, tmp, grad_ptr(cx, op.A.p), nullptr, ld, off, (int)k, (int)o, (int)v, op.eps, C1(),
                            1, op.po, op.pv, cx.stream);
        cx.pool.put(tmp);
      }
      launch_fill(gYa, k * per, C0(), cx.stream);
      break;
    }
    case TapeOp::PACK_EE: {
      // S = P(ij) A0 + P(ab) A1 + P(ij)P(ab) A2 at the packed positions (+ D Y):
      // G_Ak += the same antisymmetriser applied to G_S embedded at the packed
      // positions; the overwrite clears G_S
      if (!has_grad(T, op.C.p)) break;
      const int64_t ld = op.n[0], off = op.n[1], k = op.n[2], o = op.n[3], v = op.n[4];
      const int64_t per = o * o * v * v;
      double2* gS = grad_ptr(cx, op.C.p);
      const Tensor* acc[3] = {&op.A, &op.B, &op.extra};
      bool any = false;
      for (const Tensor* t : acc) any = any || (t->p && T.rg(t->p));
      if (any) {
        double2* tmp = cx.pool.get(k * per);
        launch_unpack_doubles(0, gS, ld, off, (int)k, (int)o, (int)v, nullptr, tmp, cx.stream);
        for (int m = 0; m < 3; ++m)
          if (acc[m]->p && T.rg(acc[m]->p))
            launch_antisym_add(tmp, grad_ptr(cx, acc[m]->p), k, o, o, v, v, m, C1(), cx.stream);
        cx.pool.put(tmp);
      }
      Tensor g;
      g.p = gS + off;
      g.d = {k, packed_n2(0, o, v)};
      g.st = {ld, 1};
      scale_view(cx, g, C0());
      break;
    }
    case TapeOp::LADDER: {
      if (!has_grad(T, op.C.p)) break;
      double2* gY = T.rg(op.A.p) ? grad_ptr(cx, op.A.p) : nullptr;
      op.ladder_bw(cx, op, grad_ptr(cx, op.C.p), gY);
      break;
    }
  }
}

}  // namespace

Tensor grad_view(Ctx& cx, const Tensor& t) {
  Tensor g = t;
  g.p = grad_ptr(cx, t.p);
  return g;
}

void tape_backward(Ctx& cx) {
  Tape* T = cx.tape;
  if (!T) throw std::logic_error("no tape");
  T->recording = false;
  cx.pool.tape = nullptr;  // temporaries of the sweep are ordinary pool blocks
  for (auto it = T->ops.rbegin(); it != T->ops.rend(); ++it) bw_op(cx, *it);
}

void tape_release(Ctx& cx) {
  Tape* T = cx.tape;
  if (!T) return;
  cx.pool.tape = nullptr;
  for (auto& a : T->allocs)
    if (a.grad) cx.pool.put(a.grad);
  for (double2* p : T->deferred) cx.pool.put(p);
  T->ops.clear();
  T->allocs.clear();
  T->deferred.clear();
  T->recording = false;
  cx.tape = nullptr;
}

// ---------------------------------------------------------------- recorded launches
void rec_div_d2(Ctx& cx, Tensor& t, const double* eps, int o, int v) {
  TapeOp op{};
  op.kind = TapeOp::DIV_D2;
  op.A = t; op.C = t; op.eps = eps; op.n[0] = o; op.n[1] = v;
  tape_record(cx, op);
  launch_div_d2(t.p, eps, o, v, cx.stream);
}

void rec_div_d1(Ctx& cx, Tensor& t, const double* eps, int o, int v) {
  TapeOp op{};
  op.kind = TapeOp::DIV_D1;
  op.A = t; op.C = t; op.eps = eps; op.n[0] = o; op.n[1] = v;
  tape_record(cx, op);
  launch_div_d1(t.p, eps, o, v, cx.stream);
}

void rec_antisym_add(Ctx& cx, const Tensor& X, Tensor& out, int64_t k, int64_t d1, int64_t d2, int64_t d3, int64_t d4,
                     int which, cplx alpha) {
  TapeOp op{};
  op.kind = TapeOp::ANTISYM;
  op.A = X; op.C = out; op.alpha = alpha;
  op.n[0] = k; op.n[1] = d1; op.n[2] = d2; op.n[3] = d3; op.n[4] = d4; op.n[5] = which;
  tape_record(cx, op);
  launch_antisym_add(X.p, out.p, k, d1, d2, d3, d4, which, alpha, cx.stream);
}

void rec_herm_add(Ctx& cx, const Tensor& X, Tensor& out, int64_t n) {
  TapeOp op{};
  op.kind = TapeOp::HERM_ADD;
  op.A = X; op.C = out; op.n[0] = n;
  tape_record(cx, op);
  launch_herm_add(X.p, out.p, n, cx.stream);
}

void rec_m11_add_delta(Ctx& cx, Tensor& M, const Tensor& f, int o, int v, int which) {
  TapeOp op{};
  op.kind = TapeOp::M11_DELTA;
  op.A = f; op.C = M; op.n[0] = o; op.n[1] = v; op.n[2] = which;
  tape_record(cx, op);
  launch_m11_add_delta(M.p, f.p, o, v, which, cx.stream);
}

void rec_pack_doubles(Ctx& cx, int kind, const Tensor& U, double2* S, const double2* Y, int64_t ld, int64_t off,
                      int k, int o, int v, const double* eps, cplx alpha, int accumulate, const int2* po,
                      const int2* pv) {
  TapeOp op{};
  op.kind = TapeOp::PACK;
  op.A = U; op.C.p = S; op.alpha = alpha; op.eps = eps; op.po = po; op.pv = pv;
  op.n[0] = kind; op.n[1] = ld; op.n[2] = off; op.n[3] = k; op.n[4] = o; op.n[5] = v; op.n[6] = accumulate;
  tape_record(cx, op);
  launch_pack_doubles(kind, U.p, S, Y, ld, off, k, o, v, eps, alpha, accumulate, po, pv, cx.stream);
}

void rec_unpack_doubles(Ctx& cx, int kind, const double2* Y, int64_t ld, int64_t off, int k, int o, int v, Tensor& Ya,
                        const double* eps, const int2* po, const int2* pv) {
  TapeOp op{};
  op.kind = TapeOp::UNPACK;
  op.A.p = const_cast<double2*>(Y); op.C = Ya; op.eps = eps; op.po = po; op.pv = pv;
  op.n[0] = kind; op.n[1] = ld; op.n[2] = off; op.n[3] = k; op.n[4] = o; op.n[5] = v;
  tape_record(cx, op);
  launch_unpack_doubles(kind, Y, ld, off, k, o, v, Ya.p, nullptr, cx.stream);
}

void rec_pack_ee(Ctx& cx, const Tensor& A0, const Tensor& A1, const Tensor& A2, double2* S, const double2* Y,
                 int64_t ld, int64_t off, int k, int o, int v, const double* eps, const int2* po, const int2* pv) {
  if (cx.tape && cx.tape->recording) {
    TapeOp op{};
    op.kind = TapeOp::PACK_EE;
    op.A = A0; op.B = A1; op.extra = A2; op.C.p = S;
    op.n[0] = ld; op.n[1] = off; op.n[2] = k; op.n[3] = o; op.n[4] = v;
    // an op with three inputs: mark the output from all of them
    Tape* t = cx.tape;
    if (A2.p && t->rg(A2.p)) {
      const int ic = t->find(S);
      if (ic >= 0) t->allocs[ic].rg = true;
      const int ia = t->find(A2.p);
      if (ia >= 0) t->allocs[ia].ref = true;
    }
    tape_record(cx, op);
  }
  if (A0.f32 != A1.f32 || (A2.p && A2.f32 != A0.f32)) throw std::logic_error("pack_ee: mixed accumulator types");
  launch_pack_ee(A0.p, A1.p, A2.p, S, Y, ld, off, k, o, v, eps, po, pv, cx.stream, A0.f32 ? 1 : 0);
}

}  // namespace adc

