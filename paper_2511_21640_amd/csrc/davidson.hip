// Device side of the Davidson iteration (Section 2.1, eq. 10): the small
// Hermitian eigenproblems of the subspace and of the new directions, and the
// per-root bookkeeping (convergence test, Olsen's correction, the choice of
// the new directions), so that an iteration runs without the host and can be
// captured as one hipGraph.
//
// Eigensolver: cyclic complex Jacobi in the round-robin ordering, one
// workgroup.  Each round's n/2 index pairs are disjoint, so their rotations
// are computed together and applied as A <- J^H A J (all row rotations, then
// all column rotations) and U <- U J.  For a pair (p, q) with
// a_pq = |a_pq| e^{i phi}, theta = atan2(2 |a_pq|, a_qq - a_pp) / 2,
// c = cos theta and s = sin theta:
//   rows     p' = c p - s e^{i phi} q,      q' = s e^{-i phi} p + c q
//   columns  p' = c p - s e^{-i phi} q,     q' = s e^{i phi} p + c q
// which zeroes a_pq.  Sweeps run until the off-diagonal weight is at most
// 1e-30 of the total (at most 60 sweeps); the eigenvalues are then put in
// ascending order (equal values keep their index order) with their columns.
// A and the rotation accumulator live in LDS when both fit (mode 2), else A
// alone (mode 1), else both in the global workspace the caller passes
// (mode 0).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace adc {

namespace {

constexpr int kJacobiThreads = 1024;
constexpr int kJacobiMaxN = 256;
constexpr int kCombineMaxM = 256;  // rows a of a combination: 64 KB of staged coefficients at most

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// player in slot j of round r of the round-robin over m (even) players:
// slot 0 keeps player 0, the others rotate
__device__ __forceinline__ int rr_player(int slot, int r, int m) {
  if (slot == 0) return 0;
  return 1 + (slot - 1 + r) % (m - 1);
}

__device__ __forceinline__ double wave_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
  return x;
}

__global__ __launch_bounds__(kJacobiThreads) void heev_jacobi_kernel(const double2* G, int ldg, int n,
                                                                      double2* Ag, double2* Vg, int mode,
                                                                      double2* U, int ldu, double* w) {
  extern __shared__ double2 dyn[];
  __shared__ double cs[kJacobiMaxN / 2], ss[kJacobiMaxN / 2];
  __shared__ double2 ph[kJacobiMaxN / 2];
  __shared__ int pp[kJacobiMaxN / 2], qq[kJacobiMaxN / 2];
  __shared__ double red[2][kJacobiThreads / 64];
  __shared__ double dg[kJacobiMaxN];
  __shared__ int order[kJacobiMaxN];
  __shared__ int stop, bad;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nn = n * n;
  double2* A = mode >= 1 ? dyn : Ag;
  double2* V = mode == 2 ? dyn + nn : Vg;
  if (tid == 0) bad = 0;
  __syncthreads();
  // A = (G + G^H) / 2, V = I
  for (int e = tid; e < nn; e += nt) {
    const int r = e / n, c = e - r * n;
    const double2 a = G[(int64_t)r * ldg + c], b = G[(int64_t)c * ldg + r];
    if (!isfinite(a.x) || !isfinite(a.y)) bad = 1;
    A[e] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    V[e] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  if (bad) {
    // a non-finite subspace matrix: NaN eigenvalues tell the caller
    for (int c = tid; c < n; c += nt) w[c] = __builtin_nan("");
    for (int e = tid; e < nn; e += nt) U[(int64_t)(e / n) * ldu + e % n] = make_double2(0.0, 0.0);
    return;
  }
  const int m = (n + 1) / 2 * 2;  // players; player n (n odd) sits out
  const int half = m / 2;
  for (int sweep = 0; sweep < 60 && n > 1; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < nn; e += nt) {
      const int r = e / n, c = e - r * n;
      const double x = A[e].x * A[e].x + A[e].y * A[e].y;
      tot += x;
      if (r != c) off += x;
    }
    off = wave_sum(off);
    tot = wave_sum(tot);
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = off;
      red[1][tid >> 6] = tot;
    }
    __syncthreads();
    if (tid == 0) {
      double so = 0.0, st = 0.0;
      for (int i = 0; i < nt / 64; ++i) {
        so += red[0][i];
        st += red[1][i];
      }
      stop = !(so > 1e-30 * fmax(st, 1e-300));
    }
    __syncthreads();
    if (stop) break;
    for (int r = 0; r < m - 1; ++r) {
      for (int j = tid; j < half; j += nt) {
        int p = rr_player(j, r, m), q = rr_player(m - 1 - j, r, m);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        pp[j] = p;
        qq[j] = q;
        double c = 1.0, s = 0.0;
        double2 e = make_double2(1.0, 0.0);
        if (q < n) {
          const double2 apq = A[p * n + q];
          const double mag = sqrt(apq.x * apq.x + apq.y * apq.y);
          if (mag > 1e-300) {
            e = make_double2(apq.x / mag, apq.y / mag);
            const double th = 0.5 * atan2(2.0 * mag, A[q * n + q].x - A[p * n + p].x);
            c = cos(th);
            s = sin(th);
          }
        }
        cs[j] = c;
        ss[j] = s;
        ph[j] = e;
      }
      __syncthreads();
      // rows p and q of A
      for (int t = tid; t < half * n; t += nt) {
        const int j = t / n, x = t - j * n;
        const int p = pp[j], q = qq[j];
        if (q >= n || ss[j] == 0.0) continue;
        const double c = cs[j], s = ss[j];
        const double2 e = ph[j], ec = make_double2(e.x, -e.y);
        const double2 ap = A[p * n + x], aq = A[q * n + x];
        const double2 t1 = cmul(e, aq), t2 = cmul(ec, ap);
        A[p * n + x] = make_double2(c * ap.x - s * t1.x, c * ap.y - s * t1.y);
        A[q * n + x] = make_double2(s * t2.x + c * aq.x, s * t2.y + c * aq.y);
      }
      __syncthreads();
      // columns p and q of A and of V
      for (int t = tid; t < half * n; t += nt) {
        const int j = t / n, x = t - j * n;
        const int p = pp[j], q = qq[j];
        if (q >= n || ss[j] == 0.0) continue;
        const double c = cs[j], s = ss[j];
        const double2 e = ph[j], ec = make_double2(e.x, -e.y);
        const double2 ap = A[x * n + p], aq = A[x * n + q];
        const double2 t1 = cmul(ec, aq), t2 = cmul(e, ap);
        A[x * n + p] = make_double2(c * ap.x - s * t1.x, c * ap.y - s * t1.y);
        A[x * n + q] = make_double2(s * t2.x + c * aq.x, s * t2.y + c * aq.y);
        const double2 vp = V[x * n + p], vq = V[x * n + q];
        const double2 u1 = cmul(ec, vq), u2 = cmul(e, vp);
        V[x * n + p] = make_double2(c * vp.x - s * u1.x, c * vp.y - s * u1.y);
        V[x * n + q] = make_double2(s * u2.x + c * vq.x, s * u2.y + c * vq.y);
      }
      __syncthreads();
      for (int j = tid; j < half; j += nt) {
        const int p = pp[j], q = qq[j];
        if (q < n && ss[j] != 0.0) {
          A[p * n + q] = make_double2(0.0, 0.0);
          A[q * n + p] = make_double2(0.0, 0.0);
        }
      }
      __syncthreads();
    }
  }
  // ascending order by rank (ties by index)
  for (int c = tid; c < n; c += nt) dg[c] = A[c * n + c].x;
  __syncthreads();
  for (int c = tid; c < n; c += nt) {
    const double x = dg[c];
    int rank = 0;
    for (int j = 0; j < n; ++j) rank += (dg[j] < x || (dg[j] == x && j < c)) ? 1 : 0;
    order[rank] = c;
  }
  __syncthreads();
  for (int c = tid; c < n; c += nt) w[c] = dg[order[c]];
  for (int e = tid; e < nn; e += nt) {
    const int r = e / n, c = e - r * n;
    U[(int64_t)r * ldu + c] = V[r * n + order[c]];
  }
}

// out[r][c] (row stride ldo) = sum_s part[s][r][c] over parts of rows x cols
__global__ void sum_parts_kernel(const double2* part, int nparts, int rows, int cols, double2* out, int ldo) {
  const int64_t n = (int64_t)rows * cols;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double sx = 0.0, sy = 0.0;
  for (int s = 0; s < nparts; ++s) {
    sx += part[(int64_t)s * n + e].x;
    sy += part[(int64_t)s * n + e].y;
  }
  out[(e / cols) * ldo + e % cols] = make_double2(sx, sy);
}

// C[j][r] /= (w[r] - lam[j]) for j < n1, r < rows: the spectral form of
// (w_r - M11)^-1 on coefficients in the eigenbasis of M11 (denominators
// below 1e-4 in magnitude are held there, as in the diagonal preconditioner)
__global__ void shift_scale_kernel(double2* C, const double* lam, const double* w, int64_t n1, int rows) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n1 * rows) return;
  const int64_t j = e / rows;
  const int r = (int)(e - j * rows);
  double den = w[r] - lam[j];
  if (fabs(den) < 1e-4) den = den < 0.0 ? -1e-4 : 1e-4;
  C[e] = make_double2(C[e].x / den, C[e].y / den);
}

// First stage of a sum over many parts of n elements: slice ps of the grid's
// y dimension sums parts ps, ps + nsl, ps + 2 nsl, ... into out[ps][e]; the
// four waves of a workgroup take every fourth of them for the same 64
// elements and are added in a fixed order
__global__ __launch_bounds__(256) void sum_parts_stage_kernel(const double2* part, int nparts, int64_t n,
                                                              double2* out) {
  __shared__ double2 acc[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ps = blockIdx.y, nsl = gridDim.y;
  const int64_t e = (int64_t)blockIdx.x * 64 + lane;
  double sx = 0.0, sy = 0.0;
  if (e < n)
    for (int s = ps + nsl * wave; s < nparts; s += 4 * nsl) {
      const double2 v = part[(int64_t)s * n + e];
      sx += v.x;
      sy += v.y;
    }
  acc[wave][lane] = make_double2(sx, sy);
  __syncthreads();
  if (wave == 0 && e < n) {
    double2 r = acc[0][lane];
    for (int w = 1; w < 4; ++w) {
      r.x += acc[w][lane].x;
      r.y += acc[w][lane].y;
    }
    out[(int64_t)ps * n + e] = r;
  }
}

// G[j][a] = conj(G[a][j]) for c0 <= j < m, a < c0 (the rows of new columns)
__global__ void gram_mirror_kernel(double2* G, int ldg, int c0, int m) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int nc = m - c0;
  if (e >= nc * c0) return;
  const int j = c0 + e / c0, a = e % c0;
  const double2 g = G[(int64_t)a * ldg + j];
  G[(int64_t)j * ldg + a] = make_double2(g.x, -g.y);
}

// when *flag is set: G[0:mc][0:mc] = diag(w[0:mc]) (the Gram matrix of the
// subspace collapsed onto Ritz vectors)
__global__ void gram_diag_kernel(const double* flag, const double* w, int mc, double2* G, int ldg) {
  if (*flag == 0.0) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mc * mc) return;
  const int a = e / mc, b = e % mc;
  G[(int64_t)a * ldg + b] = make_double2(a == b ? w[a] : 0.0, 0.0);
}

// out[r] = sum_b partial[r * nb + b]: one workgroup per row, a strided sum
// per thread and a fixed-order tree over the workgroup
__global__ __launch_bounds__(256) void row_sums_kernel(const double2* partial, int nb, double2* out) {
  __shared__ double sx[256], sy[256];
  const int r = blockIdx.x, t = threadIdx.x;
  double ax = 0.0, ay = 0.0;
  for (int b = t; b < nb; b += 256) {
    ax += partial[(int64_t)r * nb + b].x;
    ay += partial[(int64_t)r * nb + b].y;
  }
  sx[t] = ax;
  sy[t] = ay;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      sx[t] += sx[t + w];
      sy[t] += sy[t + w];
    }
    __syncthreads();
  }
  if (t == 0) out[r] = make_double2(sx[0], sy[0]);
}

// Convergence of the k roots: root r is converged when |r_r| <= par[0] and
// |w_r - wold_r| <= par[1]; wold <- w.  rep = [status, w[k], |r|[k], conv[k],
// (two counts written later), collapse] with status 1 (all converged), 0 (not
// all) or -1 (a non-finite value), and collapse = 1 when the subspace of m
// vectors cannot take one new direction per unconverged root (m + nn > mmax).
__global__ void dav_converge_kernel(const double* w, const double2* rn2, double* wold, int k, int m, int mmax,
                                    const double* par, double* rep) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double tol = par[0], dwtol = par[1];
  int all = 1, finite = 1, nn = 0;
  for (int r = 0; r < k; ++r) {
    const double rn = sqrt(fmax(0.0, rn2[r].x));
    if (!isfinite(w[r]) || !isfinite(rn)) finite = 0;
    const int c = (rn <= tol && fabs(w[r] - wold[r]) <= dwtol) ? 1 : 0;
    all = all && c;
    nn += 1 - c;
    rep[1 + r] = w[r];
    rep[1 + k + r] = rn;
    rep[1 + 2 * k + r] = c;
    wold[r] = w[r];
  }
  rep[0] = finite ? all : -1;
  rep[3 + 3 * k] = (finite && !all && m + nn > mmax) ? 1.0 : 0.0;
}

// Out[r][i] = alpha sum_a C[a][r] In[a][i] + beta Out[r][i] for r < nr,
// a < m (C row stride ldc), skipped when flag is given and *flag is zero.
// Tall and skinny (a few rows over a long dim): one thread per column i,
// outputs in groups of NQ so that In is read once per group; the group's C
// entries are staged in LDS, and four rows of In are loaded at once.
template <int NQ>
__global__ __launch_bounds__(256) void combine_cols_kernel(const double* flag, const double2* C, int ldc, int m,
                                                           int nr, const double2* In, double2* Out, int64_t dim,
                                                           cplx alpha, cplx beta) {
  if (flag && *flag == 0.0) return;
  extern __shared__ double2 cs[];  // [m][NQ]
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < dim;
  const bool has_beta = beta.re != 0.0 || beta.im != 0.0;
  for (int r0 = 0; r0 < nr; r0 += NQ) {
    const int nq = nr - r0 < NQ ? nr - r0 : NQ;
    __syncthreads();
    for (int e = threadIdx.x; e < m * NQ; e += blockDim.x) {
      const int a = e / NQ, j = e % NQ;
      cs[e] = j < nq ? C[(int64_t)a * ldc + r0 + j] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (!live) continue;
    double ax[NQ], ay[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j) ax[j] = ay[j] = 0.0;
    const double2* col = In + i;
    int a = 0;
    for (; a + 4 <= m; a += 4) {
      double2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = col[(int64_t)(a + u) * dim];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
          const double2 c = cs[(a + u) * NQ + j];
          ax[j] += c.x * v[u].x - c.y * v[u].y;
          ay[j] += c.x * v[u].y + c.y * v[u].x;
        }
    }
    for (; a < m; ++a) {
      const double2 v = col[(int64_t)a * dim];
#pragma unroll
      for (int j = 0; j < NQ; ++j) {
        const double2 c = cs[a * NQ + j];
        ax[j] += c.x * v.x - c.y * v.y;
        ay[j] += c.x * v.y + c.y * v.x;
      }
    }
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      if (j < nq) {
        double2* o = Out + (int64_t)(r0 + j) * dim + i;
        double2 r = make_double2(alpha.re * ax[j] - alpha.im * ay[j], alpha.re * ay[j] + alpha.im * ax[j]);
        if (has_beta) {
          const double2 b = *o;
          r.x += beta.re * b.x - beta.im * b.y;
          r.y += beta.re * b.y + beta.im * b.x;
        }
        *o = r;
      }
    }
  }
}

// when *flag is set: Out[r] = T[r] for r < mc, Out[r] = 0 for mc <= r < m
__global__ void collapse_copy_kernel(const double* flag, const double2* T, double2* Out, int m, int mc, int64_t dim) {
  if (*flag == 0.0) return;
  const int64_t total = (int64_t)m * dim;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    Out[e] = e < (int64_t)mc * dim ? T[e] : make_double2(0.0, 0.0);
}

// Olsen's correction of the preconditioned residuals, N_r -= (a_r / b_r) P_r;
// rows whose flag is set (converged roots) are zeroed instead
__global__ void olsen_kernel(double2* N, const double2* P, const double2* a, const double2* b, const double* flags,
                             int rows, int64_t dim) {
  const int64_t total = (int64_t)rows * dim;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / dim);
    if (flags[r] != 0.0) {
      N[e] = make_double2(0.0, 0.0);
      continue;
    }
    const double2 bb = b[r], aa = a[r];
    const double den = bb.x * bb.x + bb.y * bb.y;
    if (den < 1e-300) continue;
    const double2 f = make_double2((aa.x * bb.x + aa.y * bb.y) / den, (aa.y * bb.x - aa.x * bb.y) / den);
    const double2 p = P[e];
    N[e].x -= f.x * p.x - f.y * p.y;
    N[e].y -= f.x * p.y + f.y * p.x;
  }
}

// Canonical orthonormalisation coefficients of k vectors from the
// eigenpairs (lam ascending, columns of U) of their Gram matrix: the
// eigenvalues above 1e-12 of the largest (and above 1e-20) are kept; kept
// direction c (ascending) is sum_a U[a][j] / sqrt(lam_j) * vector a, so
// C[a][c] = U[a][j] / sqrt(lam_j), and the columns past the kept count are
// zero.  *count gets the kept count, or -1 for a non-finite eigenvalue.
__global__ void canon_kernel(const double* lam, const double2* U, int ldu, int k, double2* C, double* count) {
  __shared__ int nk, lo;
  if (threadIdx.x == 0) {
    double lmax = 0.0;
    int finite = 1;
    for (int j = 0; j < k; ++j) {
      if (!isfinite(lam[j])) finite = 0;
      lmax = fmax(lmax, lam[j]);
    }
    int c = 0;
    for (int j = 0; j < k; ++j)
      if (lam[j] > 1e-12 * fmax(lmax, 1e-300) && lam[j] > 1e-20) ++c;
    nk = finite ? c : 0;
    lo = k - nk;
    *count = finite ? (double)c : -1.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int a = e / k, c = e - a * k;
    double2 v = make_double2(0.0, 0.0);
    if (c < nk) {
      const int j = lo + c;
      const double f = 1.0 / sqrt(lam[j]);
      const double2 u = U[(int64_t)a * ldu + j];
      v = make_double2(u.x * f, u.y * f);
    }
    C[e] = v;
  }
}

}  // namespace

int heev_device_max() { return kJacobiMaxN; }

size_t heev_lds_bytes(int n, int mode) { return sizeof(double2) * (size_t)mode * n * n; }

size_t heev_static_lds() {
  hipFuncAttributes a{};
  if (hipFuncGetAttributes(&a, (const void*)heev_jacobi_kernel) != hipSuccess) {
    (void)hipGetLastError();
    return 16384;
  }
  return a.sharedSizeBytes;
}

void launch_heev_jacobi(const double2* G, int ldg, int n, double2* Aw, double2* Vw, int mode, double2* U, int ldu,
                        double* w, hipStream_t s) {
  hipLaunchKernelGGL(heev_jacobi_kernel, dim3(1), dim3(kJacobiThreads), heev_lds_bytes(n, mode), s, G, ldg, n, Aw,
                     Vw, mode, U, ldu, w);
}

void heev_allow_lds(size_t bytes) {
  (void)hipFuncSetAttribute((const void*)heev_jacobi_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  (void)hipGetLastError();
}

void launch_shift_scale(double2* C, const double* lam, const double* w, int64_t n1, int rows, hipStream_t s) {
  const int64_t n = n1 * rows;
  if (n <= 0) return;
  hipLaunchKernelGGL(shift_scale_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, C, lam, w, n1, rows);
}

int sum_parts_slices(int nparts) { return nparts > 64 ? 32 : 1; }

void launch_sum_parts(const double2* part, int nparts, int rows, int cols, double2* stage, double2* out, int ldo,
                      hipStream_t s) {
  const int64_t n = (int64_t)rows * cols;
  if (n <= 0) return;
  const int nsl = sum_parts_slices(nparts);
  if (nsl > 1) {
    if (!stage) throw HipError{hipErrorInvalidValue, "sum_parts: no staging buffer"};
    hipLaunchKernelGGL(sum_parts_stage_kernel, dim3((unsigned)((n + 63) / 64), (unsigned)nsl), dim3(256), 0, s, part,
                       nparts, n, stage);
    part = stage;
    nparts = nsl;
  }
  hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, nparts, rows, cols,
                     out, ldo);
}

void launch_gram_mirror(double2* G, int ldg, int c0, int m, hipStream_t s) {
  const int n = (m - c0) * c0;
  if (n <= 0) return;
  hipLaunchKernelGGL(gram_mirror_kernel, dim3((n + 255) / 256), dim3(256), 0, s, G, ldg, c0, m);
}

void launch_gram_diag(const double* flag, const double* w, int mc, double2* G, int ldg, hipStream_t s) {
  hipLaunchKernelGGL(gram_diag_kernel, dim3((mc * mc + 255) / 256), dim3(256), 0, s, flag, w, mc, G, ldg);
}

void launch_combine_cols(const double* flag, const double2* C, int ldc, int m, int nr, const double2* In,
                         double2* Out, int64_t dim, cplx alpha, cplx beta, hipStream_t s) {
  if (m <= 0 || nr <= 0 || dim <= 0) return;
  if (m > kCombineMaxM) throw HipError{hipErrorInvalidValue, "combination over more than 256 rows"};
  const dim3 grid((unsigned)((dim + 255) / 256));
  if (nr <= 8)
    hipLaunchKernelGGL(combine_cols_kernel<8>, grid, dim3(256), sizeof(double2) * 8 * m, s, flag, C, ldc, m, nr, In,
                       Out, dim, alpha, beta);
  else
    hipLaunchKernelGGL(combine_cols_kernel<16>, grid, dim3(256), sizeof(double2) * 16 * m, s, flag, C, ldc, m, nr,
                       In, Out, dim, alpha, beta);
}

void launch_row_sums(const double2* partial, int nb, int rows, double2* out, hipStream_t s) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(row_sums_kernel, dim3((unsigned)rows), dim3(256), 0, s, partial, nb, out);
}

void launch_dav_converge(const double* w, const double2* rn2, double* wold, int k, int m, int mmax,
                         const double* par, double* rep, hipStream_t s) {
  hipLaunchKernelGGL(dav_converge_kernel, dim3(1), dim3(64), 0, s, w, rn2, wold, k, m, mmax, par, rep);
}

void launch_collapse(const double* flag, const double2* U, int ldu, int m, int mc, const double2* In, double2* T,
                     double2* Out, int64_t dim, hipStream_t s) {
  launch_combine_cols(flag, U, ldu, m, mc, In, T, dim, {1.0, 0.0}, {0.0, 0.0}, s);
  const int64_t total = (int64_t)m * dim;
  int64_t g = (total + 255) / 256;
  // a grid-stride copy: a few thousand workgroups keep HBM busy when the
  // flag is set and cost little to launch when it is not (the usual case)
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(collapse_copy_kernel, dim3((unsigned)g), dim3(256), 0, s, flag, T, Out, m, mc, dim);
}

void launch_olsen(double2* N, const double2* P, const double2* a, const double2* b, const double* flags, int rows,
                  int64_t dim, hipStream_t s) {
  const int64_t total = (int64_t)rows * dim;
  int64_t g = (total + 255) / 256;
  if (g > 65535LL * 16) g = 65535LL * 16;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(olsen_kernel, dim3((unsigned)g), dim3(256), 0, s, N, P, a, b, flags, rows, dim);
}

void launch_canon(const double* lam, const double2* U, int ldu, int k, double2* C, double* count, hipStream_t s) {
  hipLaunchKernelGGL(canon_kernel, dim3(1), dim3(256), 0, s, lam, U, ldu, k, C, count);
}

}  // namespace adc
