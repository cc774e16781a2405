// One-step pivoted Cholesky of the electron-repulsion matrix (Section 2.5,
// eq. 41 and the one-step procedure) and the transform of the vectors to the
// molecular spinor basis (eq. 42), on the device.
//
// Step k takes the largest remaining diagonal element d_p of V - sum_{q<k}
// L_q L_q^T; below tau (or not positive) the procedure ends, otherwise
//     L_k[i] = (V[p][i] - sum_{q<k} L_q[i] L_q[p]) / sqrt(d_p),   d_i -= L_k[i]^2.
// Every step is two launches on the caller's stream: a one-block argmax
// reduction of d into a small state record, then the column update over i
// (row p of the symmetric V read along i, the L_q[p] of earlier vectors
// staged in LDS).  The stopping test is made on the device, so the host
// enqueues steps in batches and reads the state once per batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/adc.h"
#include "internal.h"

namespace adc {

namespace {

struct CholState {
  double dmax;   // largest remaining diagonal element of the current step
  long long p;   // its index
  int count;     // vectors made
  int done;      // 1 once the procedure has ended
  int bad;       // number of non-finite diagonal elements of V
};

__global__ __launch_bounds__(256) void chol_init_kernel(const double* V, int64_t m, double* d, CholState* st) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const double x = V[i * m + i];
    d[i] = x;
    bad += isfinite(x) ? 0 : 1;
  }
  __shared__ int sb[256];
  sb[threadIdx.x] = bad;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sb[threadIdx.x] += sb[threadIdx.x + w];
    __syncthreads();
  }
  // one block (the launch below uses a single block)
  if (threadIdx.x == 0) {
    st->dmax = 0.0;
    st->p = 0;
    st->count = 0;
    st->done = sb[0] > 0 ? 1 : 0;
    st->bad = sb[0];
  }
}

// largest d[i]; among equal values the lowest index
__global__ __launch_bounds__(1024) void chol_argmax_kernel(const double* d, int64_t m, CholState* st) {
  if (st->done) return;
  double best = -INFINITY;
  int64_t bi = m;
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
    const double x = d[i];
    if (x > best) {
      best = x;
      bi = i;
    }
  }
  __shared__ double sv[1024];
  __shared__ long long si[1024];
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double a = sv[threadIdx.x], b = sv[threadIdx.x + w];
      const long long ia = si[threadIdx.x], ib = si[threadIdx.x + w];
      if (b > a || (b == a && ib < ia)) {
        sv[threadIdx.x] = b;
        si[threadIdx.x] = ib;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    st->dmax = sv[0];
    st->p = si[0];
  }
}

// vector k of the factor; L is [max_vec][m]
__global__ __launch_bounds__(256) void chol_column_kernel(const double* V, int64_t m, double tau, double* L, int k,
                                                          double* d, int* piv, CholState* st) {
  if (st->done) return;
  const double dmax = st->dmax;
  const int64_t p = st->p;
  if (!(dmax > 0.0) || dmax < tau || p >= m) {
    if (blockIdx.x == 0 && threadIdx.x == 0) st->done = 1;
    return;
  }
  __shared__ double lp[256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = i < m ? V[p * m + i] : 0.0;
  for (int q0 = 0; q0 < k; q0 += 256) {
    const int nq = min(256, k - q0);
    __syncthreads();
    if ((int)threadIdx.x < nq) lp[threadIdx.x] = L[(int64_t)(q0 + threadIdx.x) * m + p];
    __syncthreads();
    if (i < m)
      for (int q = 0; q < nq; ++q) acc -= L[(int64_t)(q0 + q) * m + i] * lp[q];
  }
  if (i < m) {
    const double l = acc / sqrt(dmax);
    L[(int64_t)k * m + i] = l;
    d[i] -= l * l;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    piv[k] = (int)p;
    st->count = k + 1;
  }
}

// packed pairs mu <= nu of n_vec vectors -> symmetric complex [n_vec][n][n]
__global__ __launch_bounds__(256) void chol_unpack_kernel(const double* Lp, int64_t nvec, int n, double2* out) {
  const int64_t np = (int64_t)n * (n + 1) / 2;
  const int64_t total = nvec * n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t P = e / ((int64_t)n * n), r = e - P * n * n;
    int mu = (int)(r / n), nu = (int)(r - (int64_t)mu * n);
    if (mu > nu) {
      const int t = mu;
      mu = nu;
      nu = t;
    }
    // pair (mu, nu), mu <= nu, in row-major upper-triangle order
    const int64_t pr = (int64_t)mu * n - (int64_t)mu * (mu - 1) / 2 + (nu - mu);
    out[e] = make_double2(Lp[P * np + pr], 0.0);
  }
}

}  // namespace
}  // namespace adc

using namespace adc;

extern "C" {

int adc_cholesky(const double* V, long long m, double tau, int max_vec, double* L, int* pivots, int* n_vec,
                 void* stream) {
  if (!V || m < 1 || max_vec < 0 || !(tau >= 0.0) || !std::isfinite(tau) || !n_vec || (max_vec > 0 && (!L || !pivots)))
    return ADC_ERR_INVALID_ARG;
  if (m > (1LL << 31) - 1) return ADC_ERR_INVALID_ARG;
  *n_vec = 0;
  if (max_vec == 0) return ADC_OK;
  hipStream_t s = (hipStream_t)stream;
  double* d = nullptr;
  CholState* st = nullptr;
  int* piv = nullptr;
  auto cleanup = [&]() {
    if (d) (void)hipFree(d);
    if (st) (void)hipFree(st);
    if (piv) (void)hipFree(piv);
  };
  if (hipMalloc(&d, sizeof(double) * m) != hipSuccess || hipMalloc(&st, sizeof(CholState)) != hipSuccess ||
      hipMalloc(&piv, sizeof(int) * max_vec) != hipSuccess) {
    (void)hipGetLastError();
    cleanup();
    return ADC_ERR_OUT_OF_MEMORY;
  }
  hipLaunchKernelGGL(chol_init_kernel, dim3(1), dim3(256), 0, s, V, (int64_t)m, d, st);
  const unsigned ncol = (unsigned)((m + 255) / 256);
  CholState hs{};
  int rc = ADC_OK;
  for (int k0 = 0; k0 < max_vec; k0 += 32) {
    const int k1 = std::min(max_vec, k0 + 32);
    for (int k = k0; k < k1; ++k) {
      hipLaunchKernelGGL(chol_argmax_kernel, dim3(1), dim3(1024), 0, s, d, (int64_t)m, st);
      hipLaunchKernelGGL(chol_column_kernel, dim3(ncol), dim3(256), 0, s, V, (int64_t)m, tau, L, k, d, piv, st);
    }
    if (hipMemcpyAsync(&hs, st, sizeof(CholState), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = ADC_ERR_HIP;
      break;
    }
    if (hs.bad > 0) {
      rc = ADC_ERR_NONFINITE_INPUT;
      break;
    }
    if (hs.done) break;
  }
  if (rc == ADC_OK && hipGetLastError() != hipSuccess) rc = ADC_ERR_HIP;
  if (rc == ADC_OK) {
    *n_vec = hs.count;
    if (hs.count > 0) {
      std::vector<int> hp(hs.count);
      if (hipMemcpy(hp.data(), piv, sizeof(int) * hs.count, hipMemcpyDeviceToHost) != hipSuccess) rc = ADC_ERR_HIP;
      else std::copy(hp.begin(), hp.end(), pivots);
    }
  }
  (void)hipGetLastError();
  cleanup();
  return rc;
}

int adc_cholesky_mo(const double* Lp, int n_vec, int n_ao, const void* C, int n_mo, void* Lmo, void* stream) {
  if (!Lp || !C || !Lmo || n_vec < 0 || n_ao < 1 || n_mo < 1) return ADC_ERR_INVALID_ARG;
  if (n_vec == 0) return ADC_OK;
  try {
    Ctx cx;
    cx.stream = (hipStream_t)stream;
    const int64_t n = n_ao, nm = n_mo, nv = n_vec;
    Tensor Lc = tnew(cx, {nv, n, n}, false);
    hipLaunchKernelGGL(chol_unpack_kernel, dim3((unsigned)std::min<int64_t>((nv * n * n + 255) / 256, 65535 * 16)),
                       dim3(256), 0, cx.stream, Lp, nv, n_ao, Lc.p);
    // T[P][mu][q] = sum_nu L[P][mu][nu] C[nu][q]
    Tensor T = tnew(cx, {nv, n, nm}, false);
    GemmDesc g{};
    g.M = n; g.N = nm; g.K = n; g.batch = nv;
    g.A = Lc.p; g.sam = n; g.sak = 1; g.sab = n * n;
    g.B = (const double2*)C; g.sbk = nm; g.sbn = 1; g.sbb = 0;
    g.C = T.p; g.scm = nm; g.scn = 1; g.scb = n * nm;
    g.alpha = C1(); g.beta = C0();
    gemm(cx, g);
    // Lmo[P][p][q] = sum_mu conj(C[mu][p]) T[P][mu][q]
    GemmDesc h{};
    h.M = nm; h.N = nm; h.K = n; h.batch = nv;
    h.A = (const double2*)C; h.sam = 1; h.sak = nm; h.sab = 0; h.conjA = 1;
    h.B = T.p; h.sbk = nm; h.sbn = 1; h.sbb = n * nm;
    h.C = (double2*)Lmo; h.scm = nm; h.scn = 1; h.scb = nm * nm;
    h.alpha = C1(); h.beta = C0();
    gemm(cx, h);
    hipcheck(hipStreamSynchronize(cx.stream), "cholesky mo");
    tfree(cx, Lc);
    tfree(cx, T);
    hipcheck(hipGetLastError(), "cholesky mo launch");
  } catch (const HipError& e) {
    (void)hipGetLastError();
    return e.e == hipErrorOutOfMemory ? ADC_ERR_OUT_OF_MEMORY : ADC_ERR_HIP;
  } catch (...) {
    return ADC_ERR_HIP;
  }
  return ADC_OK;
}

}  // extern "C"
