// One-time FP64 factorisation of the fixed KKT system of eq. (7b) on the GPU.
//
// F and A are block diagonal with identical per-axis blocks, so
// [[I + rho F^T F, A^T], [A, 0]] splits into identical per-axis systems
// [[Q, A_ax^T], [A_ax, 0]] with Q = I + rho (n_obs P^T P + Pdot^T Pdot +
// Pddot^T Pddot) (n_coeff x n_coeff, built on the host in FP64).  Its inverse
// is formed by the range-space method:
//   Q = R R^T (Cholesky),   Y = Q^-1 A^T,   S = A Y = C C^T (Cholesky),
//   M12 = Y S^-1,   M11 = Q^-1 - M12 Y^T,   Pi = M11 Q,
// so that xi_bar = M11 eta_top + M12 b.  The system is tiny (<= 16 + 6
// unknowns) and solved once per problem shape; a single lane does it in
// FP64 and writes FP64 and FP32 copies.  A non-positive pivot of S means the
// selected boundary rows are linearly dependent: flag = PRIEST_ERR_SINGULAR.
#include "priest_internal.h"

namespace priest {
namespace {

constexpr int kE = 6;

__device__ bool chol_inplace(double* a, int n, int ld) {
  double mx = 0.0;
  for (int i = 0; i < n; ++i) mx = fmax(mx, fabs(a[i * ld + i]));
  for (int j = 0; j < n; ++j) {
    double d = a[j * ld + j];
    for (int k = 0; k < j; ++k) d -= a[j * ld + k] * a[j * ld + k];
    if (!(d > 1e-13 * mx)) return false;
    d = sqrt(d);
    a[j * ld + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = a[i * ld + j];
      for (int k = 0; k < j; ++k) s -= a[i * ld + k] * a[j * ld + k];
      a[i * ld + j] = s / d;
    }
  }
  return true;
}

// Solve (L L^T) x = b in place for a lower factor L (leading dim ld).
__device__ void chol_solve(const double* L, int n, int ld, double* x) {
  for (int i = 0; i < n; ++i) {
    double s = x[i];
    for (int k = 0; k < i; ++k) s -= L[i * ld + k] * x[k];
    x[i] = s / L[i * ld + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    for (int k = i + 1; k < n; ++k) s -= L[k * ld + i] * x[k];
    x[i] = s / L[i * ld + i];
  }
}

__global__ void kkt_kernel(const double* Qin, const double* Ain, int nv, int E, const int* rowsel,
                           double* out64, float* M11f, float* Pif, float* M12f, int* flag) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double R[kMaxNV * kMaxNV], Qi[kMaxNV * kMaxNV], Y[kMaxNV * kE], Sm[kE * kE];
  double M12[kMaxNV * kE], M11[kMaxNV * kMaxNV], col[kMaxNV];
  for (int i = 0; i < nv * nv; ++i) R[i] = Qin[i];
  if (!chol_inplace(R, nv, nv)) { *flag = PRIEST_ERR_SINGULAR; return; }
  for (int j = 0; j < nv; ++j) {
    for (int i = 0; i < nv; ++i) col[i] = (i == j) ? 1.0 : 0.0;
    chol_solve(R, nv, nv, col);
    for (int i = 0; i < nv; ++i) Qi[i * nv + j] = col[i];
  }
  for (int r = 0; r < E; ++r) {
    for (int i = 0; i < nv; ++i) {
      double s = 0.0;
      for (int k = 0; k < nv; ++k) s += Qi[i * nv + k] * Ain[r * nv + k];
      Y[i * kE + r] = s;
    }
  }
  for (int r = 0; r < E; ++r)
    for (int c = 0; c < E; ++c) {
      double s = 0.0;
      for (int k = 0; k < nv; ++k) s += Ain[r * nv + k] * Y[k * kE + c];
      Sm[r * kE + c] = s;
    }
  if (E > 0 && !chol_inplace(Sm, E, kE)) { *flag = PRIEST_ERR_SINGULAR; return; }
  // M12 = Y S^-1 (rows of Y solved against S, which is symmetric)
  for (int i = 0; i < nv; ++i) {
    double x[kE];
    for (int r = 0; r < E; ++r) x[r] = Y[i * kE + r];
    if (E > 0) chol_solve(Sm, E, kE, x);
    for (int r = 0; r < E; ++r) M12[i * kE + r] = x[r];
  }
  for (int i = 0; i < nv; ++i)
    for (int j = 0; j < nv; ++j) {
      double s = Qi[i * nv + j];
      for (int r = 0; r < E; ++r) s -= M12[i * kE + r] * Y[j * kE + r];
      M11[i * nv + j] = s;
    }
  for (int i = 0; i < nv; ++i)
    for (int j = 0; j < nv; ++j) {
      double s = 0.0;
      for (int k = 0; k < nv; ++k) s += M11[i * nv + k] * Qin[k * nv + j];
      out64[nv * nv + i * nv + j] = s;
      Pif[i * nv + j] = static_cast<float>(s);
      out64[i * nv + j] = M11[i * nv + j];
      M11f[i * nv + j] = static_cast<float>(M11[i * nv + j]);
    }
  for (int i = 0; i < nv; ++i) {
    for (int c = 0; c < 6; ++c) M12f[i * 6 + c] = 0.0f;
    for (int r = 0; r < E; ++r) {
      out64[2 * nv * nv + i * kE + r] = M12[i * kE + r];
      M12f[i * 6 + rowsel[r]] = static_cast<float>(M12[i * kE + r]);
    }
  }
  *flag = PRIEST_OK;
}

}  // namespace

hipError_t launch_kkt(const double* Q, const double* A, int nv, int E, const int* rowsel,
                      double* out64, float* M11, float* Pi, float* M12, int* flag,
                      hipStream_t s) {
  hipLaunchKernelGGL(kkt_kernel, dim3(1), dim3(64), 0, s, Q, A, nv, E, rowsel, out64, M11, Pi,
                     M12, flag);
  return hipGetLastError();
}

}  // namespace priest
