// Host-side float64 parts of the library: Pauli-transfer matrices of noisy
// gates (Sec. 2.2.1), the noise-strength extrapolations of Sec. 2.2.2 (B) and
// App. B.2, the fidelity extrapolation of Sec. 2.2.2 (A) with App. B.1's
// criterion, and the error strings.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <cstdlib>
#include <vector>

#include "nze.h"
#include "nze_internal.h"

namespace nze {

thread_local std::string g_last_error;

int fail(int code, const char* msg) {
  g_last_error = msg;
  return code;
}

}  // namespace nze

using nze::fail;
typedef std::complex<double> cplx;

// ------------------------------------------------------------------ PTMs

namespace {

// sigma_0..3 = I, X, Y, Z
void pauli1(int p, cplx m[2][2]) {
  const cplx I(0, 1);
  switch (p) {
    case 0: m[0][0] = 1; m[0][1] = 0; m[1][0] = 0; m[1][1] = 1; break;
    case 1: m[0][0] = 0; m[0][1] = 1; m[1][0] = 1; m[1][1] = 0; break;
    case 2: m[0][0] = 0; m[0][1] = -I; m[1][0] = I; m[1][1] = 0; break;
    default: m[0][0] = 1; m[0][1] = 0; m[1][0] = 0; m[1][1] = -1; break;
  }
}

// 4x4 matrix of the two-qubit Pauli P = 4*p_left + p_right; the left qubit is
// the more significant bit of the computational-basis index.
void pauli2(int P, cplx m[4][4]) {
  cplx a[2][2], b[2][2];
  pauli1(P >> 2, a);
  pauli1(P & 3, b);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) m[i][j] = a[i >> 1][j >> 1] * b[i & 1][j & 1];
}

void matmul4(const cplx a[4][4], const cplx b[4][4], cplx c[4][4]) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cplx s = 0;
      for (int k = 0; k < 4; ++k) s += a[i][k] * b[k][j];
      c[i][j] = s;
    }
}

// R[P][Q] = Tr(P U Q U^dag) / 4
void unitary_ptm(const cplx U[4][4], double R[16][16]) {
  cplx Ud[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) Ud[i][j] = std::conj(U[j][i]);
  cplx P[16][4][4];
  for (int p = 0; p < 16; ++p) pauli2(p, P[p]);
  for (int q = 0; q < 16; ++q) {
    cplx t[4][4], m[4][4];
    matmul4(U, P[q], t);
    matmul4(t, Ud, m);
    for (int p = 0; p < 16; ++p) {
      cplx tr = 0;
      for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 4; ++k) tr += P[p][i][k] * m[k][i];
      R[p][q] = tr.real() / 4.0;
    }
  }
}

void mul16(const double A[16][16], const double B[16][16], double C[16][16]) {
  double T[16][16];
  for (int i = 0; i < 16; ++i)
    for (int j = 0; j < 16; ++j) {
      double s = 0;
      for (int k = 0; k < 16; ++k) s += A[i][k] * B[k][j];
      T[i][j] = s;
    }
  std::memcpy(C, T, sizeof(T));
}

// Single-qubit channel PTM a (4x4) applied to both qubits: (a (x) a).
void both_qubits(const double a[4][4], double R[16][16]) {
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q < 4; ++q)
      for (int pp = 0; pp < 4; ++pp)
        for (int qq = 0; qq < 4; ++qq)
          R[4 * p + q][4 * pp + qq] = a[p][pp] * a[q][qq];
}

}  // namespace

extern "C" int nze_build_ptm(const double* u_re, const double* u_im,
                             const nze_noise* noise, double scale,
                             double* ptm_out) {
  if (!u_re || !u_im || !ptm_out) return fail(NZE_EINVAL, "null argument");
  nze_noise nz = {0, 0, 0, 0, 0};
  if (noise) nz = *noise;
  const double dep = nz.dep * scale, ad = nz.ad * scale;
  const double px = nz.px * scale, py = nz.py * scale, pz = nz.pz * scale;
  if (!(dep >= 0 && dep <= 1 && ad >= 0 && ad <= 1 && px >= 0 && py >= 0 &&
        pz >= 0 && px + py + pz <= 1))
    return fail(NZE_EINVAL, "noise parameters outside [0, 1]");
  cplx U[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) U[i][j] = cplx(u_re[4 * i + j], u_im[4 * i + j]);
  double R[16][16];
  unitary_ptm(U, R);
  if (dep != 0.0) {
    // rho -> (1 - dep) rho + dep I/4 (App. C.2.1) keeps I, scales the rest
    for (int p = 1; p < 16; ++p)
      for (int q = 0; q < 16; ++q) R[p][q] *= (1.0 - dep);
  }
  if (ad != 0.0) {
    const double s = std::sqrt(1.0 - ad);
    const double a[4][4] = {{1, 0, 0, 0}, {0, s, 0, 0}, {0, 0, s, 0},
                            {ad, 0, 0, 1.0 - ad}};
    double C[16][16];
    both_qubits(a, C);
    mul16(C, R, R);
  }
  if (px != 0.0 || py != 0.0 || pz != 0.0) {
    const double a[4][4] = {{1, 0, 0, 0},
                            {0, 1 - 2 * (py + pz), 0, 0},
                            {0, 0, 1 - 2 * (px + pz), 0},
                            {0, 0, 0, 1 - 2 * (px + py)}};
    double C[16][16];
    both_qubits(a, C);
    mul16(C, R, R);
  }
  for (int p = 0; p < 16; ++p)
    for (int q = 0; q < 16; ++q) ptm_out[16 * p + q] = R[p][q];
  return NZE_OK;
}

namespace {

// Single-qubit Paulis a and b anticommute iff both differ from I and from
// each other.
inline int anti1(int a, int b) { return (a != 0 && b != 0 && a != b) ? 1 : 0; }

// Eigenvalues of a Pauli channel rho -> sum_s p_s s rho s on the Pauli basis:
// f_t = sum_s p_s (-1)^[s and t anticommute].  nq = 1 or 2 qubits; the
// probabilities are p_s = lambda * rates[s] for s != I and the rest on I.
bool pauli_channel_diag(int nq, const double* rates, double lambda, double* f) {
  const int n = nq == 1 ? 4 : 16;
  double p[16], tot = 0.0;
  for (int s = 1; s < n; ++s) {
    if (!(rates[s] >= 0.0)) return false;
    p[s] = lambda * rates[s];
    tot += p[s];
  }
  p[0] = 1.0 - tot;
  if (!(lambda >= 0.0) || !(p[0] >= 0.0) || !(p[0] <= 1.0)) return false;
  for (int t = 0; t < n; ++t) {
    double v = 0.0;
    for (int s = 0; s < n; ++s) {
      const int anti = nq == 1 ? anti1(s, t) : anti1(s >> 2, t >> 2) + anti1(s & 3, t & 3);
      v += (anti & 1) ? -p[s] : p[s];
    }
    f[t] = v;
  }
  return true;
}

}  // namespace

extern "C" int nze_build_ptm_pauli(const double* u_re, const double* u_im,
                                   const double* rates, double lambda,
                                   double* ptm_out) {
  if (!u_re || !u_im || !rates || !ptm_out) return fail(NZE_EINVAL, "null argument");
  double f[16];
  if (!pauli_channel_diag(2, rates, lambda, f))
    return fail(NZE_EINVAL, "Pauli error rates give probabilities outside [0, 1]");
  cplx U[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) U[i][j] = cplx(u_re[4 * i + j], u_im[4 * i + j]);
  double R[16][16];
  unitary_ptm(U, R);
  for (int p = 0; p < 16; ++p)
    for (int q = 0; q < 16; ++q) ptm_out[16 * p + q] = f[p] * R[p][q];
  return NZE_OK;
}

extern "C" int nze_ptm_compose_1q(const double* ptm_in, const double* u_re,
                                  const double* u_im, const double* rates,
                                  double lambda, int32_t qubit, int32_t after,
                                  double* ptm_out) {
  if (!ptm_in || !u_re || !u_im || !rates || !ptm_out)
    return fail(NZE_EINVAL, "null argument");
  if (qubit != 0 && qubit != 1) return fail(NZE_EINVAL, "qubit must be 0 (left) or 1 (right)");
  double f[4];
  if (!pauli_channel_diag(1, rates, lambda, f))
    return fail(NZE_EINVAL, "Pauli error rates give probabilities outside [0, 1]");
  // r[p][q] = f_p Tr(s_p u s_q u^dagger) / 2
  cplx u[2][2], ud[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) u[i][j] = cplx(u_re[2 * i + j], u_im[2 * i + j]);
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) ud[i][j] = std::conj(u[j][i]);
  double r[4][4];
  for (int q = 0; q < 4; ++q) {
    cplx sq[2][2], t[2][2], m[2][2];
    pauli1(q, sq);
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) t[i][j] = u[i][0] * sq[0][j] + u[i][1] * sq[1][j];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) m[i][j] = t[i][0] * ud[0][j] + t[i][1] * ud[1][j];
    for (int p = 0; p < 4; ++p) {
      cplx sp[2][2];
      pauli1(p, sp);
      cplx tr = 0;
      for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 2; ++k) tr += sp[i][k] * m[k][i];
      r[p][q] = f[p] * tr.real() / 2.0;
    }
  }
  // embedding on the pair, index 4 p_left + p_right
  double E[16][16] = {};
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      for (int c = 0; c < 4; ++c)
        for (int d = 0; d < 4; ++d)
          E[4 * a + b][4 * c + d] = qubit == 0 ? (b == d ? r[a][c] : 0.0)
                                              : (a == c ? r[b][d] : 0.0);
  double Rin[16][16], Rout[16][16];
  for (int p = 0; p < 16; ++p)
    for (int q = 0; q < 16; ++q) Rin[p][q] = ptm_in[16 * p + q];
  if (after) mul16(E, Rin, Rout);
  else mul16(Rin, E, Rout);
  for (int p = 0; p < 16; ++p)
    for (int q = 0; q < 16; ++q) ptm_out[16 * p + q] = Rout[p][q];
  return NZE_OK;
}

extern "C" int nze_ptm_compose(const double* first, const double* second,
                               double* ptm_out) {
  if (!first || !second || !ptm_out) return fail(NZE_EINVAL, "null argument");
  double A[16][16], B[16][16], C[16][16];
  for (int p = 0; p < 16; ++p)
    for (int q = 0; q < 16; ++q) {
      A[p][q] = first[16 * p + q];
      B[p][q] = second[16 * p + q];
    }
  mul16(B, A, C);
  for (int p = 0; p < 16; ++p)
    for (int q = 0; q < 16; ++q) ptm_out[16 * p + q] = C[p][q];
  return NZE_OK;
}

extern "C" int nze_ptm_swap_qubits(const double* ptm_in, double* ptm_out) {
  if (!ptm_in || !ptm_out) return fail(NZE_EINVAL, "null argument");
  double T[16][16];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      for (int c = 0; c < 4; ++c)
        for (int d = 0; d < 4; ++d) T[4 * a + b][4 * c + d] = ptm_in[16 * (4 * b + a) + 4 * d + c];
  for (int p = 0; p < 16; ++p)
    for (int q = 0; q < 16; ++q) ptm_out[16 * p + q] = T[p][q];
  return NZE_OK;
}

extern "C" int nze_route_chain(int32_t n, int32_t n_gates, const int32_t* qa,
                               const int32_t* qb, int32_t restore, int32_t max_ops,
                               int32_t* op_site, int32_t* op_gate, uint8_t* op_flip,
                               int32_t* n_ops, int32_t* perm_out) {
  if (n < 2 || n_gates < 0 || max_ops < 0 || !n_ops || (n_gates > 0 && (!qa || !qb)))
    return fail(NZE_EINVAL, "bad routing arguments");
  for (int g = 0; g < n_gates; ++g)
    if (qa[g] < 0 || qa[g] >= n || qb[g] < 0 || qb[g] >= n || qa[g] == qb[g])
      return fail(NZE_EINVAL, "gate qubits out of range or equal");
  const bool write = op_site && op_gate && op_flip;
  std::vector<int> pos(n), at(n);
  for (int q = 0; q < n; ++q) pos[q] = at[q] = q;
  int64_t k = 0;
  auto emit = [&](int site, int gate, int flip) {
    if (write && k < max_ops) {
      op_site[k] = site;
      op_gate[k] = gate;
      op_flip[k] = static_cast<uint8_t>(flip);
    }
    ++k;
  };
  auto exchange = [&](int s) {
    emit(s, -1, 0);
    const int x = at[s], y = at[s + 1];
    at[s] = y;
    at[s + 1] = x;
    pos[y] = s;
    pos[x] = s + 1;
  };
  std::vector<int> walked;
  for (int g = 0; g < n_gates; ++g) {
    const int a = qa[g], b = qb[g];
    // the second qubit walks towards the first, one exchange per step
    walked.clear();
    while (std::abs(pos[a] - pos[b]) > 1) {
      const int sb = pos[b];
      const int s = pos[a] > sb ? sb : sb - 1;
      exchange(s);
      walked.push_back(s);
    }
    emit(std::min(pos[a], pos[b]), g, pos[a] > pos[b] ? 1 : 0);
    // and walks back (layout unchanged) when asked to
    if (restore)
      for (int i = static_cast<int>(walked.size()) - 1; i >= 0; --i) exchange(walked[i]);
  }
  if (k > INT32_MAX) return fail(NZE_EINVAL, "routed sequence too long");
  *n_ops = static_cast<int32_t>(k);
  if (perm_out)
    for (int q = 0; q < n; ++q) perm_out[q] = pos[q];
  if (write && k > max_ops) return fail(NZE_ENOMEM, "max_ops too small for the routed sequence");
  return NZE_OK;
}

// ------------------------------------------------------------------- fits

namespace {

// Least squares min ||A x - y|| for a small dense A (n x k, row-major) by
// Householder QR.  Returns false when A is rank deficient.
bool lstsq(int n, int k, std::vector<double> A, std::vector<double> y,
           std::vector<double>& x) {
  if (n < k) return false;
  for (int j = 0; j < k; ++j) {
    double norm = 0;
    for (int i = j; i < n; ++i) norm += A[i * k + j] * A[i * k + j];
    norm = std::sqrt(norm);
    if (norm == 0) return false;
    const double alpha = A[j * k + j] > 0 ? -norm : norm;
    std::vector<double> v(n, 0.0);
    for (int i = j; i < n; ++i) v[i] = A[i * k + j];
    v[j] -= alpha;
    double vv = 0;
    for (int i = j; i < n; ++i) vv += v[i] * v[i];
    if (vv == 0) continue;
    for (int c = j; c < k; ++c) {
      double d = 0;
      for (int i = j; i < n; ++i) d += v[i] * A[i * k + c];
      d = 2 * d / vv;
      for (int i = j; i < n; ++i) A[i * k + c] -= d * v[i];
    }
    double d = 0;
    for (int i = j; i < n; ++i) d += v[i] * y[i];
    d = 2 * d / vv;
    for (int i = j; i < n; ++i) y[i] -= d * v[i];
  }
  double amax = 0;
  for (int j = 0; j < k; ++j) amax = std::fmax(amax, std::fabs(A[j * k + j]));
  x.assign(k, 0.0);
  for (int j = k - 1; j >= 0; --j) {
    if (std::fabs(A[j * k + j]) <= 1e-14 * amax) return false;
    double s = y[j];
    for (int c = j + 1; c < k; ++c) s -= A[j * k + c] * x[c];
    x[j] = s / A[j * k + j];
  }
  return true;
}

int fit_poly(int n, const double* lam, const double* y, int degree,
             double target, double* value, double* coef) {
  const int k = degree + 1;
  if (degree < 0 || n < k) return fail(NZE_EFIT, "too few points for POLY");
  std::vector<double> A(n * k), b(y, y + n), x;
  for (int i = 0; i < n; ++i) {
    double p = 1;
    for (int j = 0; j < k; ++j) { A[i * k + j] = p; p *= lam[i]; }
  }
  if (!lstsq(n, k, A, b, x)) return fail(NZE_EFIT, "degenerate lambdas");
  double v = 0, p = 1;
  for (int j = 0; j < k; ++j) { v += x[j] * p; p *= target; }
  *value = v;
  if (coef)
    for (int j = 0; j < 3; ++j) coef[j] = j < k ? x[j] : 0.0;
  return NZE_OK;
}

// For fixed b, (a, c) of a exp(-b l) + c by least squares; returns the RSS.
double exp3_profile(int n, const double* lam, const double* y, double b,
                    double* a, double* c) {
  std::vector<double> A(2 * n), yy(y, y + n), x;
  for (int i = 0; i < n; ++i) { A[2 * i] = std::exp(-b * lam[i]); A[2 * i + 1] = 1; }
  if (!lstsq(n, 2, A, yy, x)) {
    // b -> 0: the exponential column equals the constant; use the mean
    double m = 0;
    for (int i = 0; i < n; ++i) m += y[i];
    x = {0.0, m / n};
  }
  double rss = 0;
  for (int i = 0; i < n; ++i) {
    const double r = x[0] * std::exp(-b * lam[i]) + x[1] - y[i];
    rss += r * r;
  }
  if (a) *a = x[0];
  if (c) *c = x[1];
  return rss;
}

int fit_exp3(int n, const double* lam, const double* y, double target,
             double b_max, double* value, double* coef) {
  if (n < 3) return fail(NZE_EFIT, "too few points for EXP3");
  double lo = lam[0], hi = lam[0];
  for (int i = 1; i < n; ++i) { lo = std::fmin(lo, lam[i]); hi = std::fmax(hi, lam[i]); }
  if (hi - lo <= 0) return fail(NZE_EFIT, "degenerate lambdas");
  if (!(b_max > 0)) b_max = 50.0 / (hi - lo);
  // scan, then golden-section refinement, then Newton polish of the profile
  const int NG = 512;
  int best = 0;
  double fbest = 1e300;
  for (int i = 0; i <= NG; ++i) {
    const double f = exp3_profile(n, lam, y, b_max * i / NG, nullptr, nullptr);
    if (f < fbest) { fbest = f; best = i; }
  }
  double a0 = b_max * (best > 0 ? best - 1 : 0) / NG;
  double a1 = b_max * (best < NG ? best + 1 : NG) / NG;
  const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
  double x1 = a1 - gr * (a1 - a0), x2 = a0 + gr * (a1 - a0);
  double f1 = exp3_profile(n, lam, y, x1, nullptr, nullptr);
  double f2 = exp3_profile(n, lam, y, x2, nullptr, nullptr);
  for (int it = 0; it < 300 && a1 - a0 > 1e-15 * std::fmax(1.0, a1); ++it) {
    if (f1 < f2) { a1 = x2; x2 = x1; f2 = f1; x1 = a1 - gr * (a1 - a0); f1 = exp3_profile(n, lam, y, x1, nullptr, nullptr); }
    else { a0 = x1; x1 = x2; f1 = f2; x2 = a0 + gr * (a1 - a0); f2 = exp3_profile(n, lam, y, x2, nullptr, nullptr); }
  }
  double b = 0.5 * (a0 + a1);
  for (int it = 0; it < 30; ++it) {
    const double h = 1e-5 * std::fmax(1.0, std::fabs(b));
    const double fm = exp3_profile(n, lam, y, b - h, nullptr, nullptr);
    const double f0 = exp3_profile(n, lam, y, b, nullptr, nullptr);
    const double fp = exp3_profile(n, lam, y, b + h, nullptr, nullptr);
    const double d2 = (fp - 2 * f0 + fm) / (h * h);
    if (!(d2 > 0)) break;
    double nb = b - ((fp - fm) / (2 * h)) / d2;
    nb = std::fmin(std::fmax(nb, 0.0), b_max);
    if (exp3_profile(n, lam, y, nb, nullptr, nullptr) > f0) break;
    const bool done = std::fabs(nb - b) <= 1e-14 * std::fmax(1.0, std::fabs(b));
    b = nb;
    if (done) break;
  }
  double a, c;
  exp3_profile(n, lam, y, b, &a, &c);
  *value = a * std::exp(-b * target) + c;
  if (coef) { coef[0] = a; coef[1] = b; coef[2] = c; }
  return NZE_OK;
}

int fit_loglin(int n, const double* lam, const double* y, const double* fid,
               double target, const nze_fit_opts& o, double* value,
               double* coef, uint8_t* used) {
  if (!fid) return fail(NZE_EINVAL, "LOGLIN_W needs fidelities");
  int imin = 0;
  for (int i = 1; i < n; ++i) if (lam[i] < lam[imin]) imin = i;
  double sign = o.ref_sign != 0 ? (o.ref_sign > 0 ? 1.0 : -1.0)
                                : (y[imin] >= 0 ? 1.0 : -1.0);
  // dip size: smallest lambda > 0 with F > threshold, else the largest lambda
  double d = -1, lmax = lam[0];
  for (int i = 0; i < n; ++i) {
    lmax = std::fmax(lmax, lam[i]);
    if (lam[i] > 0 && fid[i] > o.dip_threshold && (d < 0 || lam[i] < d)) d = lam[i];
  }
  if (d <= 0) d = lmax;
  if (!(d > 0)) return fail(NZE_EFIT, "no positive lambda");
  std::vector<double> A, b;
  int m = 0;
  for (int i = 0; i < n; ++i) {
    const bool ok = std::fabs(y[i]) >= o.small &&      // criterion 2
                    (y[i] > 0 ? 1.0 : -1.0) == sign;   // criterion 3
    if (used) used[i] = ok ? 1 : 0;
    if (!ok) continue;
    const double w = std::pow(fid[i], o.delta_f) *
                     std::exp(-o.delta_d * std::fabs(target - lam[i]) / d);
    A.push_back(w);
    A.push_back(-w * lam[i]);
    b.push_back(w * std::log(std::fabs(y[i])));
    ++m;
  }
  if (m < 2) return fail(NZE_EFIT, "fewer than two points pass criteria 2-3");
  std::vector<double> x;
  if (!lstsq(m, 2, A, b, x)) return fail(NZE_EFIT, "degenerate log-linear fit");
  const double a = sign * std::exp(x[0]);
  *value = a * std::exp(-x[1] * target);
  if (coef) { coef[0] = a; coef[1] = x[1]; coef[2] = 0.0; }
  return NZE_OK;
}

}  // namespace

extern "C" void nze_fit_opts_default(nze_fit_opts* o) {
  if (!o) return;
  o->degree = 2;
  o->delta_f = 2.0;
  o->delta_d = 20.0;
  o->small = 1e-10;
  o->dip_threshold = 0.99;
  o->ref_sign = 0;
  o->b_max = 0.0;
}

extern "C" int nze_extrapolate(int32_t n_pts, const double* lambda,
                               const double* value, const double* fidelity,
                               double lambda_target, int32_t method,
                               const nze_fit_opts* opts, double* out_value,
                               double* out_coef, uint8_t* used_mask,
                               int32_t* method_used) {
  if (n_pts <= 0 || !lambda || !value || !out_value)
    return fail(NZE_EINVAL, "bad arguments");
  nze_fit_opts o;
  nze_fit_opts_default(&o);
  if (opts) o = *opts;
  for (int i = 0; i < n_pts; ++i)
    if (!std::isfinite(lambda[i]) || !std::isfinite(value[i]))
      return fail(NZE_EINVAL, "non-finite input");
  auto all_used = [&](uint8_t v) {
    if (used_mask) for (int i = 0; i < n_pts; ++i) used_mask[i] = v;
  };
  int rc;
  if (method == NZE_POLY) {
    rc = fit_poly(n_pts, lambda, value, o.degree, lambda_target, out_value, out_coef);
    all_used(rc == NZE_OK);
    if (method_used) *method_used = NZE_POLY;
    return rc;
  }
  if (method == NZE_LOGLIN_W) {
    rc = fit_loglin(n_pts, lambda, value, fidelity, lambda_target, o, out_value,
                    out_coef, used_mask);
    if (rc == NZE_OK) {
      if (method_used) *method_used = NZE_LOGLIN_W;
      return rc;
    }
    if (rc != NZE_EFIT) return rc;
    // fall back to the direct exponential fit on every point (criteria 2-3
    // dropped); criterion 1 is the caller's selection of points
  } else if (method != NZE_EXP3) {
    return fail(NZE_EINVAL, "unknown method");
  }
  rc = fit_exp3(n_pts, lambda, value, lambda_target, o.b_max, out_value, out_coef);
  all_used(rc == NZE_OK);
  if (method_used) *method_used = rc == NZE_OK ? NZE_EXP3 : -1;
  return rc;
}

extern "C" int nze_fidelity_extrapolate(int32_t n_pts, const double* value,
                                        const double* fidelity,
                                        double* out_value, int32_t* converged) {
  if (n_pts < 2 || !value || !fidelity || !out_value)
    return fail(NZE_EINVAL, "need at least two runs");
  std::vector<double> A(2 * n_pts), y(value, value + n_pts), x;
  for (int i = 0; i < n_pts; ++i) { A[2 * i] = 1; A[2 * i + 1] = fidelity[i]; }
  if (!lstsq(n_pts, 2, A, y, x)) return fail(NZE_EFIT, "equal fidelities");
  *out_value = x[0] + x[1];
  if (converged) {
    const double o1 = value[n_pts - 2], o2 = value[n_pts - 1];
    const double f1 = fidelity[n_pts - 2], f2 = fidelity[n_pts - 1];
    const double slope = std::fabs((o2 - o1) / (f2 - f1));
    *converged = slope * (1.0 - f2) < std::fabs(o2) / 2.0 ? 1 : 0;
  }
  return NZE_OK;
}

extern "C" const char* nze_strerror(int code) {
  switch (code) {
    case NZE_OK: return "ok";
    case NZE_EINVAL: return "invalid argument";
    case NZE_ENOMEM: return "workspace too small";
    case NZE_EHIP: return "HIP runtime error";
    case NZE_ENOCONV: return "Jacobi SVD did not converge within the sweep cap";
    case NZE_EFIT: return "too few admissible points for extrapolation";
    case NZE_ENUM: return "NaN or Inf in the state";
    default: return "unknown error";
  }
}

extern "C" const char* nze_last_error(void) { return nze::g_last_error.c_str(); }

extern "C" const char* nze_version(void) { return "nze-mi355x 0.1 (gfx950)"; }
