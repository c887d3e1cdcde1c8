// The phases of one two-site update and of one centre move, as device
// functions executed by the G workgroups serving one MPO (local index g).
//
// Update of the gate on (k, k+1) (Sec. 2.1.2 "Approximate emulation"):
//   theta   Theta' = (R x 1)(M_k M_{k+1}) written as the row-major matrix X
//           in the orientation whose rows carry the factor that stays
//           orthonormal (rows (q',b) left to right, (a,p') right to left),
//           with a copy of it in W                               [MFMA]
//   jacobi  block one-sided Jacobi on the rows of X (no accumulator):
//           afterwards X has orthogonal rows s_i (singular vector)^T
//                                                                 [MFMA + LDS]
//   norms   squared row norms in float64
//   select  sort, truncation rank r (tie rule), kept-row order  [one WG]
//   refine  float64: the kept rows divided by their norms, orthonormalised
//           (Newton-Schulz), give the orthonormal factor Q; the other factor
//           is the projection Y = Q X0^T of the unrotated block; a
//           Rayleigh-Ritz polish of the directions around a chi cut; partial
//           fidelity f = kept / total, emulation fidelity *= f, log-scale;
//           the two new sites from Q and Y / ||kept||
// Centre move (the canonical form of App. A.1's footnote): the same Jacobi on
// the centre site viewed as (chi_r x 4 chi_l) (left to right) or
// (chi_l x 4 chi_r) (right to left), then the orthonormal factor from the
// kept rows (float64, as above) stays and the projection of the site onto it
// is multiplied into the neighbour in float64.
#ifndef NZE_PHASES_H
#define NZE_PHASES_H

#include "nze_device.h"

namespace nze {

// ---------------------------------------------------------------- helpers

template <typename T>
__device__ inline T* site_ptr(const Slot& s, int k) {
  return reinterpret_cast<T*>(s.sites) + (size_t)k * s.site_cap;
}

// W = I (n x n), distributed by rows.
template <typename T>
__device__ __forceinline__ void set_identity(T* W, int n, int g, int G) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int r = g * 4 + w; r < n; r += 4 * G)
    for (int c = lane; c < n; c += 64) W[(size_t)r * n + c] = T(r == c ? 1 : 0);
}

// ------------------------------------------------------------ theta phase

// X <- (R x 1)(M_k M_{k+1}); also W = I (init_w), or a second copy of the
// block in X2 (the float64 refinement's unrotated block).
template <typename T>
__device__ __forceinline__ void phase_theta(const Slot& s, int k, bool ltr, const double* R,
                            int g, int G, double* smem, bool count = true,
                            bool init_w = true, T* X2 = nullptr) {
  typedef typename AccT<T>::type acc_t;
  const int cl = s.dims[k], cm = s.dims[k + 1], cr = s.dims[k + 2];
  const T* A = site_ptr<T>(s, k);          // (4 cl) x cm
  const T* B = site_ptr<T>(s, k + 1);      // cm x (4 cr)
  T* X = reinterpret_cast<T*>(s.X);
  const int ldb = 4 * cr;
  const int ldx = ltr ? 4 * cr : 4 * cl;
  T* tile = reinterpret_cast<T*>(smem);                          // [64][65]
  double* Rs = smem + (64 * 65 * sizeof(T) + 7) / 8;              // [256]
  const int tid = threadIdx.x;
  Rs[tid] = R[tid];
  const int lane = tid & 63, w = tid >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const int ta = (cl + 15) / 16, tb = (cr + 15) / 16;
  for (int t = g; t < ta * tb; t += G) {
    const int a0 = (t / tb) * 16, b0 = (t % tb) * 16;
    const int row = a0 * 4 + 16 * w + i;
    const bool rok = row < 4 * cl;
    const bool cok = b0 + i < cr;
    acc_t acc[4];
    for (int q = 0; q < 4; ++q) acc[q] = acc_t{0, 0, 0, 0};
    for (int c0 = 0; c0 < cm; c0 += 4) {
      const int c = c0 + kq;
      const bool kok = c < cm;
      const T av = (rok && kok) ? A[(size_t)row * cm + c] : T(0);
      for (int q = 0; q < 4; ++q) {
        const T bv = (kok && cok) ? B[(size_t)c * ldb + q * cr + b0 + i] : T(0);
        acc[q] = mfma4(av, bv, acc[q]);
      }
    }
    __syncthreads();
    for (int q = 0; q < 4; ++q)
      for (int r = 0; r < 4; ++r)
        tile[(16 * w + mrow<T>(kq, r)) * 65 + 16 * q + i] = acc[q][r];
    __syncthreads();
    int al, bl;
    if (ltr) { bl = tid & 15; al = tid >> 4; } else { al = tid & 15; bl = tid >> 4; }
    if (a0 + al < cl && b0 + bl < cr) {
      T th[16];
      for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 4; ++q) th[4 * p + q] = tile[(al * 4 + p) * 65 + q * 16 + bl];
      const int a = a0 + al, b = b0 + bl;
      for (int q2 = 0; q2 < 4; ++q2)
        for (int p2 = 0; p2 < 4; ++p2) {
          const int P = 4 * p2 + q2;
          T o = T(0);
          for (int Q = 0; Q < 16; ++Q) o += T(Rs[P * 16 + Q]) * th[Q];
          const size_t e = ltr ? (size_t)(a * 4 + p2) * ldx + q2 * cr + b
                               : (size_t)(q2 * cr + b) * ldx + a * 4 + p2;
          X[e] = o;
          if (X2) X2[e] = o;
        }
    }
  }
  if (count && g == 0 && tid == 0)   // contraction 2 (4cl) cm (4cr) + superoperator 512 cl cr
    s.scal[SC_FLOPS] += 32.0 * cl * cm * cr + 512.0 * cl * cr;
  if (init_w) set_identity(reinterpret_cast<T*>(s.W), ltr ? 4 * cl : 4 * cr, g, G);
}

// --------------------------------------------------------- Jacobi phase

// Relative off-diagonal threshold of the Jacobi convergence test on rows of
// length C.  Float64: at least 8 sqrt(C) eps, the worst-case rounding of a
// length-C dot product.  Float32 rows: at least eps itself.  Rounding of the
// float32 rows and of the MFMA Gram leaves a relative coupling of about
// eps / sqrt(C) between orthogonal rows, far below the worst-case bound, and a
// threshold at that bound (8 sqrt(C) eps = 7.6e-6 at C = 256) leaves exactly
// the near-degenerate pairs around a truncation cut unrotated: their mixing
// angle tol / (2 relative gap) then decides which directions are kept.
template <typename T>
__device__ inline double jacobi_threshold(const Slot& s, int C) {
  if (sizeof(T) == 4) return fmax(s.tol_rel, 5.96e-8);
  return fmax(s.tol_rel, 8.0 * sqrt((double)C) * 1.11e-16);
}

// LDS layout of one pair step
struct PairLds {
  double* Gp;     // [4][1024] per-wave partial Grams; during the inner solve
                  // the second Gram buffer
  double* Gs;     // [32][GLD]
  double* Qs;     // [32][GLD]
  int* rows;      // [32] global row of each pair row (-1 = none)
  int* flag;      // [2]
};

__device__ inline PairLds pair_lds(double* smem) {
  PairLds L;
  L.Gp = smem;
  L.Gs = L.Gp + 4 * 1024;
  L.Qs = L.Gs + 32 * GLD;
  int* ib = reinterpret_cast<int*>(L.Qs + 32 * GLD);
  L.rows = ib;
  L.flag = ib + 32;
  return L;
}

// Gs = X_rows X_rows^T (32 x 32) in float64 from MFMA partials.  X holds R
// rows of length C (leading dimension ld).  Each wave takes 64-column chunks
// 256 apart; the loads of the next chunk are issued before the MFMAs of the
// current one (branch-free buffer loads, zeros outside the rows and columns).
// VEC = 0 (the kernel built for two workgroups per CU, which hides latency
// with the other workgroup and has half the registers): one register set.
// r0, r1: rows i = lane mod 16 of the two blocks (-1: none).
template <typename T, int VEC = 1>
__device__ __forceinline__ void pair_gram(const T* X, int ld, int C, int R, const PairLds& L,
                                          int r0, int r1) {
  typedef typename AccT<T>::type acc_t;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const rsrc_t rs = make_rsrc(X, (size_t)R * ld * sizeof(T));
  const uint32_t base0 = r0 >= 0 ? uint32_t(r0) * uint32_t(ld) * uint32_t(sizeof(T)) : OOB;
  const uint32_t base1 = r1 >= 0 ? uint32_t(r1) * uint32_t(ld) * uint32_t(sizeof(T)) : OOB;
  // MFMA partial sums over 64 columns, accumulated in float64 across chunks
  double g00[4] = {0, 0, 0, 0}, g01[4] = {0, 0, 0, 0}, g11[4] = {0, 0, 0, 0};
  T xa0[4][4], xa1[4][4], xb0[4][4], xb1[4][4];
  auto fetch = [&](int c0, T (&x0)[4][4], T (&x1)[4][4]) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int c = c0 + 64 * h + 4 * kq;   // C is a multiple of 4
      const uint32_t cb = uint32_t(c) * uint32_t(sizeof(T));
      bload4(rs, (c < C && base0 != OOB) ? base0 + cb : OOB, x0[h]);
      bload4(rs, (c < C && base1 != OOB) ? base1 + cb : OOB, x1[h]);
    }
  };
  auto accum = [&](const T (&x0)[4][4], const T (&x1)[4][4]) {
    acc_t a00 = {0, 0, 0, 0}, a01 = {0, 0, 0, 0}, a11 = {0, 0, 0, 0};
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        a00 = mfma4(x0[h][s], x0[h][s], a00);
        a01 = mfma4(x0[h][s], x1[h][s], a01);
        a11 = mfma4(x1[h][s], x1[h][s], a11);
      }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      g00[r] += double(a00[r]);
      g01[r] += double(a01[r]);
      g11[r] += double(a11[r]);
    }
  };
  int c0 = 16 * w;
  if constexpr (VEC == 0) {
    for (; c0 < C; c0 += 256) {
      fetch(c0, xa0, xa1);
      accum(xa0, xa1);
    }
  } else if (C == 1024 || C == 2048) {
    // the saturated shapes (chi 256 / 512): every wave takes exactly 4 / 8
    // chunks, fully unrolled, so that the compiler waits for the loads of
    // the chunk it multiplies only (in a loop it waits for all of them)
    auto run = [&](auto nch) {
      constexpr int NCH = decltype(nch)::value;
      fetch(c0, xa0, xa1);
#pragma unroll
      for (int k = 0; k < NCH; ++k) {
        if (k % 2 == 0) {
          if (k + 1 < NCH) fetch(c0 + 256 * (k + 1), xb0, xb1);
          __builtin_amdgcn_sched_barrier(0);
          accum(xa0, xa1);
        } else {
          if (k + 1 < NCH) fetch(c0 + 256 * (k + 1), xa0, xa1);
          __builtin_amdgcn_sched_barrier(0);
          accum(xb0, xb1);
        }
      }
    };
    if (C == 1024) run(std::integral_constant<int, 4>());
    else run(std::integral_constant<int, 8>());
  } else if (c0 < C) {
    // two register sets in turn: chunk k + 1 loads while chunk k multiplies
    // (the scheduling barriers keep the compiler from sinking the loads of
    // the next chunk down to their uses)
    fetch(c0, xa0, xa1);
    while (true) {
      fetch(c0 + 256, xb0, xb1);
      __builtin_amdgcn_sched_barrier(0);
      accum(xa0, xa1);
      c0 += 256;
      if (c0 >= C) break;
      fetch(c0 + 256, xa0, xa1);
      __builtin_amdgcn_sched_barrier(0);
      accum(xb0, xb1);
      c0 += 256;
      if (c0 >= C) break;
    }
  }
  double* P = L.Gp + w * 1024;
  for (int r = 0; r < 4; ++r) {
    const int u = mrow<T>(kq, r);
    P[u * 32 + i] = g00[r];
    P[u * 32 + 16 + i] = g01[r];
    P[(16 + u) * 32 + 16 + i] = g11[r];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 1024; e += NT) {
    const int u = e >> 5, v = e & 31;
    if (u >= 16 && v < 16) continue;
    const double val = L.Gp[e] + L.Gp[1024 + e] + L.Gp[2048 + e] + L.Gp[3072 + e];
    L.Gs[u * GLD + v] = val;
    if (u < 16 && v >= 16) L.Gs[v * GLD + u] = val;
  }
  __syncthreads();
}

// Reciprocal square root: hardware seed (v_rsq_f64) refined by two
// Newton-Raphson steps y_{k+1} = y_k (3 - a y_k^2) / 2, each of which squares
// the relative error.
__device__ inline double nr_rsq(double a) {
  double y = __builtin_amdgcn_rsq(a);
  y = y * fma(-0.5 * a * y, y, 1.5);
  y = y * fma(-0.5 * a * y, y, 1.5);
  return y;
}

// Jacobi rotation (c, s) that zeroes g_pq of the symmetric 2x2 block
// [[g_pp, g_pq], [g_pq, g_qq]] (J = [[c, s], [-s, c]], J^T G J diagonal):
// tau = (g_qq - g_pp) / (2 g_pq), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
// c = 1 / sqrt(1 + t^2), s = t c.  Identity below the threshold.
// t only sets how much of g_pq the rotation removes: the unrefined hardware
// reciprocal and root (about 1e-7 relative) leave ~1e-7 g_pq for the next
// visit.  c must make (c, t c) orthonormal to rounding, so its root is
// refined.
__device__ inline void jacobi_cs(double gpp, double gqq, double gpq,
                                 double floor_abs, double& c, double& sn) {
  const bool ra = fabs(gpq) > floor_abs && gpq * gpq > 1e-30 * fabs(gpp * gqq);
  const double ta = (gqq - gpp) * __builtin_amdgcn_rcp(2.0 * (ra ? gpq : 1.0));
  const double ua = fma(ta, ta, 1.0);
  const double xa = (ta >= 0 ? 1.0 : -1.0) *
                    __builtin_amdgcn_rcp(fabs(ta) + ua * __builtin_amdgcn_rsq(ua));
  const double ca = nr_rsq(fma(xa, xa, 1.0));
  c = ra ? ca : 1.0;
  sn = ra ? xa * ca : 0.0;
}

// v moved down by one lane inside each row of 16 lanes: lane l takes the
// value of lane 16 (l / 16) + (l + 1) % 16 (DPP row rotate right by 15).
__device__ __forceinline__ double row_next(double v) { return dpp_f64<0x12F>(v); }

// One cyclic parallel Jacobi sweep on the 32x32 symmetric Gram in Ga
// (float64, LDS), cross-block steps first (both blocks enter with nearly
// orthogonal rows once a sweep has visited them, so the cross entries carry
// most of the off-diagonal weight); Qs accumulates the rotations.  Thread t
// owns the 2x2 block (pair t/16, pair t%16) of G and rows 2(t/16),
// 2(t/16)+1 of Qs at pair t%16.  Lane l of a wave computes the rotation of
// pair l & 15 (its column pair) from the step's pivots; the rotation of its
// row pair P = t/16 = 4 w + l/16 comes from lane P of the same wave, which
// computed it as its own column pair from the same values with the same
// instructions.  G ping-pongs between Ga and Gb (swapped on return, Ga holds
// the result): one workgroup barrier a step.  In the cross-block steps the
// block-I row and column of a thread's pairs stay P and P2, and the block-J
// column moves from pair P2 + 1 to pair P2: the thread keeps its two rows of
// Qs at its columns, and its entries G[P][P2] and G[P][J], in registers,
// taking the block-J ones from the next lane of its 16-lane row (row_next);
// only the block-J rows of G pass through LDS, plus the entries that are
// the next step's pivots (G[P][P] and G[P][J] of pair P + 1), and all of G
// and Qs after the last of these steps.  With cross_only the sweep stops
// after the 16 cross-block steps.  Pivots with |g_pq| <= floor_abs are
// not rotated.  q_identity: Qs starts as the identity (taken in registers;
// Qs in LDS need not be filled), else from the Qs in LDS.
// skip_tol > 0: after the cross-block steps, the intra-block steps run only
// if some intra-block entry fails the visit's convergence test
// (|g_uv| > skip_tol (sqrt(g_uu g_vv) + ratio_abs sqrt(F2 max(g_uu, g_vv))));
// entries that pass it are left to later visits, and the sweeps still end
// only when every pair of every visit passes the test.
__device__ __forceinline__ void gram_sweep32(const PairLds& L, double*& Ga, double*& Gb,
                                             double floor_abs, bool cross_only,
                                             double skip_tol = 0.0, double ratio_abs = 0.0,
                                             double F2 = 0.0, bool q_identity = false) {
  const int tid = threadIdx.x;
  if (tid == 0) L.flag[0] = 0;   // ordered by the barrier of the first step
  const int P = tid >> 4, P2 = tid & 15, u0 = 2 * P;
  const int srcP = P & 15;
  auto step = [&](int p, int q, int p2, int q2) {
    const double bpp = Ga[p2 * GLD + p2], bqq = Ga[q2 * GLD + q2], bpq = Ga[p2 * GLD + q2];
    const double g11 = Ga[p * GLD + p2], g12 = Ga[p * GLD + q2];
    const double g21 = Ga[q * GLD + p2], g22 = Ga[q * GLD + q2];
    const double qa = L.Qs[u0 * GLD + p2], qb = L.Qs[u0 * GLD + q2];
    const double qc = L.Qs[(u0 + 1) * GLD + p2], qd = L.Qs[(u0 + 1) * GLD + q2];
    double c2, s2;
    jacobi_cs(bpp, bqq, bpq, floor_abs, c2, s2);
    const double c = __shfl(c2, srcP, 64), sn = __shfl(s2, srcP, 64);
    const double h11 = c * g11 - sn * g21, h12 = c * g12 - sn * g22;
    const double h21 = sn * g11 + c * g21, h22 = sn * g12 + c * g22;
    Gb[p * GLD + p2] = c2 * h11 - s2 * h12;
    Gb[p * GLD + q2] = s2 * h11 + c2 * h12;
    Gb[q * GLD + p2] = c2 * h21 - s2 * h22;
    Gb[q * GLD + q2] = s2 * h21 + c2 * h22;
    L.Qs[u0 * GLD + p2] = c2 * qa - s2 * qb;
    L.Qs[u0 * GLD + q2] = s2 * qa + c2 * qb;
    L.Qs[(u0 + 1) * GLD + p2] = c2 * qc - s2 * qd;
    L.Qs[(u0 + 1) * GLD + q2] = s2 * qc + c2 * qd;
    double* t = Ga; Ga = Gb; Gb = t;
    __syncthreads();
  };
  // pairing of the 32 rows (rows 0-15: block I, 16-31: block J), 16
  // disjoint rotations a step: steps 0-15 pair row k of I with row
  // 16 + (k + st) mod 16 of J (all 256 cross pairs) ...  (the arithmetic of
  // step(), with the entries that stay on a thread in registers)
  {
    double qa, qb, qc, qd;
    if (q_identity) {
      qa = u0 == P2 ? 1.0 : 0.0; qb = u0 == 16 + P2 ? 1.0 : 0.0;
      qc = u0 + 1 == P2 ? 1.0 : 0.0; qd = u0 + 1 == 16 + P2 ? 1.0 : 0.0;
    } else {
      qa = L.Qs[u0 * GLD + P2]; qb = L.Qs[u0 * GLD + 16 + P2];
      qc = L.Qs[(u0 + 1) * GLD + P2]; qd = L.Qs[(u0 + 1) * GLD + 16 + P2];
    }
    double g11 = Ga[P * GLD + P2], g12 = Ga[P * GLD + 16 + P2];
    const bool piv11 = P == P2, piv12 = P2 == ((P + 1) & 15);
    for (int st = 0; st < 16; ++st) {
      const int p = P, q = 16 + ((P + st) & 15), p2 = P2, q2 = 16 + ((P2 + st) & 15);
      const double bpp = Ga[p2 * GLD + p2], bqq = Ga[q2 * GLD + q2], bpq = Ga[p2 * GLD + q2];
      const double g21 = Ga[q * GLD + p2], g22 = Ga[q * GLD + q2];
      double c2, s2;
      jacobi_cs(bpp, bqq, bpq, floor_abs, c2, s2);
      const double c = __shfl(c2, srcP, 64), sn = __shfl(s2, srcP, 64);
      const double h11 = c * g11 - sn * g21, h12 = c * g12 - sn * g22;
      const double h21 = sn * g11 + c * g21, h22 = sn * g12 + c * g22;
      const double n11 = c2 * h11 - s2 * h12, n12 = s2 * h11 + c2 * h12;
      Gb[q * GLD + p2] = c2 * h21 - s2 * h22;
      Gb[q * GLD + q2] = s2 * h21 + c2 * h22;
      if (st == 15 || piv11) Gb[p * GLD + p2] = n11;
      if (st == 15 || piv12) Gb[p * GLD + q2] = n12;
      const double na = c2 * qa - s2 * qb, nb = s2 * qa + c2 * qb;
      const double nc = c2 * qc - s2 * qd, nd = s2 * qc + c2 * qd;
      qa = na; qc = nc; g11 = n11;
      if (st < 15) {
        qb = row_next(nb); qd = row_next(nd); g12 = row_next(n12);
      } else {
        const int jc = 16 + ((P2 + 15) & 15);
        L.Qs[u0 * GLD + P2] = na; L.Qs[u0 * GLD + jc] = nb;
        L.Qs[(u0 + 1) * GLD + P2] = nc; L.Qs[(u0 + 1) * GLD + jc] = nd;
      }
      double* t = Ga; Ga = Gb; Gb = t;
      __syncthreads();
    }
  }
  if (cross_only) return;
  if (skip_tol > 0.0) {
    // thread t: entry (t / 16, t % 16) of each block's 16 x 16 corner
    const int u = tid >> 4, v = tid & 15;
    float worst = 0.f;
    if (v > u) {
      for (int b = 0; b < 32; b += 16) {
        const double guu = Ga[(b + u) * GLD + b + u], gvv = Ga[(b + v) * GLD + b + v];
        const double guv = fabs(Ga[(b + u) * GLD + b + v]);
        const double den = __builtin_amdgcn_sqrt(guu * gvv) +
                           ratio_abs * __builtin_amdgcn_sqrt(F2 * fmax(guu, gvv));
        const double q = den > 0.0 ? guv * __builtin_amdgcn_rcp(den) : (guv > 0.0 ? 1.0 : 0.0);
        worst = fmaxf(worst, (q == q) ? float(q) : 1.0f);
      }
    }
    worst = wave_max(worst);
    if ((tid & 63) == 0 && worst > float(skip_tol)) L.flag[0] = 1;
    __syncthreads();
    const int need = L.flag[0];   // rewritten only after later barriers
    if (!need) return;
  }
  {
    // ... steps 16-30 a round-robin tournament inside each block (pairs
    // 0-7 in I, 8-15 in J; all 2 x 120 intra pairs): pair k = base + j
    // (base 0 or 16) takes rows base + (j == 0 ? 0 : 1 + (j - 1 + r) mod 15)
    // and base + 1 + (14 - j + r) mod 15 at r = st - 16, stepped here
    // incrementally
    const int bP = P < 8 ? 0 : 16, jP = P & 7, bQ = P2 < 8 ? 0 : 16, jQ = P2 & 7;
    int aP = jP == 0 ? 0 : jP - 1, cP = 14 - jP, aQ = jQ == 0 ? 0 : jQ - 1, cQ = 14 - jQ;
    for (int r = 0; r < 15; ++r) {
      step(bP + (jP == 0 ? 0 : 1 + aP), bP + 1 + cP, bQ + (jQ == 0 ? 0 : 1 + aQ), bQ + 1 + cQ);
      aP = aP == 14 ? 0 : aP + 1;
      cP = cP == 14 ? 0 : cP + 1;
      aQ = aQ == 14 ? 0 : aQ + 1;
      cQ = cQ == 14 ? 0 : cQ + 1;
    }
  }
}

// The pair solve: one sweep of gram_sweep32 on the pair's Gram in Gs, from
// Qs = I, its intra-block steps skipped when those entries already pass the
// visit's convergence test (skip_tol = the test's threshold).  Returns the
// buffer that holds the rotated Gram Q^T G Q.
// The Gram is complete and Gp free after the barriers of pair_gram and the
// convergence test; Qs starts as the identity inside gram_sweep32.
__device__ const double* inner_eigh(const PairLds& L, bool cross_only, double skip_tol,
                                   double ratio_abs, double F2) {
  const int lane = threadIdx.x & 63;
  const double dmax = wave_max(lane < 32 ? L.Gs[lane * GLD + lane] : 0.0);
  const double floor_abs = 1e-30 * dmax;
  double* Ga = L.Gs;
  double* Gb = L.Gp;          // 32 x GLD, free once the Gram is reduced
  gram_sweep32(L, Ga, Gb, floor_abs, cross_only, skip_tol, ratio_abs, F2, true);
  return Ga;   // the rotated Gram Q^T G Q
}

// rows <- Q^T rows for the pair's 32 rows of M (nrows rows, leading
// dimension ld, ncols columns), in place.
template <typename T, int VEC = 1>
__device__ __forceinline__ void pair_rotate(T* M, int ld, int ncols, int nrows, const PairLds& L) {
  typedef typename AccT<T>::type acc_t;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  T qa[2][8];
  for (int h = 0; h < 2; ++h)
    for (int s = 0; s < 8; ++s) qa[h][s] = T(L.Qs[(4 * s + kq) * GLD + 16 * h + i]);
  int src[8];
  for (int s = 0; s < 8; ++s) src[s] = L.rows[4 * s + kq];
  int dst0[4], dst1[4];
  for (int r = 0; r < 4; ++r) { dst0[r] = L.rows[mrow<T>(kq, r)]; dst1[r] = L.rows[16 + mrow<T>(kq, r)]; }
  if (VEC && (ld & 3) == 0 && (ncols & 3) == 0 && (reinterpret_cast<uintptr_t>(M) & 15) == 0) {
    // vector path: lane (i, kq) loads four consecutive columns c0 + 4i .. +3
    // of row 4s + kq; MFMA j takes column c0 + 4i + j, and each output row's
    // four columns leave as one vector store.  Branch-free buffer accesses
    // (rows past the pair and columns past the end read zeros and drop
    // their stores); the loads of the next 64-column chunk are issued
    // before the MFMAs of the current one.
    const rsrc_t rs = make_rsrc(M, (size_t)nrows * ld * sizeof(T));
    const uint32_t rowb = uint32_t(ld) * uint32_t(sizeof(T));
    uint32_t sb[8], db0[4], db1[4];
#pragma unroll
    for (int s = 0; s < 8; ++s) sb[s] = src[s] >= 0 ? uint32_t(src[s]) * rowb : OOB;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      db0[r] = dst0[r] >= 0 ? uint32_t(dst0[r]) * rowb : OOB;
      db1[r] = dst1[r] >= 0 ? uint32_t(dst1[r]) * rowb : OOB;
    }
    T xa[8][4], xb[8][4];
    auto fetch = [&](int c0, T (&x)[8][4]) {
      const int c = c0 + 4 * i;
      const uint32_t cb = uint32_t(c) * uint32_t(sizeof(T));
#pragma unroll
      for (int s = 0; s < 8; ++s) bload4(rs, (c < ncols && sb[s] != OOB) ? sb[s] + cb : OOB, x[s]);
    };
    auto rotate = [&](int c0, const T (&x)[8][4]) {
      const int c = c0 + 4 * i;
      const bool cok = c < ncols;
      // two column pairs at a time (fewer live accumulators)
#pragma unroll
      for (int jh = 0; jh < 4; jh += 2) {
        acc_t d0a = {0, 0, 0, 0}, d0b = {0, 0, 0, 0}, d1a = {0, 0, 0, 0}, d1b = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          d0a = mfma4(qa[0][s], x[s][jh], d0a);
          d0b = mfma4(qa[0][s], x[s][jh + 1], d0b);
          d1a = mfma4(qa[1][s], x[s][jh], d1a);
          d1b = mfma4(qa[1][s], x[s][jh + 1], d1b);
        }
        const uint32_t cb = uint32_t(c + jh) * uint32_t(sizeof(T));
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          bstore2(rs, (cok && db0[r] != OOB) ? db0[r] + cb : OOB, T(d0a[r]), T(d0b[r]));
          bstore2(rs, (cok && db1[r] != OOB) ? db1[r] + cb : OOB, T(d1a[r]), T(d1b[r]));
        }
      }
    };
    int c0 = 64 * w;
    if constexpr (sizeof(T) == 8) {
      // float64 rows: one register set (two do not fit without spilling)
      for (; c0 < ncols; c0 += 256) {
        fetch(c0, xa);
        rotate(c0, xa);
      }
    } else if (ncols == 1024 || ncols == 2048) {
      // the saturated shapes: every wave takes exactly 4 / 8 chunks, fully
      // unrolled so that the compiler waits for the current chunk only
      auto run = [&](auto nch) {
        constexpr int NCH = decltype(nch)::value;
        fetch(c0, xa);
#pragma unroll
        for (int k = 0; k < NCH; ++k) {
          if (k % 2 == 0) {
            if (k + 1 < NCH) fetch(c0 + 256 * (k + 1), xb);
            __builtin_amdgcn_sched_barrier(0);
            rotate(c0 + 256 * k, xa);
          } else {
            if (k + 1 < NCH) fetch(c0 + 256 * (k + 1), xa);
            __builtin_amdgcn_sched_barrier(0);
            rotate(c0 + 256 * k, xb);
          }
        }
      };
      if (ncols == 1024) run(std::integral_constant<int, 4>());
      else run(std::integral_constant<int, 8>());
    } else if (c0 < ncols) {
      fetch(c0, xa);
      while (true) {
        fetch(c0 + 256, xb);
        __builtin_amdgcn_sched_barrier(0);
        rotate(c0, xa);
        c0 += 256;
        if (c0 >= ncols) break;
        fetch(c0 + 256, xa);
        __builtin_amdgcn_sched_barrier(0);
        rotate(c0, xb);
        c0 += 256;
        if (c0 >= ncols) break;
      }
    }
    return;
  }
  constexpr int NCH = 4;   // 16-column chunks in flight per wave
  for (int c0 = 16 * w; c0 < ncols; c0 += 64 * NCH) {
    T xb[NCH][8];
#pragma unroll
    for (int h = 0; h < NCH; ++h) {
      const int c = c0 + 64 * h + i;
      const bool cok = c < ncols;
#pragma unroll
      for (int s = 0; s < 8; ++s)
        xb[h][s] = (cok && src[s] >= 0) ? load1(M + (size_t)src[s] * ld + c) : T(0);
    }
#pragma unroll
    for (int h = 0; h < NCH; ++h) {
      const int c = c0 + 64 * h + i;
      acc_t d0 = {0, 0, 0, 0}, d1 = {0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        d0 = mfma4(qa[0][s], xb[h][s], d0);
        d1 = mfma4(qa[1][s], xb[h][s], d1);
      }
      if (c < ncols) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (dst0[r] >= 0) store1(M + (size_t)dst0[r] * ld + c, T(d0[r]));
          if (dst1[r] >= 0) store1(M + (size_t)dst1[r] * ld + c, T(d1[r]));
        }
      }
    }
  }
}

// Global row of pair row tid (< 32) of the visit of blocks I, J: rows are
// numbered in the sweep's order (fixed for the sweep), -1 past the end:
// r0 = row (lane mod 16) of block I, r1 = the same row of block J.
__device__ inline void pair_rows(const int* order, int I, int J, int nb, int R, int& r0,
                                 int& r1) {
  const int i = threadIdx.x & 15;
  const int a = I * BW + i, b = J * BW + i;
  r0 = (I < nb && a < R) ? load1(order + a) : -1;
  r1 = (J < nb && b < R) ? load1(order + b) : -1;
}

// One pair step of sweep `sw`: Gram, convergence test, inner solve, rotate.
// r0, r1: pair_rows of this thread, loaded before the wait for the blocks
// (which ends with workgroup barriers, so the LDS of the previous visit is
// free here).
template <typename T, int VEC = 1>
__device__ __forceinline__ bool jacobi_pair(const Slot& s, T* X, T* W, int R, int C, int I,
                            int J, int nb, int sw, double F2, double* smem,
                            bool timed, Group& grp,
                            int* verX, int* verW, int target, bool last_round,
                            bool cross_only, bool forced, int r0, int r1) {
  const PairLds L = pair_lds(smem);
  const int tid = threadIdx.x;
  PhaseClock clk(timed && s.prof != nullptr);
  // read after the barriers of pair_gram
  if (tid < 32) L.rows[tid] = tid < 16 ? r0 : r1;
  if (tid == 0) L.flag[1] = 0;
  pair_gram<T, VEC>(X, C, C, R, L, r0, r1);
  clk.lap(s.prof, PF_GRAM);
  int go = 1;
  const double tol = jacobi_threshold<T>(s, C);
  const double ratio_abs = s.tol_abs / tol;
  if (!forced) {
    // convergence test: |g_uv| > tol sqrt(g_uu g_vv) + tol_abs sqrt(F2 max)
    float worst = 0.f;   // largest |g_uv| / (sqrt(g_uu g_vv) + ratio_abs sqrt(F2 max))
    for (int e = tid; e < 1024; e += NT) {
      const int u = e >> 5, v = e & 31;
      if (v <= u) continue;
      const double guu = L.Gs[u * GLD + u], gvv = L.Gs[v * GLD + v];
      const double guv = fabs(L.Gs[u * GLD + v]);
      // a tolerance test: hardware root and reciprocal (~1e-7 relative) suffice
      const double den = __builtin_amdgcn_sqrt(guu * gvv) +
                         ratio_abs * __builtin_amdgcn_sqrt(F2 * fmax(guu, gvv));
      const double q = den > 0.0 ? guv * __builtin_amdgcn_rcp(den) : (guv > 0.0 ? 1.0 : 0.0);
      worst = fmaxf(worst, (q == q) ? float(q) : 1.0f);
    }
    worst = wave_max(worst);
    const int need = worst > float(tol);
    if ((tid & 63) == 0 && worst > 0.f)
      atomicMax(&s.ctr[CT_OFFMAX], __float_as_int(worst));
    if (need) L.flag[1] = 1;
    __syncthreads();
    go = L.flag[1];   // rewritten only after later barriers
  }
  clk.lap(s.prof, PF_CHECK);
  const double* Gfin = L.Gs;
  if (go) {
    if (tid == 0) atomicAdd(&s.ctr[CT_ROT + sw], 1);
    Gfin = inner_eigh(L, cross_only, tol, ratio_abs, F2);
    clk.lap(s.prof, PF_EIGH);
    if (clk.on && tid == 0) s.prof[PF_PAIRS] += 1.0;
    pair_rotate<T, VEC>(X, C, C, R, L);
    clk.lap(s.prof, PF_ROTX);
  }
  // the last round visits every block once: the diagonal of the pair's Gram
  // after the visit (Q^T G Q when it rotated) gives the squared row norms
  // that order the next sweep, without a pass over X
  if (last_round && tid < 32 && L.rows[tid] >= 0) store1(s.norms + L.rows[tid], Gfin[tid * GLD + tid]);
  blocks_release(grp, verX, I, J);
  if (s.no_acc) return true;
  // accumulator rows: previous visits of both blocks first, in visit order
  if (!blocks_wait(grp, verW, I, J, target)) return false;
  if (go) pair_rotate<T, VEC>(W, R, R, R, L);
  blocks_release(grp, verW, I, J);
  clk.lap(s.prof, PF_ROTW);
  return true;
}

// squared row norms in float64
template <typename T>
__device__ __forceinline__ void phase_norms(const Slot& s, const T* X, int R, int C, int g,
                            int G) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int r = g * 4 + w; r < R; r += 4 * G) {
    double acc = 0.0;
    const T* x = X + (size_t)r * C;
    for (int c = lane; c < C; c += 64) {
      const double v = double(load1(x + c));
      acc += v * v;
    }
    acc = wave_sum(acc);
    if (lane == 0) s.norms[r] = acc;
  }
}

// One workgroup: s.perm[0..R) = rows ordered by decreasing squared norm
// (ties by index).  Bitonic sort of (key, index) pairs in LDS.
__device__ __forceinline__ void sort_rows(const Slot& s, int R, double* key, int* idx) {
  int N = 1;
  while (N < R) N <<= 1;
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NT) {
    key[i] = i < R ? s.norms[i] : -1.0;
    idx[i] = i;
  }
  __syncthreads();
  for (int size = 2; size <= N; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < N; i += NT) {
        const int j = i ^ stride;
        if (j > i) {
          const bool desc = (i & size) == 0;
          const double ki = key[i], kj = key[j];
          const int ii = idx[i], ij = idx[j];
          const bool i_first = ki > kj || (ki == kj && ii < ij);
          if (desc ? !i_first : i_first) {
            key[i] = kj; key[j] = ki; idx[i] = ij; idx[j] = ii;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Round-robin tournament: block at position `pos` in round t (nbe even).
__device__ inline int tourney_block(int pos, int t, int nbe) {
  return pos == 0 ? 0 : 1 + ((pos - 1 + t) % (nbe - 1));
}

template <typename T, int VEC = 1>
__device__ __forceinline__ bool phase_jacobi(const Slot& s, T* X, T* W, int R, int C, int g,
                             int G, Group& grp, double* smem) {
  const int nb = (R + BW - 1) / BW;
  const int nbe = nb + (nb & 1);
  const int rounds = nbe - 1, npair = nbe / 2;
  int* ver = s.ctr + CT_BVER;
  int* wver = s.ctr + CT_WVER;
  int sweeps = 0;
  bool conv = false;
  for (int sw = 0; sw < s.max_sweeps && sw < MAXSW; ++sw) {
    PhaseClock sclk(g == 0 && s.prof != nullptr);
    // blocks are consecutive runs of the rows sorted by decreasing norm; the
    // norms come from a pass over X before the first sweep and from the last
    // round's visits afterwards
    if (sw == 0) {
      phase_norms<T>(s, X, R, C, g, G);
      if (!group_sync(grp)) return false;
    }
    if (g == 0) {
      double* key = smem;
      int* idx = reinterpret_cast<int*>(smem + 4 * CHI_LIMIT);
      // ||X||_F^2 in a fixed summation order (the absolute convergence floor)
      double f2 = 0.0;
      for (int i = threadIdx.x; i < R; i += NT) f2 += s.norms[i];
      f2 = block_sum(f2, smem + 6 * CHI_LIMIT);
      sort_rows(s, R, key, idx);
      for (int i = threadIdx.x; i < R; i += NT) s.perm[i] = idx[i];
      if (threadIdx.x == 0) {
        s.scal[SC_F2] = f2;
        if (sw == 0) s.scal[SC_TOT] = f2;
        s.ctr[CT_OFFMAX] = 0;
      }
      if (sw == 0)
        for (int b = threadIdx.x; b < nbe; b += NT) { ver[b] = 0; wver[b] = 0; }
    }
    if (!group_sync(grp)) return false;
    sclk.lap(s.prof, PF_SWEEP);
    const double F2 = __hip_atomic_load(&s.scal[SC_F2], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
    // early sweeps of a large problem (cross_min_blocks blocks or more; 64
    // by default, the first cross_sweeps = 8 sweeps), while every pair still
    // rotated in the sweep before: the inner solves take only their 256
    // cross-block rotations.  Far from convergence the outer sweeps, not the
    // pair solves, set the pace, and the rows are re-blocked by norm at every
    // sweep, so pairs left inside a block meet as cross pairs later; every
    // later sweep runs full inner sweeps, which polish all pairs.
    bool cross_only = false;
    if (nb >= s.cross_min_blocks && sw < s.cross_sweeps)
      cross_only = sw == 0 ||
                   __hip_atomic_load(&s.ctr[CT_ROT + sw - 1], __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT) == rounds * npair;
    // after the first sweep such a sweep rotates every pair without the
    // convergence test (the sweep before rotated every pair; the later full
    // sweeps test and polish all of them)
    // (never the last sweep the cap allows: that one measures the largest
    // off-diagonal that decides between a benign cap and ERR_NOCONV)
    const bool forced = cross_only && sw > 0 && sw + 1 < s.max_sweeps;
    // visit v = t npair + q (pair q of round t) belongs to workgroup v mod G;
    // each workgroup takes its visits in increasing order, and a visit waits
    // only for the previous round's visits of its two blocks, so rounds
    // overlap when G exceeds the pairs per round
    const int base = sw * rounds;
    for (int v = g; v < rounds * npair; v += G) {
      const int t = v / npair, q = v - t * npair;
      {
        const int I = tourney_block(q, t, nbe);
        const int J = tourney_block(nbe - 1 - q, t, nbe);
        // the row order is fixed for the sweep: its load overlaps the wait
        int r0, r1;
        pair_rows(s.perm, I, J, nb, R, r0, r1);
        PhaseClock wclk(s.prof != nullptr);
        if (!blocks_wait(grp, ver, I, J, base + t)) return false;
        if (wclk.on) {
          const uint64_t now = wall_clock64();
          if (threadIdx.x == 0) {
            if (g == 0) s.prof[PF_WAIT] += double(now - wclk.t);
            atomicAdd(&s.prof[PF_WAIT_ALL], double(now - wclk.t) / G);
          }
        }
        if (!jacobi_pair<T, VEC>(s, X, W, R, C, I, J, nb, sw, F2, smem, g == 0, grp, ver, wver, base + t, t == rounds - 1, cross_only, forced,
                            r0, r1))
          return false;
      }
    }
    // every visit of the sweep is complete before the norms are taken
    sclk.t = sclk.on ? wall_clock64() : 0;
    if (!group_sync(grp)) return false;
    sclk.lap(s.prof, PF_SWEEP);
    sweeps = sw + 1;
    const int rot = __hip_atomic_load(&s.ctr[CT_ROT + sw], __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
    if (rot == 0) { conv = true; break; }
  }
  if (g == 0 && threadIdx.x == 0) {
    s.scal[SC_FLOPS] += 4.0 * sweeps * double(R) * double(R) * (2.0 * C + (s.no_acc ? 0.0 : R));
    s.ctr[CT_SWTOT] += sweeps;
    if (sweeps > s.ctr[CT_MAXSW]) s.ctr[CT_MAXSW] = sweeps;
    if (!conv) {
      // the cap was reached: fine at the rounding floor, an error beyond it
      const double tol = jacobi_threshold<T>(s, C);
      const float worst = __int_as_float(s.ctr[CT_OFFMAX]);
      s.scal[SC_CAPQ] = fmax(s.scal[SC_CAPQ], double(worst) / tol);
      if (double(worst) > 1e3 * tol) s.ctr[CT_ERR] |= ERR_NOCONV;
      else s.ctr[CT_CAPHIT] += 1;
    }
  }
  return true;
}

// One workgroup: sort the squared norms, pick the rank, update fidelity and
// log-scale.  gate: truncation rule with chi cap and tie rule; otherwise
// (centre move) only numerical zeros (s_i <= tau s_1) are dropped.
__device__ __forceinline__ void phase_select(const Slot& s, int R, bool gate, double* smem,
                             bool defer = false) {
  int N = 1;
  while (N < R) N <<= 1;
  double* key = smem;
  int* idx = reinterpret_cast<int*>(smem + N);
  double* red = smem + N + (N + 1) / 2 + 2;
  int* sh = reinterpret_cast<int*>(red + 8);
  const int tid = threadIdx.x;
  sort_rows(s, R, key, idx);
  double tot = 0.0;
  for (int i = tid; i < R; i += NT) tot += fmax(key[i], 0.0);
  tot = block_sum(tot, red);
  const double s1 = sqrt(fmax(key[0], 0.0));
  int above = 0;
  for (int i = tid; i < R; i += NT) above += (sqrt(fmax(key[i], 0.0)) > s.tau * s1) ? 1 : 0;
  above = (int)block_sum((double)above, red);
  if (tid == 0) {
    int r;
    if (!(s1 > 0.0)) {
      r = 1;
    } else if (gate) {
      r = above < s.chi ? above : s.chi;
      if (r < 1) r = 1;
      if (r == s.chi && r < above) {
        const int r0 = r;
        while (r > 0) {
          const double a = sqrt(fmax(key[r - 1], 0.0)), b = sqrt(fmax(key[r], 0.0));
          if (a - b <= s.tie * a) --r; else break;
        }
        if (r == 0) r = r0;
      }
    } else {
      r = above < 1 ? 1 : above;
    }
    sh[0] = r;
  }
  __syncthreads();
  const int r = sh[0];
  double kept = 0.0;
  for (int i = tid; i < r; i += NT) {
    kept += fmax(key[i], 0.0);
    s.sval[i] = sqrt(fmax(key[i], 0.0));
  }
  for (int i = tid; i < R; i += NT) s.perm[i] = idx[i];   // the whole order
  kept = block_sum(kept, red);
  if (tid == 0) {
    s.ctr[CT_RANK] = r;
    s.scal[SC_KEPT] = kept;
    s.scal[SC_ABOVE] = above;
    if (!(tot == tot) || tot > 1e300 || !(kept > 0.0)) s.ctr[CT_ERR] |= ERR_NAN;
    if (gate) {
      // with defer the refinement books the partial fidelity of the block it
      // builds (refine_gate)
      if (!defer) {
        const double f = kept / tot;
        s.scal[SC_FID] *= f;
        s.scal[SC_LOG] += 0.5 * log(kept);
        s.scal[SC_MAXDISC] = fmax(s.scal[SC_MAXDISC], 1.0 - f);
      }
      if (r < R && key[r] > 0.0) {
        const double gap = (sqrt(key[r - 1]) - sqrt(key[r])) / s1;
        s.scal[SC_MINGAP] = fmin(s.scal[SC_MINGAP], gap);
      }
      s.ctr[CT_UPD] += 1;
    }
    s.scal[SC_F2] = 0.0;
  }
  for (int i = tid; i < MAXSW; i += NT) s.ctr[CT_ROT + i] = 0;
}

// ------------------------------------------------ float64 refinement
//
// The Jacobi keeps no accumulator: its rotated rows are s_i times a singular
// vector plus rounding of order eps ||X|| (eps of the row precision), so the
// direction of a row with a small s_i carries a relative error of order
// eps s_1 / s_i.  The refinement keeps the Jacobi's decisions (rank, kept
// rows) and rebuilds the two factors in float64: the kept rows divided by
// their norms, orthonormalised by Newton-Schulz iterations
// Q <- (3 I - Q Q^T) Q / 2, give the orthonormal factor, and the other factor
// is the projection of the unrotated block onto it (no division by singular
// values).  The product of the two factors is then the orthogonal projection
// of the block onto the kept span: a direction error theta_ij between kept
// row i and dropped direction j changes the state by theta_ij s_j <= eps s_1
// (s_j <= s_i), and the partial fidelity kept / total is exactly that
// projection's (Sec. 2.1.2, eq. for f_l).

// C (M x N, float64, row-major ldc) = A op(B) over the group's workgroups on
// 64 x 64 tiles with float64 MFMA: A is M x K (row-major lda), B is K x N
// (row-major ldb) or, with TB_T, N x K (row-major ldb) used transposed.
// K advances 16 at a time: lane (i, q) reads k = k0 + 4q .. 4q + 3 of its A
// row as one vector, and MFMA step u takes k = k0 + 4q + u on both operands
// (any assignment of the four k of a step to q is a valid 16x16x4 product).
template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef nze_v4f type; };
template <> struct Vec4<double> { typedef double type __attribute__((ext_vector_type(4))); };

template <typename T>
__device__ inline void load4_or0(const T* p, bool ok_all, int nvalid, double v[4]) {
  if (ok_all && (reinterpret_cast<uintptr_t>(p) & (4 * sizeof(T) - 1)) == 0) {
    const typename Vec4<T>::type x = *(__attribute__((address_space(1))) const typename Vec4<T>::type*)p;
    v[0] = double(x[0]); v[1] = double(x[1]); v[2] = double(x[2]); v[3] = double(x[3]);
  } else {
    for (int u = 0; u < 4; ++u) v[u] = u < nvalid ? double(load1(p + u)) : 0.0;
  }
}

template <typename TA, typename TB, bool TB_T>
__device__ __forceinline__ void gemm64(const TA* A, int lda, const TB* B, int ldb, double* C, int ldc,
                       int M, int N, int K, int g, int G) {
  typedef typename AccT<double>::type acc_t;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  const int tm = (M + 63) / 64, tn = (N + 63) / 64;
  for (int tile = g; tile < tm * tn; tile += G) {
    const int m0 = (tile / tn) * 64, n0 = (tile % tn) * 64;
    const int row = m0 + 16 * w + i;
    acc_t acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = acc_t{0, 0, 0, 0};
    for (int k0 = 0; k0 < K; k0 += 16) {
      const int kb = k0 + 4 * q;                       // this lane's four k
      const int nv = K - kb;                           // valid among them
      double av[4];
      load4_or0(A + (size_t)(row < M ? row : 0) * lda + kb, row < M && nv >= 4, row < M ? nv : 0, av);
      double bv[4][4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = n0 + 16 * j + i;
        if (TB_T) {
          load4_or0(B + (size_t)(col < N ? col : 0) * ldb + kb, col < N && nv >= 4, col < N ? nv : 0, bv[j]);
        } else {
#pragma unroll
          for (int u = 0; u < 4; ++u)
            bv[j][u] = (col < N && u < nv) ? double(load1(B + (size_t)(kb + u) * ldb + col)) : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = mfma4(av[u], bv[j][u], acc[j]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = m0 + 16 * w + mrow<double>(q, r), cc = n0 + 16 * j + i;
        if (rr < M && cc < N) C[(size_t)rr * ldc + cc] = acc[j][r];
      }
  }
}

// dst[i][c] = T(src[i][c] * scale), i < r, c < n
template <typename T>
__device__ __forceinline__ void copy_r64(const double* src, int lds, int r, int n, T* dst, int ldd,
                         double scale, int g, int G) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = g * 4 + w; i < r; i += 4 * G)
    for (int c = lane; c < n; c += 64) dst[(size_t)i * ldd + c] = T(src[(size_t)i * lds + c] * scale);
}

// dst[a][i] = T(src[i][a] * scale), i < r, a < n (LDS transpose)
template <typename T>
__device__ __forceinline__ void copy_t64(const double* src, int lds, int r, int n, T* dst, int ldd,
                         double scale, int g, int G, double* smem) {
  double* tile = smem;   // [32][33]
  const int ta = (n + 31) / 32, ti = (r + 31) / 32;
  for (int t = g; t < ta * ti; t += G) {
    const int a0 = (t / ti) * 32, i0 = (t % ti) * 32;
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += NT) {
      const int ii = e >> 5, al = e & 31;
      tile[ii * 33 + al] = (i0 + ii < r && a0 + al < n) ? src[(size_t)(i0 + ii) * lds + a0 + al] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += NT) {
      const int al = e >> 5, ii = e & 31;
      if (i0 + ii < r && a0 + al < n)
        dst[(size_t)(a0 + al) * ldd + i0 + ii] = T(tile[ii * 33 + al] * scale);
    }
  }
  __syncthreads();
}

// Newton-Schulz iteration Q <- (3 I - Q Q^T) Q / 2 on the r rows of Q
// (r x n, float64), ping-ponging between Q0 and Q1 with B (r x r) as scratch.
// It converges to the orthonormal polar factor when every singular value of
// Q lies in (0, sqrt 3); the Gershgorin bound e = max_i sum_j |(Q Q^T - I)_ij|
// of the start, reduced over the group into ctr[CT_NSMAX] (a maximum, so the
// order of the atomics does not matter), places them in
// (sqrt(max(0, 1 - e)), sqrt(1 + e)).  For e < 0.9 the number of steps
// follows from e (each step takes an error e to about 3 e^2 / 4: 1e-5 needs
// one step, 1e-3 two, 2e-2 three, 0.15 four, 0.9 six).  Otherwise the rows
// are first scaled by 1 / sqrt(1 + e), which puts every singular value below
// one, and fourteen steps are taken (a value 0.1 reaches one in eight);
// ctr[CT_NSFB] counts those cases.  Returns the buffer holding the result, or
// nullptr when a barrier failed.
__device__ inline double* ns_rows(double* Q0, double* Q1, int n, int r, double* B,
                                  const Slot& s, int g, int G, Group& grp) {
  double* cur = Q0;
  double* nxt = Q1;
  if (g == 0 && threadIdx.x == 0) s.ctr[CT_NSMAX] = 0;
  if (!group_sync(grp)) return nullptr;
  gemm64<double, double, true>(cur, n, cur, n, B, r, r, r, n, g, G);
  if (!group_sync(grp)) return nullptr;
  float emax = 0.f;
  for (int i = g * NT + threadIdx.x; i < r; i += G * NT) {
    double rs = 0.0;
    for (int j = 0; j < r; ++j) rs += fabs(B[(size_t)i * r + j] - (i == j ? 1.0 : 0.0));
    emax = fmaxf(emax, (rs == rs) ? float(rs) : 1e30f);
  }
  for (int o = 32; o > 0; o >>= 1) emax = fmaxf(emax, __shfl_xor(emax, o, 64));
  if ((threadIdx.x & 63) == 0 && emax > 0.f) atomicMax(&s.ctr[CT_NSMAX], __float_as_int(emax));
  if (!group_sync(grp)) return nullptr;
  const float e0 = __int_as_float(__hip_atomic_load(&s.ctr[CT_NSMAX], __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT));
  int steps;
  bool regram = false;
  if (e0 < 0.9f) {
    steps = e0 <= 1e-13f ? 0 : e0 <= 1e-5f ? 1 : e0 <= 1e-3f ? 2 : e0 <= 2e-2f ? 3
          : e0 <= 0.15f ? 4 : 6;
  } else {
    // scaled start: Q <- Q / sqrt(1 + e)
    const double sc = 1.0 / sqrt(1.0 + (e0 < 1e30f ? double(e0) : 1e30));
    for (size_t e = (size_t)g * NT + threadIdx.x; e < (size_t)r * n; e += (size_t)G * NT)
      cur[e] *= sc;
    if (g == 0 && threadIdx.x == 0) s.ctr[CT_NSFB] += 1;
    steps = 14;
    regram = true;
    if (!group_sync(grp)) return nullptr;
  }
  for (int st = 0; st < steps; ++st) {
    if (st > 0 || regram) {
      gemm64<double, double, true>(cur, n, cur, n, B, r, r, r, n, g, G);
      if (!group_sync(grp)) return nullptr;
    }
    for (int e = g * NT + threadIdx.x; e < r * r; e += G * NT) {
      const int i = e / r, j = e - i * r;
      B[e] = (i == j ? 1.5 : 0.0) - 0.5 * B[e];
    }
    if (!group_sync(grp)) return nullptr;
    gemm64<double, double, false>(B, r, cur, n, nxt, n, r, n, r, g, G);
    if (!group_sync(grp)) return nullptr;
    double* t = cur; cur = nxt; nxt = t;
  }
  return cur;
}

// squared norms of the r rows of A (r x n, float64) into s.norms, one wave
// per row (a fixed summation order)
__device__ inline void rows_norm64(const Slot& s, const double* A, int r, int n, int g, int G) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = g * 4 + w; i < r; i += 4 * G) {
    double acc = 0.0;
    for (int c = lane; c < n; c += 64) {
      const double v = A[(size_t)i * n + c];
      acc += v * v;
    }
    acc = wave_sum(acc);
    if (lane == 0) s.norms[i] = acc;
  }
}

constexpr int BAND = 16;   // kept and dropped directions polished at a cut

// Refinement workspace of a slot: two (chi + BAND) x m_cap row buffers around
// a square one of max((chi + BAND)^2, 32 x 32) doubles.
__device__ inline size_t r64_rows(const Slot& s) { return (size_t)s.chi + BAND; }
__device__ inline size_t r64_square(const Slot& s) {
  const size_t c = r64_rows(s);
  return c * c > 1088 ? c * c : 1088;   // the band's 32 x 32 vectors + 32 values
}

// One workgroup: the eigenvectors of the symmetric nb x nb (nb <= 32) float64
// Gram in L.Gs by cyclic Jacobi sweeps (the pairing of the pair solves) until
// every |g_uv| <= 1e-15 sqrt(g_uu g_vv), at most twelve sweeps; rows and
// columns nb..31 are inert padding.  On return Vout (32 x 32, row u column a)
// holds the eigenvector of column a in row u, columns in decreasing order of
// their eigenvalue, and EVout[a] that eigenvalue.
__device__ __forceinline__ void band_eigh(const PairLds& L, int nb, double* Vout, double* EVout) {
  const int tid = threadIdx.x;
  for (int e = tid; e < 32 * 32; e += NT) {
    const int u = e >> 5, v = e & 31;
    L.Qs[u * GLD + v] = (u == v) ? 1.0 : 0.0;
    if (u >= nb || v >= nb) L.Gs[u * GLD + v] = (u == v) ? -1.0 - u : 0.0;
  }
  __syncthreads();
  double* Ga = L.Gs;
  double* Gb = L.Gp;
  double* red = L.Gp + 2048;
  for (int sweep = 0; sweep < 12; ++sweep) {
    // convergence on the entries of the current Gram
    double worst = 0.0;
    for (int e = tid; e < 1024; e += NT) {
      const int u = e >> 5, v = e & 31;
      if (u < v && v < nb) {
        const double d = fabs(Ga[u * GLD + v]) / sqrt(fabs(Ga[u * GLD + u] * Ga[v * GLD + v]) + 1e-300);
        worst = fmax(worst, d);
      }
    }
    worst = wave_max(worst);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = worst;
    __syncthreads();
    worst = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    if (worst <= 1e-15) break;
    gram_sweep32(L, Ga, Gb, 0.0, false);
  }
  // columns in decreasing eigenvalue order (selection by rank; ties by index)
  if (tid < 32) {
    const double ev = Ga[tid * GLD + tid];
    int rank = 0;
    for (int b = 0; b < 32; ++b) {
      const double eb = Ga[b * GLD + b];
      rank += (eb > ev || (eb == ev && b < tid)) ? 1 : 0;
    }
    for (int u = 0; u < 32; ++u) Vout[u * 32 + rank] = L.Qs[u * GLD + tid];
    EVout[rank] = ev;
  }
  __syncthreads();
}

// rows [b0, b0 + nb) of M (ld columns n, float64) <- V^T rows: row a of the
// band becomes sum_u V[u][a] row_u (V from band_eigh, 32 x 32).  Column
// chunks of 64 are staged through LDS (32 x 65 doubles), so the rotation
// needs no per-thread arrays.
__device__ inline void band_rotate(double* M, int ld, int n, int b0, int nb, const double* V,
                                   int g, int G, double* smem) {
  double* tile = smem;   // [32][65]
  for (int c0 = g * 64; c0 < n; c0 += G * 64) {
    __syncthreads();
    for (int e = threadIdx.x; e < 32 * 64; e += NT) {
      const int u = e >> 6, cl = e & 63;
      tile[u * 65 + cl] = (u < nb && c0 + cl < n) ? M[(size_t)(b0 + u) * ld + c0 + cl] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 32 * 64; e += NT) {
      const int a = e >> 6, cl = e & 63;
      if (a >= nb || c0 + cl >= n) continue;
      double acc = 0.0;
      for (int u = 0; u < nb; ++u) acc = fma(V[u * 32 + a], tile[u * 65 + cl], acc);
      M[(size_t)(b0 + a) * ld + c0 + cl] = acc;
    }
  }
  __syncthreads();
}

// Gate update after phase_select(defer), from the rows of the Jacobi
// alone.  The Jacobi ran on the block oriented so that its rows carry
// the factor that stays orthonormal: left to right the rows of Theta'^T
// (indexed (q', b)), whose rotated rows are s_i u_i^T; right to left the rows
// of Theta' (indexed (a, p')), whose rotated rows are s_i v_i^T.  The kept
// rows divided by their norms, orthonormalised in float64 (ns_rows), give
// Q = U_r^T (resp. V_r^T); the other factor is the float64 projection of the
// unrotated block X0 (the copy the contraction left in W), Y = Q X0^T.  A
// float64 Rayleigh-Ritz polish of the BAND
// kept and BAND dropped directions around a chi cut resolves the mixing the
// Jacobi leaves between near-degenerate directions there (about
// tol / (2 relative gap)), and the tie rule is re-decided on its values.
// Returns 1 when done, 0 on a barrier failure.
template <typename T>
__device__ __forceinline__ int refine_gate(const Slot& s, int k, bool ltr, int Rr, int Cc,
                                           int g, int G, Group& grp, double* smem) {
  const int r = s.ctr[CT_RANK];
  // the band: only at a cut set by chi, and only over dropped directions
  // within three decades of the last kept one
  const int above = (int)s.scal[SC_ABOVE];
  int hi = 0;
  if (r == s.chi && r < above) {
    const double s_last = sqrt(fmax(s.norms[s.perm[r - 1]], 0.0));
    while (hi < BAND && r + hi < Rr &&
           sqrt(fmax(s.norms[s.perm[r + hi]], 0.0)) >= 1e-3 * s_last) ++hi;
  }
  const int lo = hi > 0 ? (r < BAND ? r : BAND) : 0;
  const int rr = r + hi;
  double* A = s.R64;                                  // rr x max(Rr, Cc)
  double* B = A + r64_rows(s) * s.m_cap;              // rr x rr, or the band's 32 x 32
  double* C = B + r64_square(s);                      // rr x max(Rr, Cc)
  const T* X = reinterpret_cast<const T*>(s.X);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = g * 4 + w; i < rr; i += 4 * G) {
    const int row = s.perm[i];
    const double nr = sqrt(fmax(s.norms[row], 0.0));
    const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
    const T* src = X + (size_t)row * Cc;
    for (int c = lane; c < Cc; c += 64) A[(size_t)i * Cc + c] = double(load1(src + c)) * inv;
  }
  double* Q = ns_rows(A, C, Cc, rr, B, s, g, G, grp);
  if (!Q) return 0;
  double* Y = Q == A ? C : A;
  // the unrotated block X0, in the Jacobi's orientation: the copy that the
  // contraction left in W
  const T* X0 = reinterpret_cast<const T*>(s.W);
  gemm64<double, T, true>(Q, Cc, X0, Cc, Y, Rr, rr, Rr, Cc, g, G);   // Y = Q X0^T
  if (!group_sync(grp)) return 0;
  const int nb = lo + hi, b0 = r - lo;
  if (hi > 0 && lo > 0) {
    double* V = B;                                    // 32 x 32
    // the band's Gram (rows b0 .. b0 + nb - 1 of Y; zero past nb): on FP64
    // MFMA in the FP64 path; in the mixed path by the dot products and wave
    // sums it has always used, whose summation order its validated results
    // depend on (a float64 rounding change there moves later float32 Jacobi
    // roundings, and the n=50 job's error by up to 20 %), spread over every
    // wave of the group and gathered in V (band_eigh overwrites V only after
    // reading the Gram from LDS)
    if constexpr (sizeof(T) == 4) {
      for (int uv = g * 4 + w; uv < nb * nb; uv += 4 * G) {
        const int u = uv / nb, v = uv - u * nb;
        if (v < u) continue;
        double acc = 0.0;
        const double* yu = Y + (size_t)(b0 + u) * Rr;
        const double* yv = Y + (size_t)(b0 + v) * Rr;
        for (int c = lane; c < Rr; c += 64) acc = fma(yu[c], yv[c], acc);
        acc = wave_sum(acc);
        if (lane == 0) { V[u * 32 + v] = acc; V[v * 32 + u] = acc; }
      }
      if (!group_sync(grp)) return 0;
    }
    if (g == 0) {
      const PairLds L = pair_lds(smem);
      if constexpr (sizeof(T) == 8) {
        const int i16 = lane & 15;
        pair_gram<double, 0>(Y, Rr, Rr, rr, L, i16 < nb ? b0 + i16 : -1,
                             16 + i16 < nb ? b0 + 16 + i16 : -1);
      } else {
        for (int e = threadIdx.x; e < 32 * 32; e += NT) {
          const int u = e >> 5, v = e & 31;
          L.Gs[u * GLD + v] = (u < nb && v < nb) ? V[u * 32 + v] : 0.0;
        }
        __syncthreads();
      }
      double* EV = V + 1024;
      band_eigh(L, nb, V, EV);
      // the truncation rule again where float64 values decide it: the tie
      // rule (drop the chained cluster whose neighbours agree within
      // tie_tol) runs on the band's values; float32 norms carry relative
      // errors of eps s_1 / s_r, as large as tie_tol at the cut
      if (threadIdx.x == 0) {
        const int r0 = above < s.chi ? above : s.chi;
        int rn = r;
        if (r0 > b0 && r0 < b0 + nb) {
          int q = r0;
          while (q > b0) {
            const double a = sqrt(fmax(EV[q - 1 - b0], 0.0)), bq = sqrt(fmax(EV[q - b0], 0.0));
            if (a - bq <= s.tie * a) --q; else break;
          }
          if (q > b0) rn = q;            // resolved inside the band
          if (q == 0) rn = r0;           // the whole spectrum tied: keep chi
        }
        s.ctr[CT_RANK] = rn;
      }
    }
    if (!group_sync(grp)) return 0;
    band_rotate(Q, Cc, Cc, b0, nb, V, g, G, smem);
    band_rotate(Y, Rr, Rr, b0, nb, V, g, G, smem);
    if (!group_sync(grp)) return 0;
  }
  const int rk = s.ctr[CT_RANK];
  rows_norm64(s, Y, rk, Rr, g, G);
  if (!group_sync(grp)) return 0;
  if (g == 0) {
    double* red = smem;
    double kept = 0.0;
    for (int i = threadIdx.x; i < rk; i += NT) kept += s.norms[i];
    kept = block_sum(kept, red);
    if (threadIdx.x == 0) {
      const double tot = s.scal[SC_TOT];
      const double f = kept / tot;
      if (!(kept > 0.0) || !(tot > 0.0) || !(f == f)) s.ctr[CT_ERR] |= ERR_NAN;
      s.scal[SC_KEPT] = kept;
      s.scal[SC_FID] *= f;
      s.scal[SC_LOG] += 0.5 * log(kept);
      s.scal[SC_MAXDISC] = fmax(s.scal[SC_MAXDISC], 1.0 - f);
    }
  }
  if (!group_sync(grp)) return 0;
  const double inv = 1.0 / sqrt(s.scal[SC_KEPT]);
  T* Mk = site_ptr<T>(s, k);
  T* Mk1 = site_ptr<T>(s, k + 1);
  if (ltr) {   // Q rows in (a, p'): M_k = Q^T (4cl x r), M_{k+1} = Y / ||.|| (r x 4cr)
    copy_t64<T>(Q, Cc, rk, Cc, Mk, rk, 1.0, g, G, smem);
    copy_r64<T>(Y, Rr, rk, Rr, Mk1, Rr, inv, g, G);
  } else {     // Q rows in (q', b): M_k = Y^T / ||.|| (4cl x r), M_{k+1} = Q (r x 4cr)
    copy_t64<T>(Y, Rr, rk, Rr, Mk, rk, inv, g, G, smem);
    copy_r64<T>(Q, Cc, rk, Cc, Mk1, Cc, 1.0, g, G);
  }
  return group_sync(grp) ? 1 : 0;
}

// Centre move after phase_select: the orthonormal factor from the kept data
// rows divided by their norms, orthonormalised in float64, and the other
// factor as the projection of the site onto it, absorbed into the neighbour
// in float64.  The projection keeps the state whatever rotation the
// iteration applies inside the kept span, so the move stays exact up to the
// dropped numerical zeros.  Returns 1 when done, 0 on a barrier failure.
template <typename T>
__device__ __forceinline__ int refine_move(const Slot& s, int c, bool ltr, int Rr, int Cc, int g, int G,
                           Group& grp, double* smem) {
  const int r = s.ctr[CT_RANK];
  double* A = s.R64;                                  // r x Cc
  double* B = A + r64_rows(s) * s.m_cap;              // r x r
  double* C = B + r64_square(s);                      // r x Cc
  const T* X = reinterpret_cast<const T*>(s.X);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = g * 4 + w; i < r; i += 4 * G) {
    const T* src = X + (size_t)s.perm[i] * Cc;
    const double inv = 1.0 / s.sval[i];
    for (int cc = lane; cc < Cc; cc += 64) A[(size_t)i * Cc + cc] = double(load1(src + cc)) * inv;
  }
  double* Q = ns_rows(A, C, Cc, r, B, s, g, G, grp);
  if (!Q) return 0;
  double* P = Q == A ? C : A;                         // second factor / product
  T* M = site_ptr<T>(s, c);
  const int cl = s.dims[c], cr = s.dims[c + 1];
  if (ltr) {
    // M (4cl x cr) = Q^T R with R = Q M (r x cr) in B; R absorbed into site c+1
    gemm64<double, T, false>(Q, Cc, M, cr, B, cr, r, cr, 4 * cl, g, G);
    if (!group_sync(grp)) return 0;
    copy_t64<T>(Q, Cc, r, Cc, M, r, 1.0, g, G, smem);
    const int c2 = s.dims[c + 2];
    T* Mn = site_ptr<T>(s, c + 1);                     // cr x 4c2
    gemm64<double, T, false>(B, cr, Mn, 4 * c2, P, 4 * c2, r, 4 * c2, cr, g, G);
    if (g == 0 && threadIdx.x == 0) s.scal[SC_FLOPS] += 8.0 * r * cr * c2;
    if (!group_sync(grp)) return 0;
    copy_r64<T>(P, 4 * c2, r, 4 * c2, Mn, 4 * c2, 1.0, g, G);
    if (!group_sync(grp)) return 0;
    if (g == 0 && threadIdx.x == 0) s.dims[c + 1] = r;
  } else {
    // M (cl x 4cr) = L Q with L = M Q^T (cl x r) in B; L absorbed into site c-1
    gemm64<T, double, true>(M, Cc, Q, Cc, B, r, cl, r, Cc, g, G);
    if (!group_sync(grp)) return 0;
    copy_r64<T>(Q, Cc, r, Cc, M, Cc, 1.0, g, G);
    const int c0 = s.dims[c - 1];
    T* Mp = site_ptr<T>(s, c - 1);                     // 4c0 x cl
    gemm64<T, double, false>(Mp, cl, B, r, P, r, 4 * c0, r, cl, g, G);
    if (g == 0 && threadIdx.x == 0) s.scal[SC_FLOPS] += 8.0 * c0 * cl * r;
    if (!group_sync(grp)) return 0;
    copy_r64<T>(P, r, 4 * c0, r, Mp, r, 1.0, g, G);
    if (!group_sync(grp)) return 0;
    if (g == 0 && threadIdx.x == 0) s.dims[c] = r;
  }
  return group_sync(grp) ? 1 : 0;
}

// ----------------------------------------------------------- full ops

template <typename T, int VEC = 1>
__device__ __forceinline__ bool op_gate(const Slot& s, int k, bool ltr, const double* R, int g,
                        int G, Group& grp, double* smem) {
  const int cl = s.dims[k], cr = s.dims[k + 2];
  // the Jacobi keeps no accumulator and runs on the orientation whose rows
  // carry the factor that stays orthonormal (rows (q', b) left to right,
  // (a, p') right to left); refine_gate builds both factors in float64
  const bool rows_ap = !ltr;
  const int Rr = rows_ap ? 4 * cl : 4 * cr, Cc = rows_ap ? 4 * cr : 4 * cl;
  T* X = reinterpret_cast<T*>(s.X);
  T* W = reinterpret_cast<T*>(s.W);
  PhaseClock clk(g == 0 && s.prof != nullptr);
  // the contraction keeps a copy of the unrotated block in W for the
  // refinement's projection
  phase_theta<T>(s, k, rows_ap, R, g, G, smem, true, false, W);
  if (!group_sync(grp)) return false;
  clk.lap(s.prof, PF_THETA);
  if (!phase_jacobi<T, VEC>(s, X, W, Rr, Cc, g, G, grp, smem)) return false;
  clk.lap(s.prof, 15);
  phase_norms<T>(s, X, Rr, Cc, g, G);
  if (!group_sync(grp)) return false;
  clk.lap(s.prof, PF_NORMS);
  if (g == 0) phase_select(s, Rr, true, smem, true);
  if (!group_sync(grp)) return false;
  clk.lap(s.prof, PF_SELECT);
  if (!refine_gate<T>(s, k, ltr, Rr, Cc, g, G, grp, smem)) return false;
  if (g == 0 && threadIdx.x == 0) s.dims[k + 1] = s.ctr[CT_RANK];
  const bool ok = group_sync(grp);
  clk.lap(s.prof, PF_ABSORB);
  return ok;
}

// SVD of the R x C block already in X alone (the tuner's unit of work):
// W = I, the Jacobi, then the squared row norms.
template <typename T, int VEC = 1>
__device__ __forceinline__ bool op_jacobi(const Slot& s, int R, int C, int g, int G,
                                          Group& grp, double* smem) {
  T* X = reinterpret_cast<T*>(s.X);
  T* W = reinterpret_cast<T*>(s.W);
  set_identity(W, R, g, G);
  if (!group_sync(grp)) return false;
  if (!phase_jacobi<T, VEC>(s, X, W, R, C, g, G, grp, smem)) return false;
  phase_norms<T>(s, X, R, C, g, G);
  return group_sync(grp);
}

// Centre move away from site c: to c+1 (ltr) or c-1.
template <typename T, int VEC = 1>
__device__ __forceinline__ bool op_move(const Slot& s, int c, bool ltr, int g, int G,
                        Group& grp, double* smem) {
  const int cl = s.dims[c], cr = s.dims[c + 1];
  T* X = reinterpret_cast<T*>(s.X);
  T* W = reinterpret_cast<T*>(s.W);
  T* M = site_ptr<T>(s, c);
  const int Rr = ltr ? cr : cl, Cc = ltr ? 4 * cl : 4 * cr;
  PhaseClock clk(g == 0 && s.prof != nullptr);
  // X = M^T (chi_r x 4 chi_l) or M (chi_l x 4 chi_r)
  {
    if (ltr) {
      T* tile = reinterpret_cast<T*>(smem);
      const int na = 4 * cl;   // rows of M
      const int ta = (na + 31) / 32, tj = (cr + 31) / 32;
      for (int t = g; t < ta * tj; t += G) {
        const int a0 = (t / tj) * 32, j0 = (t % tj) * 32;
        __syncthreads();
        for (int e = threadIdx.x; e < 1024; e += NT) {
          const int al = e >> 5, jl = e & 31;
          T v = T(0);
          if (a0 + al < na && j0 + jl < cr) v = M[(size_t)(a0 + al) * cr + j0 + jl];
          tile[al * 33 + jl] = v;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 1024; e += NT) {
          const int jl = e >> 5, al = e & 31;
          if (a0 + al < na && j0 + jl < cr)
            X[(size_t)(j0 + jl) * na + a0 + al] = tile[al * 33 + jl];
        }
      }
      __syncthreads();
    } else {
      const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
      for (int r = g * 4 + w; r < cl; r += 4 * G)
        for (int cc = lane; cc < Cc; cc += 64) {
          const T v = M[(size_t)r * Cc + cc];
          X[(size_t)r * Cc + cc] = v;
        }
    }
  }
  if (!group_sync(grp)) return false;
  clk.lap(s.prof, PF_MOVE_PREP);
  if (!phase_jacobi<T, VEC>(s, X, W, Rr, Cc, g, G, grp, smem)) return false;
  clk.lap(s.prof, 15);
  phase_norms<T>(s, X, Rr, Cc, g, G);
  if (!group_sync(grp)) return false;
  if (g == 0) phase_select(s, Rr, false, smem);
  if (!group_sync(grp)) return false;
  clk.lap(s.prof, PF_SELECT);
  const bool ok = refine_move<T>(s, c, ltr, Rr, Cc, g, G, grp, smem) == 1;
  clk.lap(s.prof, PF_MOVE_GEMM);
  return ok;
}

}  // namespace nze

#endif
