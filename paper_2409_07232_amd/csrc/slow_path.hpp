// slow_path.hpp -- exact FP64 step of one point with the positivity limiter,
// run by one lane with private arrays.  The fast kernels call it only for
// points whose cheap over-demand bound fired (rare: a bin might lose more
// mass than it holds), so its per-lane scratch traffic does not matter.
#pragma once

#include "device_common.hpp"

namespace fsbm {

struct PairNets {
  int n;
  int bin[4];
  double amt[4];
  __device__ __forceinline__ void put(int b, double v) {
    for (int e = 0; e < n; ++e)
      if (bin[e] == b) {
        amt[e] += v;
        return;
      }
    bin[n] = b;
    amt[n] = v;
    ++n;
  }
};

// Interpolated kernel of species pair ab (a <= b), bins (i, j), bracket br.
__device__ __forceinline__ double kernel_at_f64(const DevModel &m, int ab,
                                                int br, int i, int j,
                                                double w) {
  const double *e =
      m.Kd + ((((size_t)ab * m.nbr + br) * m.B + i) * m.B + j) * 2;
  return fma(e[1], w, e[0]);
}

// Nets of one bin pair (a,i) x (b,j): the collided mass leaves both source
// bins, the merged mass enters the bin k below x_i + x_j and the flux
// fraction moves on to k+1.  Returns false if the pair contributes nothing.
__device__ __forceinline__ bool pair_nets_f64(const DevModel &m,
                                              const double *Mt,
                                              const double *Nv, int a, int i,
                                              int b, int j, double K,
                                              double dt, PairNets &out) {
  const int B = m.B;
  const int k = m.kt[i * B + j];
  out.n = 0;
  if (k < 0) return false;
  double C = dt * K * Nv[a * B + i] * Nv[b * B + j];
  if (a == b && i == j) C *= 0.5;
  if (C == 0.0) return false;
  const double A = C * m.x[i];
  const double Bm = C * m.x[j];
  const double Sm = A + Bm;
  const int P = m.product[a * m.S + b];
  double F = 0.0;
  if (k <= B - 2) {
    const double r = Mt[P * B + k + 1] / (Mt[P * B + k] + Sm);
    double x1 = log_f64(r);
    if (!(x1 >= kX1Floor)) x1 = kX1Floor;
    F = flux_fraction_f64(m.ct[i * B + j], x1) * Sm;
  }
  // a source bin that also receives the merged mass gets the other
  // source's collided mass minus the flux in one subtraction (no rounded
  // A + Bm followed by the removal of Bm)
  const int qa = a * B + i, qb = b * B + j, qk = P * B + k;
  if (qk == qb && qk != qa) {
    out.put(qa, -A);
    out.put(qb, A - F);
  } else if (qk == qa && qk != qb) {
    out.put(qa, Bm - F);
    out.put(qb, -Bm);
  } else {
    out.put(qa, -A);
    out.put(qb, -Bm);
    out.put(qk, Sm - F);
  }
  if (k <= B - 2) out.put(qk + 1, F);
  return true;
}

// One FP64 step of the point whose bins sit at st[q * stride], q =
// species*B + bin, in the oracle's two-pass structure.  work holds 7 arrays
// of S*B doubles (private memory or global scratch).  Returns 1 if the
// limiter fired; *npairs counts evaluated pairs.
__device__ __noinline__ int slow_step_core(const DevModel &m, double *st,
                                           int stride, double w, int br,
                                           double dt,
                                           unsigned long long *npairs,
                                           double *work) {
  const int B = m.B, S = m.S, n = S * B;
  double *M = work, *Mt = work + n, *Nv = work + 2 * n, *G = work + 3 * n,
         *L = work + 4 * n, *D = work + 5 * n, *sig = work + 6 * n;
  double Mtot = 0.0;
  for (int q = 0; q < n; ++q) {
    Nv[q] = st[(size_t)q * stride];
    M[q] = Nv[q] * m.x[q % B];
    Mtot += M[q];
  }
  if (Mtot == 0.0) return 0;
  const double thr = m.theta * Mtot;
  for (int q = 0; q < n; ++q) {
    const bool act = M[q] > 0.0 && M[q] >= thr;
    Mt[q] = act ? M[q] : 0.0;
    G[q] = L[q] = D[q] = 0.0;
    sig[q] = 1.0;
  }
  int limited = 0;
  unsigned long long cnt = 0;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      for (int q = 0; q < n; ++q)
        if (D[q] > M[q]) limited = 1;
      if (!limited) break;
      for (int q = 0; q < n; ++q) {
        sig[q] = (D[q] > M[q]) ? M[q] / D[q] : 1.0;
        G[q] = L[q] = 0.0;
      }
    }
    for (int a = 0; a < S; ++a)
      for (int b = a; b < S; ++b) {
        const int ab = a * S - (a * (a - 1)) / 2 + (b - a);
        for (int i = 0; i < B; ++i) {
          if (Mt[a * B + i] == 0.0) continue;
          for (int j = (a == b ? i : 0); j < B; ++j) {
            if (Mt[b * B + j] == 0.0) continue;
            // counted like the fast kernels: target on the grid and a
            // kernel entry nonzero at some level (one species here)
            if (pass == 0 && m.kt[i * B + j] >= 0 &&
                ((m.nzT[j] >> i) & 1ull))
              ++cnt;
            PairNets pn;
            const double K = kernel_at_f64(m, ab, br, i, j, w);
            if (!pair_nets_f64(m, Mt, Nv, a, i, b, j, K, dt, pn)) continue;
            double scale = 1.0;
            if (pass == 1)
              for (int e = 0; e < pn.n; ++e)
                if (pn.amt[e] < 0.0 && sig[pn.bin[e]] < scale)
                  scale = sig[pn.bin[e]];
            for (int e = 0; e < pn.n; ++e) {
              const double v = pn.amt[e] * scale;
              if (v > 0.0) {
                G[pn.bin[e]] += v;
              } else if (v < 0.0) {
                L[pn.bin[e]] -= v;
                if (pass == 0) D[pn.bin[e]] -= v;
              }
            }
          }
        }
      }
  }
  for (int q = 0; q < n; ++q) {
    double Mn = M[q] + (G[q] - L[q]);
    if (Mn < 0.0) Mn = 0.0;
    st[(size_t)q * stride] = Mn / m.x[q % B];
  }
  *npairs += cnt;
  return limited;
}

// Same with private arrays for up to MAXSB bins.
template <int MAXSB>
__device__ __forceinline__ int slow_step_f64(const DevModel &m, double *st,
                                             int stride, double w, int br,
                                             double dt,
                                             unsigned long long *npairs) {
  double work[7 * MAXSB];
  return slow_step_core(m, st, stride, w, br, dt, npairs, work);
}

}  // namespace fsbm
