// sediment.hip -- sedimentation of the bin spectra of vertical columns: the
// term d((w - V_t) f)/dz of the bin equation (Sec. III, eq. (1)) in still
// air, first-order upwind in flux form, explicit, each step split into equal
// sub-steps so that no level passes on more than it holds.
//
// Mapping (gfx950): one thread per (column, species-bin) pair, consecutive
// threads on consecutive bins of a column, so that each level of a column
// is one contiguous run of S*B doubles read and written with consecutive
// lane addresses.  A thread keeps its whole column (register arrays of
// 32, 56 or kSedMaxLevels levels) in VGPRs for all steps of the call: the
// state is read once and written once per call, and the sweeps in between
// run from registers; the layer thicknesses, the same for every thread of
// a level, are scalar loads.  With one step per call the kernel is bound
// by HBM bandwidth (16 bytes per bin and point, plus the fall-speed
// factors); with many, by the FP64 division of each level update.
//
// Per sub-step of length tau, from the top level down, with the values at
// the start of the sub-step: F_l = v_l N_l tau leaves level l through its
// bottom face, N_l += (F_{l+1} - F_l) / dz_l, F_{nlev} = 0; F_0 is added to
// the column's precipitation.  v_l = V(species, bin) * vfac(column, level).
#include "device_common.hpp"

#pragma clang fp contract(off)

namespace fsbm {

namespace {

constexpr int kSedThreads = 256;

template <int NL>
__global__ void __launch_bounds__(kSedThreads) sed_steps(SedArgs a) {
  const int64_t t = (int64_t)blockIdx.x * kSedThreads + threadIdx.x;
  const int SB = a.SB;
  const int64_t col = t / SB;
  const int q = (int)(t - col * SB);
  if (col >= a.ncols) return;
  const double v = a.v[q];
  const double *fac = a.vfac ? a.vfac + col * a.nlev : nullptr;
  // the column in registers: every index below is static once the level
  // loops are unrolled (levels past nlev are predicated off)
  double n[NL];
  // sub-steps of this column and bin
  double cmax = 0.0;
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    n[l] = 0.0;
    if (l < a.nlev) {
      const double f = fac ? fac[l] : 1.0;
      const double cl = ((v * f) * a.dt) / ldc(a.dz + l);
      cmax = cl > cmax ? cl : cmax;
      n[l] = a.N[(col * a.col_stride + (int64_t)l * a.lev_stride) * SB + q];
    }
  }
  double ns = ceil(cmax);
  if (ns < 1.0) ns = 1.0;
  const int64_t nsub = (int64_t)ns;
  const double tau = a.dt / ns;
  double pr = a.precip ? a.precip[col * SB + q] : 0.0;
  for (int st = 0; st < a.nsteps; ++st)
    for (int64_t u = 0; u < nsub; ++u) {
      double fin = 0.0;  // flux entering from above
#pragma unroll
      for (int l = NL - 1; l >= 0; --l) {
        if (l < a.nlev) {
          const double f = fac ? fac[l] : 1.0;
          const double fout = ((v * f) * n[l]) * tau;
          n[l] = n[l] + (fin - fout) / ldc(a.dz + l);
          fin = fout;
        }
      }
      pr += fin;  // what left the bottom level
    }
#pragma unroll
  for (int l = 0; l < NL; ++l)
    if (l < a.nlev)
      a.N[(col * a.col_stride + (int64_t)l * a.lev_stride) * SB + q] = n[l];
  if (a.precip) a.precip[col * SB + q] = pr;
}

}  // namespace

hipError_t launch_sed_steps(const SedArgs &a, hipStream_t st) {
  if (a.nlev < 1 || a.nlev > kSedMaxLevels) return hipErrorInvalidValue;
  const int64_t threads = a.ncols * a.SB;
  const int64_t blocks = (threads + kSedThreads - 1) / kSedThreads;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (a.nlev <= 32)
    hipLaunchKernelGGL(sed_steps<32>, dim3((unsigned)blocks),
                       dim3(kSedThreads), 0, st, a);
  else if (a.nlev <= 56)
    hipLaunchKernelGGL(sed_steps<56>, dim3((unsigned)blocks),
                       dim3(kSedThreads), 0, st, a);
  else
    hipLaunchKernelGGL(sed_steps<kSedMaxLevels>, dim3((unsigned)blocks),
                       dim3(kSedThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace fsbm
