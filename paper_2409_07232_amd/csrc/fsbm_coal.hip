// fsbm_coal.hip -- host side of the C ABI (include/fsbm_coal.h): handle,
// model tables, workspace, launch sequence, hipGraph cache, diagnostics.
//
// A call of fsbm_coal_step enqueues, on the caller's stream:
//   zero counters -> compaction (count, scan, gather, padding) ->
//   ceil(nsteps / steps_per_launch) step kernels -> scatter back.
// With a non-null stream the sequence is captured once into a hipGraph and
// replayed while (N, p, npoints, dt, nsteps, stream, launch shape) repeat.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/fsbm_coal.h"
#include "fsbm_internal.hpp"

using namespace fsbm;

namespace {

constexpr int kCompactBlock = 256;
constexpr double kDefaultX1 = 3.3510321638291124e-11;  // 2 um water drop
constexpr double kHitTol = 1e-12;

struct GraphKey {
  const void *N = nullptr;
  const void *p = nullptr;
  int64_t npoints = -1;
  double dt = 0.0;
  int nsteps = -1;
  void *stream = nullptr;
  int spl = 0, wpb = 0;
  bool operator==(const GraphKey &o) const {
    return N == o.N && p == o.p && npoints == o.npoints && dt == o.dt &&
           nsteps == o.nsteps && stream == o.stream && spl == o.spl &&
           wpb == o.wpb;
  }
};

}  // namespace

struct fsbm_coal_s {
  int device = 0;
  int B = 0, S = 0, L = 0, s = 1, precision = FSBM_FP64, flags = 0;
  int steps_per_launch = 0, waves_per_block = 0;
  double x1 = kDefaultX1, theta = 1e-30;
  std::vector<double> x, ct;
  std::vector<int> kt, product;
  // device model
  void *dmem = nullptr;
  DevModel dm{};
  // workspace
  void *wmem = nullptr;
  size_t wbytes = 0;
  int64_t wpoints = -1;  // points the workspace was laid out for
  DevWork ws{};
  int nblocks = 0;
  // graph cache
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  GraphKey gkey;
  // profiling (FSBM_FLAG_PROFILE): event pairs around collision launches
  std::vector<hipEvent_t> ev_start, ev_stop;
  int ev_used = 0;
  int prof_launches = 0;
  double prof_ms = 0.0;
  // last call
  hipStream_t last_stream = nullptr;
  int64_t last_npoints = 0;
  std::string last_error;
};

namespace {

int hip_fail(fsbm_coal_t h, hipError_t e, const char *what) {
  if (h) {
    h->last_error = std::string(what) + ": " + hipGetErrorString(e);
  }
  return FSBM_EHIP;
}

#define HIP_TRY(h, call)                                   \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hip_fail((h), e_, #call); \
  } while (0)

double grid_mass(double x1, int s, int k) {
  return ldexp(x1 * pow(2.0, (double)(k % s) / (double)s), k / s);
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Tunable launch shape: the cache file holds lines
// "B S precision steps_per_launch waves_per_block".
void read_tune_cache(fsbm_coal_t h) {
  const char *path = getenv("FSBM_TUNE_CACHE");
  if (!path) return;
  FILE *f = fopen(path, "r");
  if (!f) return;
  int B, S, pr, spl, wpb;
  while (fscanf(f, "%d %d %d %d %d", &B, &S, &pr, &spl, &wpb) == 5) {
    if (B == h->B && S == h->S && pr == h->precision && spl > 0 &&
        wpb >= 1 && wpb <= 4) {
      if (h->steps_per_launch == 0) h->steps_per_launch = spl;
      h->waves_per_block = wpb;
    }
  }
  fclose(f);
}

int build_model(fsbm_coal_t h, const double *tables, const double *plev) {
  const int B = h->B, S = h->S, L = h->L;
  const int nbr = L > 1 ? L - 1 : 1;
  const int npairs = S * (S + 1) / 2;
  h->x.resize(B);
  for (int k = 0; k < B; ++k) h->x[k] = grid_mass(h->x1, h->s, k);
  h->kt.assign((size_t)B * B, -1);
  h->ct.assign((size_t)B * B, 0.0);
  for (int i = 0; i < B; ++i)
    for (int j = 0; j < B; ++j) {
      const double sum = h->x[i] + h->x[j];
      int k = 0;
      while (grid_mass(h->x1, h->s, k + 1) <= sum * (1.0 + kHitTol)) ++k;
      double c = 0.0;
      if (k >= B) {
        k = -1;
      } else if (k <= B - 2) {
        c = (sum - h->x[k]) / (h->x[k + 1] - h->x[k]);
        c = c < 0.0 ? 0.0 : (c > 1.0 ? 1.0 : c);
      }
      h->kt[(size_t)i * B + j] = k;
      h->ct[(size_t)i * B + j] = c;
    }
  // device image: x, invx, ct, Kd (FP64, 8-byte aligned first), then FP32
  // and int arrays
  const size_t nKd = (size_t)npairs * nbr * B * B * 2;
  std::vector<double> invx(B), Kd(nKd);
  std::vector<float> invxf(B), ctf((size_t)B * B), Kf(nKd);
  for (int k = 0; k < B; ++k) {
    invx[k] = 1.0 / h->x[k];
    invxf[k] = (float)invx[k];
  }
  for (size_t q = 0; q < (size_t)B * B; ++q) ctf[q] = (float)h->ct[q];
  for (int ab = 0; ab < npairs; ++ab)
    for (int br = 0; br < nbr; ++br)
      for (int q = 0; q < B * B; ++q) {
        const double *t = tables + (size_t)ab * L * B * B;
        double lo, d;
        if (L == 1) {
          lo = t[q];
          d = 0.0;
        } else {
          const double kl = t[(size_t)br * B * B + q];
          const double kl1 = t[(size_t)(br + 1) * B * B + q];
          lo = kl1;
          d = kl - kl1;
        }
        const size_t o = (((size_t)ab * nbr + br) * B * B + q) * 2;
        Kd[o] = lo;
        Kd[o + 1] = d;
        Kf[o] = (float)lo;
        Kf[o + 1] = (float)d;
      }
  // species pair 0 tables transposed to [br][j][i] for the one-point-per-
  // lane kernels
  const size_t nT = (size_t)nbr * B * B * 2;
  std::vector<double> KdT(nT), ctT((size_t)B * B);
  std::vector<float> KfT(nT), ctfT((size_t)B * B);
  for (int br = 0; br < nbr; ++br)
    for (int i = 0; i < B; ++i)
      for (int j = 0; j < B; ++j)
        for (int e = 0; e < 2; ++e) {
          const size_t src = (((size_t)br * B + i) * B + j) * 2 + e;
          const size_t dst = (((size_t)br * B + j) * B + i) * 2 + e;
          KdT[dst] = Kd[src];
          KfT[dst] = Kf[src];
        }
  for (int i = 0; i < B; ++i)
    for (int j = 0; j < B; ++j) {
      ctT[(size_t)j * B + i] = h->ct[(size_t)i * B + j];
      ctfT[(size_t)j * B + i] = ctf[(size_t)i * B + j];
    }
  struct Part {
    const void *src;
    size_t bytes;
    size_t off;
  };
  std::vector<Part> parts = {
      {h->x.data(), sizeof(double) * B, 0},
      {invx.data(), sizeof(double) * B, 0},
      {h->ct.data(), sizeof(double) * B * B, 0},
      {Kd.data(), sizeof(double) * nKd, 0},
      {plev, sizeof(double) * L, 0},
      {invxf.data(), sizeof(float) * B, 0},
      {ctf.data(), sizeof(float) * B * B, 0},
      {Kf.data(), sizeof(float) * nKd, 0},
      {h->kt.data(), sizeof(int) * B * B, 0},
      {h->product.data(), sizeof(int) * S * S, 0},
      {KdT.data(), sizeof(double) * nT, 0},
      {ctT.data(), sizeof(double) * B * B, 0},
      {KfT.data(), sizeof(float) * nT, 0},
      {ctfT.data(), sizeof(float) * B * B, 0},
  };
  size_t off = 0;
  for (auto &p : parts) {
    p.off = off;
    off = align_up(off + p.bytes, 256);
  }
  HIP_TRY(h, hipMalloc(&h->dmem, off));
  std::vector<unsigned char> img(off, 0);
  for (auto &p : parts) memcpy(img.data() + p.off, p.src, p.bytes);
  HIP_TRY(h, hipMemcpy(h->dmem, img.data(), off, hipMemcpyHostToDevice));
  unsigned char *base = (unsigned char *)h->dmem;
  DevModel &m = h->dm;
  m.B = B;
  m.S = S;
  m.L = L;
  m.s = h->s;
  m.nbr = nbr;
  m.npairs = npairs;
  m.theta = h->theta;
  m.x = (const double *)(base + parts[0].off);
  m.invx = (const double *)(base + parts[1].off);
  m.ct = (const double *)(base + parts[2].off);
  m.Kd = (const double *)(base + parts[3].off);
  m.plev = (const double *)(base + parts[4].off);
  m.invxf = (const float *)(base + parts[5].off);
  m.ctf = (const float *)(base + parts[6].off);
  m.Kf = (const float *)(base + parts[7].off);
  m.kt = (const int *)(base + parts[8].off);
  m.product = (const int *)(base + parts[9].off);
  m.KdT = (const double *)(base + parts[10].off);
  m.ctT = (const double *)(base + parts[11].off);
  m.KfT = (const float *)(base + parts[12].off);
  m.ctfT = (const float *)(base + parts[13].off);
  return FSBM_OK;
}

void drop_graph(fsbm_coal_t h) {
  if (h->gexec) hipGraphExecDestroy(h->gexec);
  if (h->graph) hipGraphDestroy(h->graph);
  h->gexec = nullptr;
  h->graph = nullptr;
  h->gkey = GraphKey();
}

// Workspace for up to npoints points: slots, SoA state, weights, compaction
// scratch, totals and counters in one allocation.
int ensure_workspace(fsbm_coal_t h, int64_t npoints) {
  if (npoints <= h->wpoints) return FSBM_OK;
  const int SB = h->S * h->B;
  const int64_t cap64 =
      (int64_t)align_up((size_t)npoints + (size_t)kWave * h->dm.nbr, kSlotAlign);
  if (cap64 > (int64_t)0x7fffff00) return FSBM_EUNSUPPORTED;
  const int cap = (int)cap64;
  const int nblocks = (int)((npoints + kCompactBlock - 1) / kCompactBlock);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const size_t o_state = take(sizeof(double) * (size_t)SB * cap);
  const size_t o_wgt = take(sizeof(double) * cap);
  const size_t o_tot = take(sizeof(double) * 4 * (size_t)npoints);
  const size_t o_slot = take(sizeof(int) * cap);
  const size_t o_bc = take(sizeof(int) * (size_t)nblocks * kMaxBuckets);
  const size_t o_bo = take(sizeof(int) * (size_t)nblocks * kMaxBuckets);
  const size_t o_meta = take(sizeof(CompactMeta));
  const size_t o_cnt = take(sizeof(unsigned long long) * 4);
  const size_t o_pend = take(sizeof(int) * cap);
  drop_graph(h);
  if (h->wmem) hipFree(h->wmem);
  h->wmem = nullptr;
  h->wpoints = -1;
  hipError_t e = hipMalloc(&h->wmem, off);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    h->last_error = "workspace allocation failed";
    return FSBM_ENOMEM;
  }
  unsigned char *b = (unsigned char *)h->wmem;
  h->wbytes = off;
  h->ws.npoints = npoints;
  h->ws.slot_cap = cap;
  h->ws.state = (double *)(b + o_state);
  h->ws.wgt = (double *)(b + o_wgt);
  h->ws.tot = (double *)(b + o_tot);
  h->ws.slot_point = (int *)(b + o_slot);
  h->ws.block_counts = (int *)(b + o_bc);
  h->ws.block_offsets = (int *)(b + o_bo);
  h->ws.meta = (CompactMeta *)(b + o_meta);
  h->ws.counters = (unsigned long long *)(b + o_cnt);
  h->ws.pending = (int *)(b + o_pend);
  // pending[] is kept at zero by the kernels after this first clear
  e = hipMemset(h->ws.pending, 0, sizeof(int) * cap);
  if (e != hipSuccess) return hip_fail(h, e, "hipMemset");
  h->nblocks = nblocks;
  h->wpoints = npoints;
  return FSBM_OK;
}

int default_steps_per_launch(fsbm_coal_t h) {
  return h->steps_per_launch > 0 ? h->steps_per_launch : 10;
}
int default_wpb(fsbm_coal_t h) {
  return h->waves_per_block > 0 ? h->waves_per_block : 1;
}

int event_pair(fsbm_coal_t h, hipEvent_t *a, hipEvent_t *b);

// The launch sequence of one step call (capturable unless profiling).
int enqueue_call(fsbm_coal_t h, double *N, const double *p, int64_t npoints,
                 double dt, int nsteps, hipStream_t st, int spl, int wpb) {
  const DevModel &m = h->dm;
  DevWork &w = h->ws;
  HIP_TRY(h, launch_zero_u64(w.counters, 4, st));
  HIP_TRY(h, launch_compact_count(N, p, npoints, m.S * m.B, m.plev, m.L,
                                  w.block_counts, h->nblocks, st));
  HIP_TRY(h, launch_compact_scan(w.block_counts, w.block_offsets, h->nblocks,
                                 m.nbr, w.meta, st));
  HIP_TRY(h, launch_compact_gather(N, p, npoints, m.S, m.B, m.plev, m.L,
                                   w.block_offsets, w.meta, h->nblocks,
                                   w.slot_point, w.state, w.wgt, w.slot_cap,
                                   m.x, w.tot, st));
  HIP_TRY(h, launch_fill_padding(w.meta, w.slot_point, w.slot_cap, st));
  StepArgs a;
  a.m = m;
  a.slot_cap = w.slot_cap;
  a.slot_point = w.slot_point;
  a.state = w.state;
  a.wgt = w.wgt;
  a.meta = w.meta;
  a.counters = w.counters;
  a.pending = w.pending;
  a.dt = dt;
  const int max_slots = w.slot_cap;
  for (int done = 0; done < nsteps; done += spl) {
    a.nsteps = (nsteps - done) < spl ? (nsteps - done) : spl;
    if (lane_kernel_supported(m.B, m.S, m.s) &&
        !(h->flags & FSBM_FLAG_FORCE_WAVE)) {
      const bool prof = (h->flags & FSBM_FLAG_PROFILE) != 0;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (prof) {
        const int rc = event_pair(h, &e0, &e1);
        if (rc != FSBM_OK) return rc;
        HIP_TRY(h, hipEventRecord(e0, st));
      }
      HIP_TRY(h, launch_lane_step(a, h->precision, wpb, max_slots, st));
      if (prof) HIP_TRY(h, hipEventRecord(e1, st));
      HIP_TRY(h, launch_slow_steps(a, max_slots, st));
    } else {
      h->last_error = "no kernel for this grid yet";
      return FSBM_EUNSUPPORTED;
    }
  }
  HIP_TRY(h, launch_scatter(N, npoints, m.S, m.B, w.meta, w.slot_point,
                            w.state, w.slot_cap, m.x, w.tot, st));
  return FSBM_OK;
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

// Collect the durations of the timed launches of the previous call (their
// stream has been synchronised by the caller or is synchronised here).
int harvest_events(fsbm_coal_t h) {
  if (h->ev_used == 0) return FSBM_OK;
  HIP_TRY(h, hipEventSynchronize(h->ev_stop[h->ev_used - 1]));
  for (int k = 0; k < h->ev_used; ++k) {
    float ms = 0.0f;
    HIP_TRY(h, hipEventElapsedTime(&ms, h->ev_start[k], h->ev_stop[k]));
    h->prof_ms += ms;
    h->prof_launches += 1;
  }
  h->ev_used = 0;
  return FSBM_OK;
}

int event_pair(fsbm_coal_t h, hipEvent_t *a, hipEvent_t *b) {
  if (h->ev_used == (int)h->ev_start.size()) {
    hipEvent_t e0, e1;
    HIP_TRY(h, hipEventCreate(&e0));
    HIP_TRY(h, hipEventCreate(&e1));
    h->ev_start.push_back(e0);
    h->ev_stop.push_back(e1);
  }
  *a = h->ev_start[h->ev_used];
  *b = h->ev_stop[h->ev_used];
  h->ev_used++;
  return FSBM_OK;
}

}  // namespace

extern "C" {

void fsbm_coal_opts_default(fsbm_coal_opts *o) {
  if (!o) return;
  o->x1_g = kDefaultX1;
  o->s = 1;
  o->product = nullptr;
  o->precision = FSBM_FP64;
  o->theta = 1e-30;
  o->steps_per_launch = 0;
  o->flags = 0;
}

int fsbm_coal_create(int32_t nbins, int32_t nspecies,
                     const double *kernel_tables, int32_t nlevels,
                     const double *p_levels_hpa, const fsbm_coal_opts *opts,
                     fsbm_coal_t *out) {
  if (!out) return FSBM_EINVAL;
  *out = nullptr;
  fsbm_coal_opts o;
  fsbm_coal_opts_default(&o);
  if (opts) o = *opts;
  if (nbins < 2 || nspecies < 1 || nspecies > kMaxSpecies || nlevels < 1 ||
      !kernel_tables || !p_levels_hpa)
    return FSBM_EINVAL;
  if (nbins > kMaxBins || nlevels - 1 > kMaxBuckets) return FSBM_EUNSUPPORTED;
  if (o.s < 1 || !finite_pos(o.x1_g) || !(o.theta >= 0.0) ||
      !isfinite(o.theta) || (o.precision != FSBM_FP64 &&
                             o.precision != FSBM_FP32C) ||
      o.steps_per_launch < 0)
    return FSBM_EINVAL;
  for (int l = 0; l < nlevels; ++l)
    if (!isfinite(p_levels_hpa[l])) return FSBM_EINVAL;
  for (int l = 0; l + 1 < nlevels; ++l)
    if (!(p_levels_hpa[l] > p_levels_hpa[l + 1])) return FSBM_EINVAL;
  const size_t nt = (size_t)nspecies * (nspecies + 1) / 2 * nlevels * nbins *
                    nbins;
  for (size_t q = 0; q < nt; ++q)
    if (!(kernel_tables[q] >= 0.0) || !isfinite(kernel_tables[q]))
      return FSBM_EINVAL;
  std::vector<int> product((size_t)nspecies * nspecies, 0);
  if (o.product) {
    for (int a = 0; a < nspecies; ++a)
      for (int b = 0; b < nspecies; ++b) {
        const int P = o.product[a * nspecies + b];
        if (P < 0 || P >= nspecies || P != o.product[b * nspecies + a])
          return FSBM_EINVAL;
        product[(size_t)a * nspecies + b] = P;
      }
  } else if (nspecies > 1) {
    return FSBM_EINVAL;
  }
  fsbm_coal_t h = new (std::nothrow) fsbm_coal_s;
  if (!h) return FSBM_ENOMEM;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return FSBM_EHIP;
  }
  h->B = nbins;
  h->S = nspecies;
  h->L = nlevels;
  h->s = o.s;
  h->x1 = o.x1_g;
  h->theta = o.theta;
  h->precision = o.precision;
  h->flags = o.flags;
  h->steps_per_launch = o.steps_per_launch;
  h->product = product;
  read_tune_cache(h);
  const int rc = build_model(h, kernel_tables, p_levels_hpa);
  if (rc != FSBM_OK) {
    fsbm_coal_destroy(h);
    return rc;
  }
  *out = h;
  return FSBM_OK;
}

int fsbm_coal_step(fsbm_coal_t h, double *N, const double *p_hpa,
                   int64_t npoints, double dt_s, int32_t nsteps,
                   void *stream) {
  if (!h || npoints < 0 || nsteps < 0 || !isfinite(dt_s) || !(dt_s > 0.0))
    return FSBM_EINVAL;
  if (npoints == 0 || nsteps == 0) return FSBM_OK;
  if (!N || !p_hpa) return FSBM_EINVAL;
  if (!lane_kernel_supported(h->B, h->S, h->s) ||
      (h->flags & FSBM_FLAG_FORCE_WAVE)) {
    h->last_error = "no kernel for this grid yet";
    return FSBM_EUNSUPPORTED;
  }
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(h, hipSetDevice(h->device));
  int rc = ensure_workspace(h, npoints);
  if (rc != FSBM_OK) return rc;
  if (h->flags & FSBM_FLAG_DEBUG_CHECKS) {
    int *bad = (int *)h->ws.block_counts;  // scratch int, rewritten later
    int hbad = 0;
    HIP_TRY(h, hipMemcpyAsync(bad, &hbad, sizeof(int), hipMemcpyHostToDevice,
                              st));
    HIP_TRY(h, launch_check_state(N, npoints * h->S * h->B, bad, st));
    HIP_TRY(h, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost,
                              st));
    HIP_TRY(h, hipStreamSynchronize(st));
    if (hbad) return FSBM_EDOMAIN;
  }
  const int spl = default_steps_per_launch(h);
  const int wpb = default_wpb(h);
  rc = harvest_events(h);
  if (rc != FSBM_OK) return rc;
  h->last_stream = st;
  h->last_npoints = npoints;
  const bool use_graph = st != nullptr &&
                         !(h->flags & (FSBM_FLAG_NO_GRAPH | FSBM_FLAG_PROFILE));
  if (!use_graph) return enqueue_call(h, N, p_hpa, npoints, dt_s, nsteps, st,
                                      spl, wpb);
  GraphKey key;
  key.N = N;
  key.p = p_hpa;
  key.npoints = npoints;
  key.dt = dt_s;
  key.nsteps = nsteps;
  key.stream = stream;
  key.spl = spl;
  key.wpb = wpb;
  if (!(h->gexec && key == h->gkey)) {
    drop_graph(h);
    HIP_TRY(h, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    rc = enqueue_call(h, N, p_hpa, npoints, dt_s, nsteps, st, spl, wpb);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (rc != FSBM_OK) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamEndCapture");
    h->graph = g;
    e = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      drop_graph(h);
      return hip_fail(h, e, "hipGraphInstantiate");
    }
    h->gkey = key;
  }
  HIP_TRY(h, hipGraphLaunch(h->gexec, st));
  return FSBM_OK;
}

int fsbm_coal_step_multi(const fsbm_coal_t *hs, int32_t ngrids,
                         double *const *N, const double *const *p_hpa,
                         const int64_t *npoints, double dt_s, int32_t nsteps,
                         void *stream) {
  if (!hs || ngrids < 0 || !N || !p_hpa || !npoints) return FSBM_EINVAL;
  for (int g = 0; g < ngrids; ++g) {
    const int rc = fsbm_coal_step(hs[g], N[g], p_hpa[g], npoints[g], dt_s,
                                  nsteps, stream);
    if (rc != FSBM_OK) return rc;
  }
  return FSBM_OK;
}

int fsbm_coal_tune(fsbm_coal_t h, int64_t npoints_hint, void *stream) {
  (void)npoints_hint;
  (void)stream;
  if (!h) return FSBM_EINVAL;
  return FSBM_OK;
}

int fsbm_coal_totals(fsbm_coal_t h, double *mass_before, double *mass_after,
                     double *num_before, double *num_after) {
  if (!h) return FSBM_EINVAL;
  if (h->wpoints < 0 || h->last_npoints == 0) return FSBM_EINVAL;
  const int64_t n = h->last_npoints;
  double *dst[4] = {mass_before, mass_after, num_before, num_after};
  for (int k = 0; k < 4; ++k)
    if (dst[k])
      HIP_TRY(h, hipMemcpyAsync(dst[k], h->ws.tot + (size_t)k * n,
                                sizeof(double) * n, hipMemcpyDeviceToDevice,
                                h->last_stream));
  return FSBM_OK;
}

int fsbm_coal_get_stats(fsbm_coal_t h, fsbm_coal_stats *out) {
  if (!h || !out) return FSBM_EINVAL;
  memset(out, 0, sizeof(*out));
  out->kernel = (lane_kernel_supported(h->B, h->S, h->s) &&
                 !(h->flags & FSBM_FLAG_FORCE_WAVE))
                    ? 0
                    : 1;
  out->steps_per_launch = default_steps_per_launch(h);
  out->waves_per_block = default_wpb(h);
  if (h->wpoints < 0) return FSBM_OK;
  HIP_TRY(h, hipStreamSynchronize(h->last_stream));
  const int rc = harvest_events(h);
  if (rc != FSBM_OK) return rc;
  out->kernel_launches = h->prof_launches;
  out->kernel_ms = h->prof_ms;
  unsigned long long c[4];
  CompactMeta meta;
  HIP_TRY(h, hipMemcpy(c, h->ws.counters, sizeof(c), hipMemcpyDeviceToHost));
  HIP_TRY(h, hipMemcpy(&meta, h->ws.meta, sizeof(meta),
                       hipMemcpyDeviceToHost));
  out->active_points = meta.nactive;
  out->pair_evals = (int64_t)c[0];
  out->limiter_steps = (int64_t)c[1];
  out->fp64_fallback_steps = (int64_t)c[2];
  return FSBM_OK;
}

int fsbm_coal_destroy(fsbm_coal_t h) {
  if (!h) return FSBM_OK;
  drop_graph(h);
  for (auto e : h->ev_start) hipEventDestroy(e);
  for (auto e : h->ev_stop) hipEventDestroy(e);
  if (h->wmem) hipFree(h->wmem);
  if (h->dmem) hipFree(h->dmem);
  delete h;
  return FSBM_OK;
}

const char *fsbm_coal_strerror(int code) {
  switch (code) {
    case FSBM_OK:
      return "success";
    case FSBM_EINVAL:
      return "invalid argument";
    case FSBM_ENOMEM:
      return "out of memory";
    case FSBM_EHIP:
      return "HIP runtime error";
    case FSBM_EUNSUPPORTED:
      return "unsupported configuration";
    case FSBM_EDOMAIN:
      return "state holds negative or non-finite values";
    default:
      return "unknown error";
  }
}

const char *fsbm_coal_last_error(fsbm_coal_t h) {
  return h ? h->last_error.c_str() : "";
}

}  // extern "C"
