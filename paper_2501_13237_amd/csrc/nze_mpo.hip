// MPO handles, the persistent per-layer kernel, readout kernels and the
// host-side orchestration behind mpo_init / mpo_apply_layer / mpo_expect.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "nze.h"
#include "nze_internal.h"
#include "nze_phases.h"

namespace nze {

__device__ inline int ld_agent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------- kernels

// One launch applies a whole layer: every MPO of the batch walks through its
// list of steps (centre moves and gates) with a group of workgroups.
//   xcd == 0: workgroup b serves MPO wgmap[2b] as member wgmap[2b + 1] of a
//             group of gsize[MPO] (sized by the host to the MPO's work),
//             device-scope group barriers.
//   xcd == 1 (nmpo a multiple of 8): MPO m is served by workgroups running on
//             XCD m % 8, identified by the hardware XCC_ID and numbered by
//             arrival; after one census of the whole grid each XCD splits its
//             workgroups evenly over its MPOs, and group barriers stay inside
//             the XCD's L2.
// bar: [nmpo] group counters, then 8 per-XCD tickets and the census counter.
template <typename T, int VEC>
__device__ __forceinline__ void layer_body(const Slot* slots,
                                             const Step* steps,
                                             const double* ptms, int nsteps,
                                             int nmpo, int G, int* bar,
                                             int* abort_flag,
                                             unsigned long long timeout,
                                             int xcd, const int* wgmap,
                                             const int* gsize, double* smem,
                                             int* sflag) {
  int mpo = 0, g = 0;
  if (!xcd) {
    mpo = wgmap[2 * blockIdx.x];
    g = wgmap[2 * blockIdx.x + 1];
    G = gsize[mpo];
  } else {
    int* tick = bar + nmpo;
    int* census = bar + nmpo + 8;
    if (threadIdx.x == 0) {
      const int x = xcc_id();
      const int j = atomicAdd(tick + x, 1);
      atomicAdd(census, 1);
      int ok = 1;
      const uint64_t t0 = wall_clock64();
      while (ld_agent(census) < (int)gridDim.x) {
        if (ld_agent(abort_flag)) { ok = 0; break; }
        if (wall_clock64() - t0 > timeout) { atomicExch(abort_flag, 1); ok = 0; break; }
        __builtin_amdgcn_s_sleep(1);
      }
      const int per = nmpo / 8;                 // MPOs on this XCD
      const int gx = ld_agent(tick + x) / per;  // workgroups per MPO here
      sflag[1] = x + 8 * (j % per);
      sflag[2] = j / per;
      sflag[3] = ok ? gx : 0;
    }
    __syncthreads();
    mpo = sflag[1];
    g = sflag[2];
    G = sflag[3];
    __syncthreads();
    if (G == 0) {
      // census timed out, or this XCD has fewer workgroups than MPOs
      if (threadIdx.x == 0) atomicOr(&slots[mpo].ctr[CT_ERR], ERR_ABORT);
      return;
    }
    if (g >= G) return;                         // surplus workgroup
  }
  const Slot s = slots[mpo];
  Group grp{bar + mpo, abort_flag, G, 0, timeout, sflag, xcd};
  for (int st = 0; st < nsteps; ++st) {
    const Step op = steps[(size_t)st * nmpo + mpo];
    bool ok = true;
    switch (op.op) {
      case OP_GATE_LR:
      case OP_GATE_RL:
        ok = op_gate<T, VEC>(s, op.k, op.op == OP_GATE_LR, ptms + (size_t)op.ptm * 256, g, G, grp, smem);
        break;
      case OP_MOVE_LR:
      case OP_MOVE_RL:
        ok = op_move<T, VEC>(s, op.k, op.op == OP_MOVE_LR, g, G, grp, smem);
        break;
      case OP_JACOBI:
        ok = op_jacobi<T, VEC>(s, op.k, op.ptm, g, G, grp, smem);
        break;
      default:
        break;
    }
    if (!ok) {
      if (g == 0 && threadIdx.x == 0) atomicOr(&s.ctr[CT_ERR], ERR_ABORT);
      return;
    }
  }
}

// Entry points.  One workgroup per CU with vectorised rotations is what a
// Jacobi chain needs (the headline case: one job's levels).
#define NZE_LAYER_ARGS const Slot* slots, const Step* steps, const double* ptms, \
    int nsteps, int nmpo, int G, int* bar, int* abort_flag,                    \
    unsigned long long timeout, int xcd, const int* wgmap, const int* gsize
__global__ __launch_bounds__(NT) void k_layer_f32(NZE_LAYER_ARGS) {
  __shared__ double smem[SMEM_DOUBLES];
  __shared__ int sflag[4];
  layer_body<float, 1>(slots, steps, ptms, nsteps, nmpo, G, bar, abort_flag, timeout,
                       xcd, wgmap, gsize, smem, sflag);
}
// Two workgroups per CU (at most 256 registers a lane, scalar rotations):
// for batches whose groups outnumber the CUs, where independent MPOs on one
// CU hide each other's latencies.
__global__ __launch_bounds__(NT, 2) void k_layer_f32x2(NZE_LAYER_ARGS) {
  __shared__ double smem[SMEM_DOUBLES];
  __shared__ int sflag[4];
  layer_body<float, 0>(slots, steps, ptms, nsteps, nmpo, G, bar, abort_flag, timeout,
                       xcd, wgmap, gsize, smem, sflag);
}
__global__ __launch_bounds__(NT) void k_layer_f64(NZE_LAYER_ARGS) {
  __shared__ double smem[SMEM_DOUBLES];
  __shared__ int sflag[4];
  layer_body<double, 1>(slots, steps, ptms, nsteps, nmpo, G, bar, abort_flag, timeout,
                        xcd, wgmap, gsize, smem, sflag);
}
#undef NZE_LAYER_ARGS

__global__ void k_fill_int(int* p, int n, int v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = v;
}

// Product state: site k holds its 4 Pauli coordinates normalised to 1.
template <typename T>
__global__ void k_init(const Slot* slots, const double* init_sites, int n) {
  const Slot s = slots[blockIdx.x];
  T* sites = reinterpret_cast<T*>(s.sites);
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    double v[4];
    for (int p = 0; p < 4; ++p) v[p] = init_sites[4 * k + p];
    const double nv = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3]);
    for (int p = 0; p < 4; ++p) sites[(size_t)k * s.site_cap + p] = T(v[p] / nv);
  }
  for (int k = threadIdx.x; k <= n; k += blockDim.x) s.dims[k] = 1;
  for (int i = threadIdx.x; i < CT_COUNT; i += blockDim.x) s.ctr[i] = 0;
  if (s.prof)
    for (int i = threadIdx.x; i < PF_N; i += blockDim.x) s.prof[i] = 0.0;
  if (threadIdx.x == 0) {
    double lg = 0.0;
    for (int k = 0; k < n; ++k) {
      double q = 0.0;
      for (int p = 0; p < 4; ++p) q += init_sites[4 * k + p] * init_sites[4 * k + p];
      lg += 0.5 * log(q);
    }
    s.scal[SC_LOG] = lg;
    s.scal[SC_FID] = 1.0;
    s.scal[SC_MAXDISC] = 0.0;
    s.scal[SC_MINGAP] = 1.0;
    s.scal[SC_F2] = 0.0;
    s.scal[SC_KEPT] = 0.0;
    s.scal[SC_FLOPS] = 0.0;
    s.scal[SC_CAPQ] = 0.0;
  }
}

// Left (dir 0) and right (dir 1) environments of the identity slices, with a
// per-site rescale: env[k] holds the normalised vector, lg[k] its log factor.
template <typename T>
__global__ __launch_bounds__(NT) void k_env(const Slot* slots, double* env,
                                            double* lg, int env_stride) {
  const int mpo = blockIdx.x, dir = blockIdx.y;
  const Slot s = slots[mpo];
  const int n = s.n;
  double* E = env + ((size_t)mpo * 2 + dir) * env_stride;
  double* Lg = lg + ((size_t)mpo * 2 + dir) * (n + 1);
  __shared__ double v[2 * CHI_LIMIT];
  __shared__ double red[8];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double acc_log = 0.0;
  if (tid == 0) v[0] = 1.0;
  int cur = 0;
  const int k0 = dir == 0 ? 0 : n;
  if (tid == 0) { E[(size_t)k0 * s.chi] = 1.0; Lg[k0] = 0.0; }
  __syncthreads();
  for (int step = 0; step < n; ++step) {
    const int k = dir == 0 ? step : n - 1 - step;
    const int cl = s.dims[k], cr = s.dims[k + 1];
    const T* M = reinterpret_cast<const T*>(s.sites) + (size_t)k * s.site_cap;
    double* vin = v + cur * CHI_LIMIT;
    double* vout = v + (1 - cur) * CHI_LIMIT;
    double mx = 0.0;
    if (dir == 0) {
      for (int j = tid; j < cr; j += NT) {
        double a = 0.0;
        for (int i = 0; i < cl; ++i) a += vin[i] * double(M[(size_t)i * 4 * cr + j]);
        vout[j] = a;
        mx = fmax(mx, fabs(a));
      }
    } else {
      for (int i = w; i < cl; i += 4) {
        double a = 0.0;
        for (int j = lane; j < cr; j += 64) a += double(M[(size_t)i * 4 * cr + j]) * vin[j];
        a = wave_sum(a);
        if (lane == 0) vout[i] = a;
        mx = fmax(mx, fabs(a));
      }
    }
    __syncthreads();
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if (lane == 0) red[w] = mx;
    __syncthreads();
    mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    const int len = dir == 0 ? cr : cl;
    const double sc = mx > 0.0 ? 1.0 / mx : 1.0;
    acc_log += mx > 0.0 ? log(mx) : 0.0;
    const int kout = dir == 0 ? k + 1 : k;
    for (int j = tid; j < len; j += NT) {
      vout[j] *= sc;
      E[(size_t)kout * s.chi + j] = vout[j];
    }
    if (tid == 0) Lg[kout] = acc_log;
    __syncthreads();
    cur = 1 - cur;
  }
}

// One workgroup per (MPO, observable): contract the Pauli slices over the
// string's support between the identity environments.
template <typename T>
__global__ __launch_bounds__(NT) void k_obs(const Slot* slots, const double* env,
                                            const double* lg, int env_stride,
                                            const uint8_t* paulis,
                                            const int* span, int n_obs,
                                            double* out) {
  const int mpo = blockIdx.y, o = blockIdx.x;
  const Slot s = slots[mpo];
  const int n = s.n;
  const double* EL = env + ((size_t)mpo * 2 + 0) * env_stride;
  const double* ER = env + ((size_t)mpo * 2 + 1) * env_stride;
  const double* LL = lg + ((size_t)mpo * 2 + 0) * (n + 1);
  const double* LR = lg + ((size_t)mpo * 2 + 1) * (n + 1);
  __shared__ double v[2 * CHI_LIMIT];
  __shared__ double red[8];
  const int tid = threadIdx.x;
  const int f = span[2 * o], l = span[2 * o + 1];
  // trace c_I = EL[n] (a scalar) with log LL[n]
  const double cI = EL[(size_t)n * s.chi];
  const double lI = LL[n];
  if (f < 0) {                   // identity string
    if (tid == 0) out[(size_t)mpo * n_obs + o] = 1.0;
    return;
  }
  const uint8_t* P = paulis + (size_t)o * n;
  int cur = 0;
  for (int j = tid; j < s.dims[f]; j += NT) v[j] = EL[(size_t)f * s.chi + j];
  double acc_log = LL[f];
  __syncthreads();
  for (int k = f; k <= l; ++k) {
    const int cl = s.dims[k], cr = s.dims[k + 1];
    const int p = P[k];
    const T* M = reinterpret_cast<const T*>(s.sites) + (size_t)k * s.site_cap;
    double* vin = v + cur * CHI_LIMIT;
    double* vout = v + (1 - cur) * CHI_LIMIT;
    double mx = 0.0;
    for (int j = tid; j < cr; j += NT) {
      double a = 0.0;
      for (int i = 0; i < cl; ++i) a += vin[i] * double(M[(size_t)i * 4 * cr + p * cr + j]);
      vout[j] = a;
      mx = fmax(mx, fabs(a));
    }
    for (int q = 32; q > 0; q >>= 1) mx = fmax(mx, __shfl_xor(mx, q, 64));
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    __syncthreads();
    mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    const double sc = mx > 0.0 ? 1.0 / mx : 1.0;
    acc_log += mx > 0.0 ? log(mx) : 0.0;
    for (int j = tid; j < cr; j += NT) vout[j] *= sc;
    __syncthreads();
    cur = 1 - cur;
  }
  // dot with the right environment at bond l + 1
  const int len = s.dims[l + 1];
  double a = 0.0;
  for (int j = tid; j < len; j += NT) a += v[cur * CHI_LIMIT + j] * ER[(size_t)(l + 1) * s.chi + j];
  a = block_sum(a, red);
  if (tid == 0) {
    const double lr = LR[l + 1];
    out[(size_t)mpo * n_obs + o] = (a / cI) * exp(acc_log + lr - lI);
  }
}

}  // namespace nze

using namespace nze;

// ================================================================ host side

namespace {

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t sites, X, W, norms, perm, sval, dims, scal, ctr, env, envlog, prof, r64, total;
};

// doubles of one slot's refinement workspace (the layout of r64_rows /
// r64_square in the device code)
size_t r64_doubles(size_t chi, size_t m) {
  const size_t rows = chi + BAND, sq = std::max<size_t>(rows * rows, 1088);
  return 2 * rows * m + sq;
}

bool cfg_valid(const mpo_config* c) {
  return c && c->n >= 2 && c->n <= 4096 && c->chi_max >= 1 &&
         c->chi_max <= CHI_LIMIT && c->n_levels >= 1 &&
         (c->precision == NZE_FP64 || c->precision == NZE_MIXED) &&
         c->max_sweeps >= 0 && c->max_sweeps <= MAXSW;
}

Layout layout_of(const mpo_config* c) {
  const size_t L = c->n_levels, n = c->n, chi = c->chi_max;
  const size_t es = c->precision == NZE_FP64 ? 8 : 4;
  const size_t site_cap = chi * 4 * chi, m = 4 * chi;
  Layout o;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t at = off; off += align_up(bytes); return at; };
  o.sites = take(L * n * site_cap * es);
  o.X = take(L * m * m * es);
  o.W = take(L * m * m * es);
  o.norms = take(L * m * 8);
  o.perm = take(L * m * 4);
  o.sval = take(L * m * 8);
  o.dims = take(L * (n + 1) * 4);
  o.scal = take(L * SC_COUNT * 8);
  o.ctr = take(L * CT_COUNT * 4);
  o.env = take(L * 2 * (n + 1) * chi * 8);
  o.envlog = take(L * 2 * (n + 1) * 8);
  o.prof = take(L * PF_N * 8);
  // float64 refinement workspace per level (chi + 16 rows: the kept
  // directions and the polished band below the cut)
  o.r64 = take(L * r64_doubles(chi, m) * 8);
  o.total = off;
  return o;
}

// Launch metadata staging: one device buffer per stream, grown on demand, fed
// from double-buffered pinned host memory.
struct Staging {
  char* dev = nullptr;
  size_t dev_bytes = 0;
  char* host[2] = {nullptr, nullptr};
  size_t host_bytes[2] = {0, 0};
  hipEvent_t copied[2] = {nullptr, nullptr};
  int cur = 0;
};
std::mutex g_stage_mu;
std::map<hipStream_t, Staging*> g_stage;

struct DevInfo {
  int cus = 0;
  int occ[2] = {0, 0};
  int occ_f32x2 = 0;        // float kernel built for two workgroups per CU
  unsigned long long timeout_ticks = 0;
  bool xcd_local = false;   // 8 XCDs with their own L2 (gfx950)
};
std::mutex g_dev_mu;
std::map<int, DevInfo> g_dev;

}  // namespace

struct mpo_handle {
  mpo_config cfg;
  hipStream_t stream;
  char* ws;
  Layout lay;
  int site_cap, m_cap;
  int centre;
  std::vector<Slot> slots;        // host copies, one per level
  int64_t layers;
  bool tuned;                     // cfg.block == 0: launches follow the tuner
};

namespace {

// Tuner records, keyed by (precision, chi cap, MPOs per launch).  The group
// size and the kernel build never change a result (every pair visit computes
// the same numbers whichever workgroup runs it); the cross-block-only
// schedule changes the rotations, so it is fixed per handle at mpo_init.
struct TuneKey {
  int prec, chi, nmpo;
  bool operator<(const TuneKey& o) const {
    if (prec != o.prec) return prec < o.prec;
    if (chi != o.chi) return chi < o.chi;
    return nmpo < o.nmpo;
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, nze_tuning> g_tune;

bool tune_lookup(int prec, int chi, int nmpo, nze_tuning* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(TuneKey{prec, chi, nmpo});
  if (it == g_tune.end()) return false;
  *out = it->second;
  return true;
}

// Per-launch overrides of the automatic rules (0 = automatic).
struct LaunchChoice {
  int group_scale = 0;   // 1: pairs per round; 2: doubled groups
  int kernel = 0;        // 1: one workgroup per CU; 2: two per CU (float)
};

}  // namespace

namespace {

int hip_fail(hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  nze::g_last_error = m;
  return NZE_EHIP;
}
#define HIPCHK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return hip_fail(e_, #x); } while (0)

int dev_info(DevInfo& out) {
  int dev;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto it = g_dev.find(dev);
  if (it != g_dev.end()) { out = it->second; return NZE_OK; }
  DevInfo di;
  HIPCHK(hipDeviceGetAttribute(&di.cus, hipDeviceAttributeMultiprocessorCount, dev));
  int occ = 0;
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_layer_f64, NT, 0));
  di.occ[0] = occ;
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_layer_f32, NT, 0));
  di.occ[1] = occ;
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_layer_f32x2, NT, 0));
  di.occ_f32x2 = occ;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    khz = 100000;
  di.timeout_ticks = (unsigned long long)khz * 1000ull * 4ull;   // 4 s
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  const char* env = std::getenv("NZE_XCD_LOCAL");
  di.xcd_local = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 && di.cus % 8 == 0 &&
                 !(env && env[0] == '0');
  g_dev[dev] = di;
  out = di;
  return NZE_OK;
}

int stage(hipStream_t stream, const void* src, size_t bytes, char** dev_out) {
  Staging* st;
  {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    auto it = g_stage.find(stream);
    if (it == g_stage.end()) {
      st = new Staging();
      g_stage[stream] = st;
    } else {
      st = it->second;
    }
  }
  const int b = st->cur;
  st->cur ^= 1;
  if (st->copied[b]) HIPCHK(hipEventSynchronize(st->copied[b]));
  else HIPCHK(hipEventCreateWithFlags(&st->copied[b], hipEventDisableTiming));
  if (st->host_bytes[b] < bytes) {
    if (st->host[b]) HIPCHK(hipHostFree(st->host[b]));
    const size_t nb = std::max(bytes, (size_t)1 << 20);
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&st->host[b]), nb, hipHostMallocDefault));
    st->host_bytes[b] = nb;
  }
  if (st->dev_bytes < bytes) {
    // the previous launch may still read the old buffer: wait for the stream
    HIPCHK(hipStreamSynchronize(stream));
    if (st->dev) HIPCHK(hipFree(st->dev));
    const size_t nb = std::max(bytes * 2, (size_t)1 << 20);
    HIPCHK(hipMalloc(reinterpret_cast<void**>(&st->dev), nb));
    st->dev_bytes = nb;
  }
  std::memcpy(st->host[b], src, bytes);
  HIPCHK(hipMemcpyAsync(st->dev, st->host[b], bytes, hipMemcpyHostToDevice, stream));
  HIPCHK(hipEventRecord(st->copied[b], stream));
  *dev_out = st->dev;
  return NZE_OK;
}

void fill_defaults(mpo_config& c) {
  const bool f64 = c.precision == NZE_FP64;
  if (c.trunc_tol <= 0) c.trunc_tol = f64 ? 1e-14 : 1e-7;
  if (c.tie_tol <= 0) c.tie_tol = f64 ? 1e-10 : 1e-5;
  if (c.jacobi_tol <= 0) c.jacobi_tol = f64 ? 1e-13 : 3e-7;
  if (c.jacobi_abs <= 0) c.jacobi_abs = f64 ? 1e-15 : 1e-9;
  if (c.max_sweeps <= 0) c.max_sweeps = MAXSW;   // dense near-degenerate spectra can need > 30
  if (c.block <= 0) c.block = BW;
}

// Host-side plan of one layer for one handle: centre moves and gates.
void plan_layer(mpo_handle* h, int n_gates, const int32_t* ls,
                std::vector<Step>& out) {
  if (n_gates == 0) return;
  const bool ltr = (ls[0] % 2) == 0;
  for (int gi = 0; gi < n_gates; ++gi) {
    const int i = ltr ? gi : n_gates - 1 - gi;
    const int k = ls[i];
    const int target = ltr ? k : k + 1;
    while (h->centre < target) { out.push_back({OP_MOVE_LR, h->centre, 0, 0}); h->centre++; }
    while (h->centre > target) { out.push_back({OP_MOVE_RL, h->centre, 0, 0}); h->centre--; }
    out.push_back({ltr ? OP_GATE_LR : OP_GATE_RL, k, i, 0});
    h->centre = ltr ? k + 1 : k;
  }
}

int check_sites(const mpo_handle* h, int n_gates, const int32_t* ls) {
  if (n_gates < 0) return fail(NZE_EINVAL, "n_gates < 0");
  if (n_gates > 0 && !ls) return fail(NZE_EINVAL, "left_site is NULL");
  for (int i = 0; i < n_gates; ++i) {
    if (ls[i] < 0 || ls[i] + 1 >= h->cfg.n) return fail(NZE_EINVAL, "gate outside the chain");
    if (i > 0 && ls[i] - ls[i - 1] < 2) return fail(NZE_EINVAL, "left sites must be increasing and disjoint");
  }
  return NZE_OK;
}

int read_errors(mpo_t* h) {
  const int L = h->cfg.n_levels;
  std::vector<int> ctr((size_t)L * CT_COUNT);
  HIPCHK(hipMemcpyAsync(ctr.data(), h->ws + h->lay.ctr, ctr.size() * 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  int err = 0;
  for (int l = 0; l < L; ++l) err |= ctr[(size_t)l * CT_COUNT + CT_ERR];
  if (err & ERR_ABORT) return fail(NZE_EHIP, "layer kernel aborted at a group barrier (timeout)");
  if (err & ERR_NAN) return fail(NZE_ENUM, "NaN/Inf or zero norm in the state");
  if (err & ERR_NOCONV) return fail(NZE_ENOCONV, "Jacobi SVD hit the sweep cap");
  return NZE_OK;
}

}  // namespace

extern "C" size_t mpo_footprint(const mpo_config* cfg) {
  if (!cfg) return 0;
  mpo_config c = *cfg;
  if (!cfg_valid(&c)) return 0;
  return layout_of(&c).total;
}

extern "C" int mpo_init(mpo_t** out, const mpo_config* cfg,
                        const double* init_sites, void* workspace,
                        size_t ws_bytes, void* stream) {
  if (!out) return fail(NZE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfg_valid(cfg)) return fail(NZE_EINVAL, "invalid mpo_config");
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return fail(NZE_EINVAL, "workspace must be a 256-byte aligned device pointer");
  mpo_config c = *cfg;
  const bool tuned = c.block == 0;
  fill_defaults(c);
  if (c.block != BW) return fail(NZE_EINVAL, "unsupported Jacobi block width (16)");
  nze_tuning tune_rec;
  const bool have_tune = tuned && tune_lookup(c.precision, c.chi_max, c.n_levels, &tune_rec);
  const Layout lay = layout_of(&c);
  if (ws_bytes < lay.total) return fail(NZE_ENOMEM, "workspace smaller than mpo_footprint(cfg)");
  DevInfo di;
  int rc = dev_info(di);
  if (rc) return rc;
  mpo_handle* h = new mpo_handle();
  h->cfg = c;
  h->stream = reinterpret_cast<hipStream_t>(stream);
  h->ws = reinterpret_cast<char*>(workspace);
  h->lay = lay;
  h->site_cap = c.chi_max * 4 * c.chi_max;
  h->m_cap = 4 * c.chi_max;
  h->centre = 0;
  h->layers = 0;
  h->tuned = tuned;
  const size_t es = c.precision == NZE_FP64 ? 8 : 4;
  const int L = c.n_levels, n = c.n;
  for (int l = 0; l < L; ++l) {
    Slot s;
    std::memset(&s, 0, sizeof(s));
    s.sites = h->ws + lay.sites + (size_t)l * n * h->site_cap * es;
    s.dims = reinterpret_cast<int*>(h->ws + lay.dims) + (size_t)l * (n + 1);
    s.scal = reinterpret_cast<double*>(h->ws + lay.scal) + (size_t)l * SC_COUNT;
    s.ctr = reinterpret_cast<int*>(h->ws + lay.ctr) + (size_t)l * CT_COUNT;
    s.X = h->ws + lay.X + (size_t)l * h->m_cap * h->m_cap * es;
    s.W = h->ws + lay.W + (size_t)l * h->m_cap * h->m_cap * es;
    s.norms = reinterpret_cast<double*>(h->ws + lay.norms) + (size_t)l * h->m_cap;
    s.perm = reinterpret_cast<int*>(h->ws + lay.perm) + (size_t)l * h->m_cap;
    s.sval = reinterpret_cast<double*>(h->ws + lay.sval) + (size_t)l * h->m_cap;
    s.n = n;
    s.chi = c.chi_max;
    s.site_cap = h->site_cap;
    s.m_cap = h->m_cap;
    s.tau = c.trunc_tol;
    s.tie = c.tie_tol;
    s.tol_rel = c.jacobi_tol;
    s.tol_abs = c.jacobi_abs;
    s.max_sweeps = c.max_sweeps;
    s.prof = reinterpret_cast<double*>(h->ws + lay.prof) + (size_t)l * PF_N;
    s.R64 = reinterpret_cast<double*>(h->ws + lay.r64) + (size_t)l * r64_doubles(c.chi_max, h->m_cap);
    s.no_acc = 1;
    s.cross_sweeps = have_tune ? tune_rec.cross_sweeps : 8;
    s.cross_min_blocks = have_tune ? tune_rec.cross_min_blocks : 64;
    h->slots.push_back(s);
  }
  std::vector<double> init((size_t)4 * n);
  for (int k = 0; k < n; ++k) {
    const double* src = init_sites ? init_sites + 4 * k : nullptr;
    double v[4] = {1, 0, 0, 1};
    if (src) for (int p = 0; p < 4; ++p) v[p] = src[p];
    if (!(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3] > 0)) {
      delete h;
      return fail(NZE_EINVAL, "zero initial site");
    }
    for (int p = 0; p < 4; ++p) init[4 * k + p] = v[p];
  }
  // metadata: slots then init sites
  std::vector<char> blob(sizeof(Slot) * L + 8 * init.size());
  std::memcpy(blob.data(), h->slots.data(), sizeof(Slot) * L);
  std::memcpy(blob.data() + sizeof(Slot) * L, init.data(), 8 * init.size());
  char* dev;
  rc = stage(h->stream, blob.data(), blob.size(), &dev);
  if (rc) { delete h; return rc; }
  const Slot* dslots = reinterpret_cast<const Slot*>(dev);
  const double* dinit = reinterpret_cast<const double*>(dev + sizeof(Slot) * L);
  if (c.precision == NZE_FP64)
    hipLaunchKernelGGL(k_init<double>, dim3(L), dim3(NT), 0, h->stream, dslots, dinit, n);
  else
    hipLaunchKernelGGL(k_init<float>, dim3(L), dim3(NT), 0, h->stream, dslots, dinit, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { delete h; return hip_fail(e, "k_init launch"); }
  *out = h;
  return NZE_OK;
}

extern "C" void mpo_free(mpo_t* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  delete h;
}

namespace {
int launch_plans(mpo_t* const* hs, int k, const std::vector<std::vector<Step>>& plans,
                 const int32_t* n_gates, const double* const* ptm,
                 const std::vector<int>& saved_centre, const LaunchChoice* forced = nullptr);
}  // namespace

extern "C" int mpo_apply_layer_batch(mpo_t* const* hs, int32_t k,
                                     const int32_t* n_gates,
                                     const int32_t* const* left_site,
                                     const double* const* ptm) {
  if (k <= 0 || !hs || !n_gates || !left_site || !ptm) return fail(NZE_EINVAL, "bad batch");
  const int prec = hs[0]->cfg.precision;
  const hipStream_t stream = hs[0]->stream;
  for (int j = 0; j < k; ++j) {
    if (!hs[j]) return fail(NZE_EINVAL, "NULL handle");
    if (hs[j]->cfg.precision != prec) return fail(NZE_EINVAL, "mixed precisions in one batch");
    if (hs[j]->stream != stream) return fail(NZE_EINVAL, "handles on different streams");
    int rc = check_sites(hs[j], n_gates[j], left_site[j]);
    if (rc) return rc;
    if (n_gates[j] > 0 && !ptm[j]) return fail(NZE_EINVAL, "ptm is NULL");
  }
  // plans (per handle; every level of a handle follows the same plan)
  std::vector<std::vector<Step>> plans(k);
  std::vector<int> saved_centre(k);
  for (int j = 0; j < k; ++j) {
    saved_centre[j] = hs[j]->centre;
    plan_layer(hs[j], n_gates[j], left_site[j], plans[j]);
  }
  int rc = launch_plans(hs, k, plans, n_gates, ptm, saved_centre);
  if (rc == NZE_OK)
    for (int j = 0; j < k; ++j) hs[j]->layers++;
  return rc;
}

namespace {

// One persistent launch running the step lists `plans` (one per handle, all
// levels of a handle alike) of handles on one stream and precision.  On a
// failure before the launch the handles' centres are restored.
int launch_plans(mpo_t* const* hs, int k, const std::vector<std::vector<Step>>& plans,
                 const int32_t* n_gates, const double* const* ptm,
                 const std::vector<int>& saved_centre, const LaunchChoice* forced) {
  const int prec = hs[0]->cfg.precision;
  const hipStream_t stream = hs[0]->stream;
  size_t nsteps = 0, nmpo = 0, nptm = 0;
  for (int j = 0; j < k; ++j) {
    nsteps = std::max(nsteps, plans[j].size());
    nmpo += hs[j]->cfg.n_levels;
    nptm += (size_t)hs[j]->cfg.n_levels * n_gates[j];
  }
  if (nsteps == 0) return NZE_OK;
  auto restore = [&]() { for (int j = 0; j < k; ++j) hs[j]->centre = saved_centre[j]; };
  DevInfo di;
  int rc = dev_info(di);
  if (rc) { restore(); return rc; }
  // Group size of each MPO: the pairs per Jacobi round at its chi cap
  // (m / 32; a pair visit waits for the previous round's visits of its
  // blocks, so more workgroups than pairs do not shorten the chain of rounds,
  // measured).  When the batch asks for more than the resident workgroups,
  // every request is scaled down alike, so that MPOs of different widths keep
  // their relative shares.
  std::vector<int> gm(nmpo);
  {
    size_t m = 0;
    for (int j = 0; j < k; ++j)
      for (int l = 0; l < hs[j]->cfg.n_levels; ++l) gm[m++] = std::max(1, hs[j]->cfg.chi_max / 8);
  }
  long long want_tot = 0;
  for (int x : gm) want_tot += x;
  // the tuner's choice for this batch shape, when every handle follows it
  LaunchChoice ch;
  if (forced) {
    ch = *forced;
  } else {
    bool all_tuned = true, same_chi = true;
    for (int j = 0; j < k; ++j) {
      all_tuned = all_tuned && hs[j]->tuned;
      same_chi = same_chi && hs[j]->cfg.chi_max == hs[0]->cfg.chi_max;
    }
    nze_tuning t;
    if (all_tuned && same_chi && tune_lookup(prec, hs[0]->cfg.chi_max, (int)nmpo, &t)) {
      ch.group_scale = t.group_scale;
      ch.kernel = t.kernel;
    }
  }
  // float batches that ask for more groups than one per CU run the kernel
  // built for two workgroups per CU (independent MPOs then share each CU)
  bool x2 = prec != NZE_FP64 && di.occ_f32x2 >= 2 && want_tot > (long long)di.occ[1] * di.cus;
  if (prec != NZE_FP64 && di.occ_f32x2 >= 2 && ch.kernel) x2 = ch.kernel == 2;
  const int occ = prec == NZE_FP64 ? di.occ[0] : (x2 ? di.occ_f32x2 : di.occ[1]);
  const int resident = std::max(1, occ * di.cus);
  if ((int)nmpo > resident) {
    restore();
    return fail(NZE_EINVAL, "batch has more MPOs than resident workgroups");
  }
  if (want_tot > resident) {
    const double scale = double(resident) / double(want_tot);
    want_tot = 0;
    for (int& x : gm) { x = std::max(1, (int)(x * scale)); want_tot += x; }
    while (want_tot > resident) {            // the max(1, .) clamps can overshoot
      auto it = std::max_element(gm.begin(), gm.end());
      if (*it <= 1) break;
      --*it;
      --want_tot;
    }
  }
  // A batch that asks for at most half of the CUs gets its groups doubled
  // (still one workgroup per CU): consecutive Jacobi rounds then alternate
  // between two sets of workgroups, so a round's visits start on workgroups
  // that are not finishing the round before.  Two such workgroups sharing a
  // CU gain nothing (measured), hence only on idle CUs.
  const bool can_double = want_tot * 2 <= (long long)resident;
  const bool dbl = ch.group_scale ? (ch.group_scale == 2 && can_double)
                                  : (!x2 && want_tot * 2 <= (long long)di.cus && occ == 1);
  if (dbl) {
    for (int& x : gm) x *= 2;
    want_tot *= 2;
  }
  const bool uniform = std::all_of(gm.begin(), gm.end(), [&](int x) { return x == gm[0]; });
  const int G = gm[0];
  // XCD-local groups: every XCD hosts nmpo / 8 whole MPOs (the grid of
  // nmpo * G workgroups is spread evenly over the 8 XCDs)
  int a_xcd = (di.xcd_local && nmpo % 8 == 0 && uniform) ? 1 : 0;
  const int grid = a_xcd ? (int)nmpo * G : (int)want_tot;
  // blob: slots | steps | ptms | bar + abort | workgroup map | group sizes
  const size_t off_steps = align_up(sizeof(Slot) * nmpo);
  const size_t off_ptm = off_steps + align_up(sizeof(Step) * nsteps * nmpo);
  const size_t off_bar = off_ptm + align_up(8 * 256 * std::max<size_t>(nptm, 1));
  const size_t off_map = off_bar + align_up(4 * (nmpo + 10));
  const size_t off_gsz = off_map + align_up(8 * (size_t)grid);
  const size_t total = off_gsz + align_up(4 * nmpo);
  std::vector<char> blob(total, 0);
  {
    int* map = reinterpret_cast<int*>(blob.data() + off_map);
    int* gsz = reinterpret_cast<int*>(blob.data() + off_gsz);
    int b = 0;
    for (size_t m = 0; m < nmpo; ++m) {
      gsz[m] = gm[m];
      for (int g = 0; g < gm[m] && !a_xcd; ++g, ++b) { map[2 * b] = (int)m; map[2 * b + 1] = g; }
    }
  }
  Slot* bslots = reinterpret_cast<Slot*>(blob.data());
  Step* bsteps = reinterpret_cast<Step*>(blob.data() + off_steps);
  double* bptm = reinterpret_cast<double*>(blob.data() + off_ptm);
  size_t mpo0 = 0, ptm0 = 0;
  for (int j = 0; j < k; ++j) {
    mpo_t* h = hs[j];
    const int L = h->cfg.n_levels, ng = n_gates[j];
    for (int l = 0; l < L; ++l) {
      bslots[mpo0 + l] = h->slots[l];
      for (size_t st = 0; st < nsteps; ++st) {
        Step s = st < plans[j].size() ? plans[j][st] : Step{OP_NONE, 0, 0, 0};
        if (s.op == OP_GATE_LR || s.op == OP_GATE_RL) s.ptm = (int)(ptm0 + (size_t)l * ng + s.ptm);
        bsteps[st * nmpo + mpo0 + l] = s;
      }
    }
    if (ng > 0) std::memcpy(bptm + ptm0 * 256, ptm[j], sizeof(double) * 256 * L * ng);
    mpo0 += L;
    ptm0 += (size_t)L * ng;
  }
  char* dev;
  rc = stage(stream, blob.data(), blob.size(), &dev);
  if (rc) {
    for (int j = 0; j < k; ++j) hs[j]->centre = saved_centre[j];
    return rc;
  }
  int* dbar = reinterpret_cast<int*>(dev + off_bar);
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(256), 0, stream, dbar, (int)nmpo + 10, 0);
  const Slot* a_slots = reinterpret_cast<const Slot*>(dev);
  const Step* a_steps = reinterpret_cast<const Step*>(dev + off_steps);
  const double* a_ptm = reinterpret_cast<const double*>(dev + off_ptm);
  int a_nsteps = (int)nsteps, a_nmpo = (int)nmpo, a_G = G;
  int* a_bar = dbar;                 // nmpo group counters, 8 tickets, census
  int* a_abort = dbar + nmpo + 9;
  unsigned long long a_to = di.timeout_ticks;
  const int* a_map = reinterpret_cast<const int*>(dev + off_map);
  const int* a_gsz = reinterpret_cast<const int*>(dev + off_gsz);
  void* args[] = {&a_slots, &a_steps, &a_ptm, &a_nsteps, &a_nmpo, &a_G, &a_bar, &a_abort,
                  &a_to, &a_xcd, &a_map, &a_gsz};
  const void* fn = prec == NZE_FP64 ? reinterpret_cast<const void*>(&k_layer_f64)
                   : x2 ? reinterpret_cast<const void*>(&k_layer_f32x2)
                        : reinterpret_cast<const void*>(&k_layer_f32);
  const hipError_t le = hipLaunchCooperativeKernel(fn, dim3((unsigned)grid), dim3(NT), args, 0, stream);
  if (le != hipSuccess) {
    restore();
    return hip_fail(le, "hipLaunchCooperativeKernel (layer)");
  }
  return NZE_OK;
}

}  // namespace

extern "C" int mpo_apply_layer(mpo_t* h, int32_t n_gates,
                               const int32_t* left_site, const double* ptm) {
  if (!h) return fail(NZE_EINVAL, "NULL handle");
  return mpo_apply_layer_batch(&h, 1, &n_gates, &left_site, &ptm);
}

extern "C" int mpo_sync(mpo_t* h) {
  if (!h) return fail(NZE_EINVAL, "NULL handle");
  return read_errors(h);
}

extern "C" int mpo_expect(mpo_t* h, int32_t n_obs, const uint8_t* paulis,
                          double* values, double* fidelity, double* trace) {
  if (!h) return fail(NZE_EINVAL, "NULL handle");
  if (n_obs < 0 || (n_obs > 0 && (!paulis || !values))) return fail(NZE_EINVAL, "bad observables");
  const int L = h->cfg.n_levels, n = h->cfg.n;
  int rc = read_errors(h);
  if (rc) return rc;
  for (size_t i = 0; i < (size_t)n_obs * n; ++i)
    if (paulis[i] > 3) return fail(NZE_EINVAL, "Pauli code > 3");
  // slots + spans + strings staged together
  std::vector<int> span(2 * std::max(n_obs, 1), -1);
  for (int o = 0; o < n_obs; ++o) {
    int f = -1, l = -1;
    for (int q = 0; q < n; ++q)
      if (paulis[(size_t)o * n + q]) { if (f < 0) f = q; l = q; }
    span[2 * o] = f;
    span[2 * o + 1] = l;
  }
  const size_t off_span = align_up(sizeof(Slot) * L);
  const size_t off_str = off_span + align_up(span.size() * 4);
  const size_t off_out = off_str + align_up((size_t)std::max(n_obs, 1) * n);
  const size_t total = off_out + align_up(8 * (size_t)L * std::max(n_obs, 1));
  std::vector<char> blob(total, 0);
  std::memcpy(blob.data(), h->slots.data(), sizeof(Slot) * L);
  std::memcpy(blob.data() + off_span, span.data(), span.size() * 4);
  if (n_obs) std::memcpy(blob.data() + off_str, paulis, (size_t)n_obs * n);
  char* dev;
  rc = stage(h->stream, blob.data(), blob.size(), &dev);
  if (rc) return rc;
  const Slot* dslots = reinterpret_cast<const Slot*>(dev);
  double* env = reinterpret_cast<double*>(h->ws + h->lay.env);
  double* lg = reinterpret_cast<double*>(h->ws + h->lay.envlog);
  const int env_stride = (n + 1) * h->cfg.chi_max;
  const bool f64 = h->cfg.precision == NZE_FP64;
  if (f64) hipLaunchKernelGGL(k_env<double>, dim3(L, 2), dim3(NT), 0, h->stream, dslots, env, lg, env_stride);
  else hipLaunchKernelGGL(k_env<float>, dim3(L, 2), dim3(NT), 0, h->stream, dslots, env, lg, env_stride);
  HIPCHK(hipGetLastError());
  double* dout = reinterpret_cast<double*>(dev + off_out);
  if (n_obs > 0) {
    const uint8_t* dstr = reinterpret_cast<const uint8_t*>(dev + off_str);
    const int* dspan = reinterpret_cast<const int*>(dev + off_span);
    if (f64) hipLaunchKernelGGL(k_obs<double>, dim3(n_obs, L), dim3(NT), 0, h->stream, dslots, env, lg, env_stride, dstr, dspan, n_obs, dout);
    else hipLaunchKernelGGL(k_obs<float>, dim3(n_obs, L), dim3(NT), 0, h->stream, dslots, env, lg, env_stride, dstr, dspan, n_obs, dout);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(values, dout, 8 * (size_t)L * n_obs, hipMemcpyDeviceToHost, h->stream));
  }
  std::vector<double> scal((size_t)L * SC_COUNT);
  HIPCHK(hipMemcpyAsync(scal.data(), h->ws + h->lay.scal, scal.size() * 8, hipMemcpyDeviceToHost, h->stream));
  std::vector<double> cI(L), lI(L);
  for (int l = 0; l < L; ++l) {
    HIPCHK(hipMemcpyAsync(&cI[l], env + (size_t)(l * 2) * env_stride + (size_t)n * h->cfg.chi_max, 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(&lI[l], lg + (size_t)(l * 2) * (n + 1) + n, 8, hipMemcpyDeviceToHost, h->stream));
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  bool finite = true;
  for (int l = 0; l < L; ++l) {
    if (fidelity) fidelity[l] = scal[(size_t)l * SC_COUNT + SC_FID];
    if (trace) trace[l] = cI[l] * std::exp(lI[l] + scal[(size_t)l * SC_COUNT + SC_LOG]);
    // <P> = c_P / c_I is undefined when the truncations removed the identity
    // string (c_I = 0); the outputs are still written
    if (!(cI[l] != 0.0) || !std::isfinite(cI[l])) finite = false;
    for (int o = 0; o < n_obs; ++o)
      if (!std::isfinite(values[(size_t)l * n_obs + o])) finite = false;
  }
  if (!finite) return fail(NZE_ENUM, "readout not finite: the trace c_I of a level is zero or not finite");
  return NZE_OK;
}

extern "C" int mpo_stats(mpo_t* h, nze_stats* stats, int32_t* bonds) {
  if (!h || !stats) return fail(NZE_EINVAL, "bad arguments");
  const int L = h->cfg.n_levels, n = h->cfg.n;
  std::vector<double> scal((size_t)L * SC_COUNT);
  std::vector<int> ctr((size_t)L * CT_COUNT), dims((size_t)L * (n + 1));
  HIPCHK(hipMemcpyAsync(scal.data(), h->ws + h->lay.scal, scal.size() * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(ctr.data(), h->ws + h->lay.ctr, ctr.size() * 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(dims.data(), h->ws + h->lay.dims, dims.size() * 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  for (int l = 0; l < L; ++l) {
    nze_stats& s = stats[l];
    const double* sc = &scal[(size_t)l * SC_COUNT];
    const int* ct = &ctr[(size_t)l * CT_COUNT];
    s.fidelity = sc[SC_FID];
    s.log_scale = sc[SC_LOG];
    s.max_discarded = sc[SC_MAXDISC];
    s.min_cut_gap = sc[SC_MINGAP];
    s.max_sweeps = ct[CT_MAXSW];
    s.updates = ct[CT_UPD];
    s.sweeps_total = ct[CT_SWTOT];
    s.flops = sc[SC_FLOPS];
    s.cap_hits = ct[CT_CAPHIT];
    s.cap_offdiag = sc[SC_CAPQ];
    s.ns_scaled = ct[CT_NSFB];
    int mb = 0;
    for (int b = 1; b < n; ++b) {
      mb = std::max(mb, dims[(size_t)l * (n + 1) + b]);
      if (bonds) bonds[(size_t)l * (n - 1) + b - 1] = dims[(size_t)l * (n + 1) + b];
    }
    s.max_bond = mb;
  }
  return read_errors(h);
}

extern "C" int mpo_profile(mpo_t* h, double* ms_out) {
  if (!h || !ms_out) return fail(NZE_EINVAL, "bad arguments");
  const int L = h->cfg.n_levels;
  std::vector<double> t((size_t)L * PF_N);
  HIPCHK(hipMemcpyAsync(t.data(), h->ws + h->lay.prof, t.size() * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  int dev, khz = 100000;
  HIPCHK(hipGetDevice(&dev));
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
  for (size_t i = 0; i < t.size(); ++i) {
    const int slot = (int)(i % PF_N);
    ms_out[i] = (slot == PF_PAIRS) ? t[i] : t[i] / khz;
  }
  return NZE_OK;
}

extern "C" int mpo_bond_spectrum(mpo_t* h, int32_t lv, int32_t l, double* s_out,
                                 int32_t cap, int32_t* count) {
  if (!h) return fail(NZE_EINVAL, "NULL handle");
  const int n = h->cfg.n;
  if (lv < 0 || lv >= h->cfg.n_levels || l < 0 || l + 1 >= n || !s_out || cap < 1 || !count)
    return fail(NZE_EINVAL, "bad bond spectrum arguments");
  int rc = read_errors(h);
  if (rc) return rc;
  // centre to l, then one more left-to-right move: its SVD is the bond's
  std::vector<std::vector<Step>> plans(1);
  std::vector<int> saved_centre{h->centre};
  while (h->centre < l) { plans[0].push_back({OP_MOVE_LR, h->centre, 0, 0}); h->centre++; }
  while (h->centre > l) { plans[0].push_back({OP_MOVE_RL, h->centre, 0, 0}); h->centre--; }
  plans[0].push_back({OP_MOVE_LR, l, 0, 0});
  h->centre = l + 1;
  const int32_t ng = 0;
  const double* no_ptm = nullptr;
  rc = launch_plans(&h, 1, plans, &ng, &no_ptm, saved_centre);
  if (rc) return rc;
  rc = read_errors(h);
  if (rc) return rc;
  int r = 0;
  const Slot& s = h->slots[lv];
  HIPCHK(hipMemcpyAsync(&r, s.ctr + CT_RANK, 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  const int m = std::min(r, (int)cap);
  HIPCHK(hipMemcpyAsync(s_out, s.sval, (size_t)m * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  *count = r;
  return NZE_OK;
}

// ------------------------------------------------------------- tuner

namespace nze {

__device__ inline uint64_t mix64(uint64_t z) {
  // splitmix64 finaliser (Steele, Lea, Flood 2014)
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Synthetic two-site blocks for the tuner: X[i][j] = d_i z_ij with standard
// normal z (Box-Muller on counter-based uniforms) and row scales d_i falling
// over four decades, a spectrum graded like that of a saturated update.
template <typename T>
__global__ void k_fill_graded(const Slot* slots, int R, int C, uint64_t seed) {
  const Slot s = slots[blockIdx.y];
  T* X = reinterpret_cast<T*>(s.X);
  const size_t total = (size_t)R * C;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const uint64_t h1 = mix64(seed ^ (2 * e + 1) ^ ((uint64_t)blockIdx.y << 44));
    const uint64_t h2 = mix64(h1 ^ 0xD1B54A32D192ED03ull);
    const double u1 = ((double)(h1 >> 11) + 0.5) * 0x1p-53;
    const double u2 = (double)(h2 >> 11) * 0x1p-53;
    const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    const int i = (int)(e / C);
    X[e] = T(z * exp(-9.210340371976184 * i / R));   // 10^(-4 i / R)
  }
}

}  // namespace nze

extern "C" size_t nze_tune_footprint(int32_t chi, int32_t precision, int32_t n_mpos) {
  mpo_config c{};
  c.n = 2;
  c.chi_max = chi;
  c.n_levels = n_mpos;
  c.precision = precision;
  return mpo_footprint(&c);
}

extern "C" int nze_tune(int32_t chi, int32_t precision, int32_t n_mpos, void* workspace,
                        size_t ws_bytes, void* stream, nze_tuning* best) {
  if (!best || chi < 4 || chi > CHI_LIMIT || n_mpos < 1 ||
      (precision != NZE_FP64 && precision != NZE_MIXED))
    return fail(NZE_EINVAL, "bad tuning arguments");
  mpo_config c{};
  c.n = 2;
  c.chi_max = chi;
  c.n_levels = n_mpos;
  c.precision = precision;
  c.block = BW;
  mpo_t* h = nullptr;
  int rc = mpo_init(&h, &c, nullptr, workspace, ws_bytes, stream);
  if (rc) return rc;
  DevInfo di;
  rc = dev_info(di);
  if (rc) { mpo_free(h); return rc; }
  const int m = 4 * chi, nb = (m + BW - 1) / BW;
  std::vector<int> kernels{1};
  if (precision == NZE_MIXED && di.occ_f32x2 >= 2) kernels.push_back(2);
  std::vector<std::pair<int, int>> cross{{0, 64}};
  if (nb >= 16) { cross.push_back({4, nb}); cross.push_back({8, nb}); }
  if (nb >= 64) cross.push_back({8, 64});
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  std::vector<std::vector<Step>> plans{{Step{OP_JACOBI, m, m, 0}}};
  const int32_t ng = 0;
  const double* no_ptm = nullptr;
  std::vector<int> centre{h->centre};
  const hipStream_t st = h->stream;
  nze_tuning top{};
  top.ms_per_svd = 1e300;
  for (int kern : kernels)
    for (int scale = 1; scale <= 2; ++scale)
      for (const auto& cr : cross) {
        for (Slot& sl : h->slots) { sl.cross_sweeps = cr.first; sl.cross_min_blocks = cr.second; }
        LaunchChoice ch;
        ch.group_scale = scale;
        ch.kernel = kern;
        float best_ms = 1e30f;
        for (int rep = 0; rep < 2 && !rc; ++rep) {
          // the slots live in the launch metadata; a separate staging copy
          // feeds the fill kernel
          char* dslots = nullptr;
          rc = stage(st, h->slots.data(), sizeof(Slot) * h->slots.size(), &dslots);
          if (rc) break;
          const Slot* ds = reinterpret_cast<const Slot*>(dslots);
          if (precision == NZE_FP64)
            hipLaunchKernelGGL(k_fill_graded<double>, dim3(256, n_mpos), dim3(256), 0, st, ds, m, m, 12345ull);
          else
            hipLaunchKernelGGL(k_fill_graded<float>, dim3(256, n_mpos), dim3(256), 0, st, ds, m, m, 12345ull);
          if (hipGetLastError() != hipSuccess) { rc = fail(NZE_EHIP, "tuner fill launch"); break; }
          if (hipEventRecord(e0, st) != hipSuccess) { rc = fail(NZE_EHIP, "event"); break; }
          rc = launch_plans(&h, 1, plans, &ng, &no_ptm, centre, &ch);
          if (rc) break;
          if (hipEventRecord(e1, st) != hipSuccess) { rc = fail(NZE_EHIP, "event"); break; }
          rc = read_errors(h);
          if (rc) break;
          float ms = 0.f;
          if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = fail(NZE_EHIP, "event"); break; }
          best_ms = std::min(best_ms, ms);
        }
        if (rc) break;
        const double per = best_ms / n_mpos;
        // a candidate must be 2 % faster than the one before it to replace it
        if (per < 0.98 * top.ms_per_svd) {
          top.block = BW;
          top.group_scale = scale;
          top.kernel = kern;
          top.cross_sweeps = cr.first;
          top.cross_min_blocks = cr.second;
          top.ms_per_svd = per;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  mpo_free(h);
  if (rc) return rc;
  *best = top;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[TuneKey{precision, chi, n_mpos}] = top;
  return NZE_OK;
}

extern "C" int nze_tuning_get(int32_t chi, int32_t precision, int32_t n_mpos, nze_tuning* out) {
  if (!out) return fail(NZE_EINVAL, "NULL output");
  if (!tune_lookup(precision, chi, n_mpos, out)) return fail(NZE_EINVAL, "no tuning record for this shape");
  return NZE_OK;
}

extern "C" int nze_tuning_set(int32_t chi, int32_t precision, int32_t n_mpos, const nze_tuning* t) {
  if (!t || t->block != BW || (t->group_scale != 1 && t->group_scale != 2) ||
      (t->kernel != 1 && t->kernel != 2) || t->cross_sweeps < 0 || t->cross_sweeps > MAXSW ||
      t->cross_min_blocks < 1)
    return fail(NZE_EINVAL, "bad tuning record");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[TuneKey{precision, chi, n_mpos}] = *t;
  return NZE_OK;
}

// ---------------------------------------------------- MPO overlaps

namespace nze {

// C (M x N, float64, row-major, ldc) = op(A) B with float64 accumulation:
// op(A)[m][k] = A[m * lda + k] (trans_a == 0) or A[k * lda + m]; B[k * ldb + n].
// 16 x 16 output tiles, K staged through LDS in chunks of 16.
template <typename TA, typename TB>
__global__ __launch_bounds__(256) void k_gemm_acc64(const TA* A, int lda, int trans_a,
                                                    const TB* B, int ldb, double* C,
                                                    int ldc, int M, int N, int K) {
  __shared__ double As[16][17];
  __shared__ double Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m = blockIdx.y * 16 + ty, n = blockIdx.x * 16 + tx;
  double acc = 0.0;
  for (int k0 = 0; k0 < K; k0 += 16) {
    const int ka = k0 + tx, kb = k0 + ty;
    const int am = blockIdx.y * 16 + ty;
    double av = 0.0;
    if (am < M && ka < K)
      av = double(trans_a ? A[(size_t)ka * lda + am] : A[(size_t)am * lda + ka]);
    As[ty][tx] = av;
    Bs[ty][tx] = (kb < K && n < N) ? double(B[(size_t)kb * ldb + n]) : 0.0;
    __syncthreads();
    for (int kk = 0; kk < 16; ++kk) acc = fma(As[ty][kk], Bs[kk][tx], acc);
    __syncthreads();
  }
  if (m < M && n < N) C[(size_t)m * ldc + n] = acc;
}

template <typename TA, typename TB>
void overlap_site(const TA* A, int ca_l, int ca_r, const TB* B, int cb_l, int cb_r,
                  const double* E, double* Y, double* E2, hipStream_t st) {
  // Y (ca_l x 4 cb_r) = E (ca_l x cb_l) B (cb_l x 4 cb_r)
  dim3 g1((4 * cb_r + 15) / 16, (ca_l + 15) / 16);
  hipLaunchKernelGGL((k_gemm_acc64<double, TB>), g1, dim3(256), 0, st, E, cb_l, 0, B,
                     4 * cb_r, Y, 4 * cb_r, ca_l, 4 * cb_r, cb_l);
  // E2 (ca_r x cb_r) = A^T Y with A as (4 ca_l) x ca_r and Y as (4 ca_l) x cb_r
  dim3 g2((cb_r + 15) / 16, (ca_r + 15) / 16);
  hipLaunchKernelGGL((k_gemm_acc64<TA, double>), g2, dim3(256), 0, st, A, ca_r, 1, Y,
                     cb_r, E2, cb_r, ca_r, cb_r, 4 * ca_l);
}

}  // namespace nze

namespace {

// <<a_la | b_lb>> of the stored (normalised-site) MPOs, contracted site by
// site with float64 environments in the scratch buffers E0, E1 (>= chi_a
// chi_b doubles each) and Y (>= 4 chi_a chi_b doubles).
int overlap_raw(mpo_t* a, int la, mpo_t* b, int lb, double* E0, double* E1, double* Y,
                hipStream_t st, double* out) {
  const int n = a->cfg.n;
  std::vector<int> da(n + 1), db(n + 1);
  HIPCHK(hipMemcpyAsync(da.data(), a->slots[la].dims, 4 * (n + 1), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(db.data(), b->slots[lb].dims, 4 * (n + 1), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double one = 1.0;
  HIPCHK(hipMemcpyAsync(E0, &one, 8, hipMemcpyHostToDevice, st));
  const bool fa = a->cfg.precision == NZE_FP64, fb = b->cfg.precision == NZE_FP64;
  const size_t esa = fa ? 8 : 4, esb = fb ? 8 : 4;
  for (int k = 0; k < n; ++k) {
    const char* A = reinterpret_cast<const char*>(a->slots[la].sites) + (size_t)k * a->site_cap * esa;
    const char* B = reinterpret_cast<const char*>(b->slots[lb].sites) + (size_t)k * b->site_cap * esb;
    if (fa && fb)
      overlap_site(reinterpret_cast<const double*>(A), da[k], da[k + 1], reinterpret_cast<const double*>(B), db[k], db[k + 1], E0, Y, E1, st);
    else if (fa)
      overlap_site(reinterpret_cast<const double*>(A), da[k], da[k + 1], reinterpret_cast<const float*>(B), db[k], db[k + 1], E0, Y, E1, st);
    else if (fb)
      overlap_site(reinterpret_cast<const float*>(A), da[k], da[k + 1], reinterpret_cast<const double*>(B), db[k], db[k + 1], E0, Y, E1, st);
    else
      overlap_site(reinterpret_cast<const float*>(A), da[k], da[k + 1], reinterpret_cast<const float*>(B), db[k], db[k + 1], E0, Y, E1, st);
    HIPCHK(hipGetLastError());
    std::swap(E0, E1);
  }
  HIPCHK(hipMemcpyAsync(out, E0, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return NZE_OK;
}

}  // namespace

extern "C" int mpo_overlap(mpo_t* a, int32_t la, mpo_t* b, int32_t lb,
                           double* fidelity, double* overlap) {
  if (!a || !b || !fidelity) return fail(NZE_EINVAL, "bad arguments");
  if (a->cfg.n != b->cfg.n) return fail(NZE_EINVAL, "MPOs of different lengths");
  if (la < 0 || la >= a->cfg.n_levels || lb < 0 || lb >= b->cfg.n_levels)
    return fail(NZE_EINVAL, "bad level");
  int rc = read_errors(a);
  if (rc) return rc;
  if (b != a) {
    rc = read_errors(b);
    if (rc) return rc;
  }
  // scratch: the two-site block and its copy (W) of the handle with the larger
  // chi cap, idle between layer launches (both streams were synchronised)
  mpo_t* s = b->cfg.chi_max >= a->cfg.chi_max ? b : a;
  const size_t es = s->cfg.precision == NZE_FP64 ? 8 : 4;
  const size_t ca = a->cfg.chi_max, cb = b->cfg.chi_max;
  const size_t cmax = std::max(ca, cb);
  const size_t blk = (size_t)s->m_cap * s->m_cap * es;          // bytes of X (= of W)
  // E0 and E1 (cmax^2 doubles each) in X, Y (4 cmax^2 doubles) in W:
  // 16 cmax^2 es >= 16 cmax^2 * 4 bytes >= what both need
  if (2 * cmax * cmax * 8 > blk || 4 * cmax * cmax * 8 > blk)
    return fail(NZE_EINVAL, "overlap scratch too small");
  double* E0 = reinterpret_cast<double*>(s->slots[0].X);
  double* E1 = E0 + cmax * cmax;
  double* Y = reinterpret_cast<double*>(s->slots[0].W);
  const hipStream_t st = s->stream;
  double ab = 0.0, aa = 0.0, bb = 0.0;
  rc = overlap_raw(a, la, b, lb, E0, E1, Y, st, &ab);
  if (!rc) rc = overlap_raw(a, la, a, la, E0, E1, Y, st, &aa);
  if (!rc) rc = overlap_raw(b, lb, b, lb, E0, E1, Y, st, &bb);
  if (rc) return rc;
  if (!(aa > 0.0) || !(bb > 0.0) || !std::isfinite(ab)) return fail(NZE_ENUM, "zero or non-finite norm");
  const double c = ab / std::sqrt(aa * bb);
  *fidelity = c * c;
  if (overlap) *overlap = c;
  return NZE_OK;
}

extern "C" int mpo_bond_entropy(mpo_t* h, int32_t lv, int32_t l, double* entropy) {
  if (!h || !entropy) return fail(NZE_EINVAL, "bad arguments");
  std::vector<double> sv((size_t)4 * h->cfg.chi_max);
  int32_t count = 0;
  int rc = mpo_bond_spectrum(h, lv, l, sv.data(), (int32_t)sv.size(), &count);
  if (rc) return rc;
  const int k = std::min<int>(count, (int)sv.size());
  // S_l = -sum_i p_i ln p_i with p_i = s_i^2 / sum_j s_j^2 (natural log)
  double tot = 0.0;
  for (int i = 0; i < k; ++i) tot += sv[i] * sv[i];
  if (!(tot > 0.0) || !std::isfinite(tot)) return fail(NZE_ENUM, "bond spectrum is zero or not finite");
  double e = 0.0;
  for (int i = 0; i < k; ++i) {
    const double p = sv[i] * sv[i] / tot;
    if (p > 0.0) e -= p * std::log(p);
  }
  *entropy = e;
  return NZE_OK;
}

// ------------------------------------------------------ kernel-level hooks

namespace nze {

template <typename T>
__global__ __launch_bounds__(NT) void k_theta_only(Slot s, const double* R,
                                                   int ltr, int G, int* bar,
                                                   int* abort_flag,
                                                   unsigned long long to) {
  __shared__ double smem[SMEM_DOUBLES];
  phase_theta<T>(s, 0, ltr != 0, R, blockIdx.x, G, smem);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_rowortho(Slot s, int R, int C, int G,
                                                 int* bar, int* abort_flag,
                                                 unsigned long long to) {
  __shared__ double smem[SMEM_DOUBLES];
  __shared__ int sflag[2];
  Group grp{bar, abort_flag, G, 0, to, sflag, 0};
  const int g = blockIdx.x;
  T* X = reinterpret_cast<T*>(s.X);
  T* W = reinterpret_cast<T*>(s.W);
  set_identity(W, R, g, G);
  if (!group_sync(grp)) { if (g == 0 && threadIdx.x == 0) atomicOr(&s.ctr[CT_ERR], ERR_ABORT); return; }
  if (!phase_jacobi<T>(s, X, W, R, C, g, G, grp, smem)) { if (g == 0 && threadIdx.x == 0) atomicOr(&s.ctr[CT_ERR], ERR_ABORT); return; }
  phase_norms<T>(s, X, R, C, g, G);
}

}  // namespace nze

namespace {

struct HookScratch {
  char* dev = nullptr;   // scal | ctr | bar | abort | norms | ptm
};
std::mutex g_hook_mu;
HookScratch g_hook;
constexpr size_t HOOK_BYTES = 1 << 16;

int hook_scratch(char** out) {
  std::lock_guard<std::mutex> lk(g_hook_mu);
  if (!g_hook.dev) HIPCHK(hipMalloc(reinterpret_cast<void**>(&g_hook.dev), HOOK_BYTES));
  *out = g_hook.dev;
  return NZE_OK;
}

}  // namespace

extern "C" void nze_shutdown(void) {
  {
    std::lock_guard<std::mutex> a(g_stage_mu), b(g_hook_mu);
    if (g_stage.empty() && !g_hook.dev) return;   // nothing was allocated
  }
  // wait for every queued use of these buffers first
  (void)hipDeviceSynchronize();
  {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    for (auto& kv : g_stage) {
      Staging* st = kv.second;
      for (int b = 0; b < 2; ++b) {
        if (st->copied[b]) (void)hipEventDestroy(st->copied[b]);
        if (st->host[b]) (void)hipHostFree(st->host[b]);
      }
      if (st->dev) (void)hipFree(st->dev);
      delete st;
    }
    g_stage.clear();
  }
  std::lock_guard<std::mutex> lk(g_hook_mu);
  if (g_hook.dev) (void)hipFree(g_hook.dev);
  g_hook.dev = nullptr;
}

extern "C" int nze_kernel_theta(int32_t precision, int32_t cl, int32_t cm,
                                int32_t cr, const void* A, const void* B,
                                const double* ptm, int32_t ltr, void* X,
                                void* stream) {
  if (precision != NZE_FP64 && precision != NZE_MIXED) return fail(NZE_EINVAL, "precision");
  if (cl < 1 || cm < 1 || cr < 1 || cl > CHI_LIMIT || cm > CHI_LIMIT || cr > CHI_LIMIT || !A || !B || !ptm || !X)
    return fail(NZE_EINVAL, "bad theta arguments");
  const size_t es = precision == NZE_FP64 ? 8 : 4;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* scr;
  int rc = hook_scratch(&scr);
  if (rc) return rc;
  // sites: two consecutive slots; the hook copies A and B into a temporary
  const size_t cap = (size_t)std::max(cl, cr) * 4 * cm + (size_t)cm * 4 * std::max(cl, cr);
  char* tmp;
  HIPCHK(hipMalloc(reinterpret_cast<void**>(&tmp), 2 * cap * es + 4096));
  int dims[3] = {cl, cm, cr};
  int* ddims = reinterpret_cast<int*>(tmp + 2 * cap * es);
  HIPCHK(hipMemcpyAsync(ddims, dims, sizeof(dims), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(tmp, A, (size_t)4 * cl * cm * es, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(tmp + cap * es, B, (size_t)cm * 4 * cr * es, hipMemcpyDeviceToDevice, st));
  double* dptm = reinterpret_cast<double*>(scr + 4096);
  HIPCHK(hipMemcpyAsync(dptm, ptm, 256 * 8, hipMemcpyHostToDevice, st));
  double* dscal = reinterpret_cast<double*>(scr);
  HIPCHK(hipMemsetAsync(dscal, 0, 64, st));
  Slot s;
  std::memset(&s, 0, sizeof(s));
  s.sites = tmp;
  s.site_cap = (int)cap;
  s.dims = ddims;
  s.scal = dscal;
  s.X = X;
  // W = I is written too: point it at a scratch matrix of the right size
  const int Rr = ltr ? 4 * cl : 4 * cr;
  char* wtmp;
  HIPCHK(hipMalloc(reinterpret_cast<void**>(&wtmp), (size_t)Rr * Rr * es));
  s.W = wtmp;
  const int G = 64;
  if (precision == NZE_FP64)
    hipLaunchKernelGGL(k_theta_only<double>, dim3(G), dim3(NT), 0, st, s, dptm, ltr, G, nullptr, nullptr, 0ull);
  else
    hipLaunchKernelGGL(k_theta_only<float>, dim3(G), dim3(NT), 0, st, s, dptm, ltr, G, nullptr, nullptr, 0ull);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipFree(wtmp));
  HIPCHK(hipFree(tmp));
  return NZE_OK;
}

namespace {

// The block one-sided Jacobi of the layer kernel on caller buffers, with its
// counters, barrier words, norms and row order in the 64 KiB scratch `scr`
// (device memory; its first 8 KiB are cleared by a fill kernel here).
int rowortho_impl(int32_t precision, int32_t R, int32_t C, void* X, void* W,
                  double tol_rel, double tol_abs, int32_t max_sweeps, double* norms,
                  int32_t* sweeps, hipStream_t st, char* scr) {
  DevInfo di;
  int rc = dev_info(di);
  if (rc) return rc;
  double* dscal = reinterpret_cast<double*>(scr);
  int* dctr = reinterpret_cast<int*>(scr + 256);
  int* dbar = reinterpret_cast<int*>(scr + 2048);
  double* dnorm = reinterpret_cast<double*>(scr + 8192);               // R <= 2048 doubles
  int* dperm = reinterpret_cast<int*>(scr + 8192 + 8 * 4 * CHI_LIMIT);   // R ints (row order)
  static_assert(8192 + 12 * 4 * CHI_LIMIT <= HOOK_BYTES, "hook scratch too small");
  static_assert(256 + 4 * CT_COUNT <= 2048, "hook counters overlap the barrier");
  hipLaunchKernelGGL(k_fill_int, dim3(8), dim3(256), 0, st, reinterpret_cast<int*>(scr), 8192 / 4, 0);
  HIPCHK(hipGetLastError());
  Slot s;
  std::memset(&s, 0, sizeof(s));
  s.scal = dscal;
  s.ctr = dctr;
  s.X = X;
  s.W = W;
  s.norms = dnorm;
  s.perm = dperm;
  s.tol_rel = tol_rel;
  s.tol_abs = tol_abs;
  s.max_sweeps = max_sweeps;
  s.cross_sweeps = 8;
  s.cross_min_blocks = 64;
  const int occ = di.occ[precision == NZE_FP64 ? 0 : 1];
  const int G = std::max(1, std::min((R + 31) / 32, occ * di.cus));
  int a_R = R, a_C = C, a_G = G;
  int* a_bar = dbar;
  int* a_abort = dbar + 1;
  unsigned long long a_to = di.timeout_ticks;
  void* args[] = {&s, &a_R, &a_C, &a_G, &a_bar, &a_abort, &a_to};
  const void* fn = precision == NZE_FP64 ? reinterpret_cast<const void*>(&k_rowortho<double>)
                                         : reinterpret_cast<const void*>(&k_rowortho<float>);
  HIPCHK(hipLaunchCooperativeKernel(fn, dim3(G), dim3(NT), args, 0, st));
  int ctr[CT_COUNT];
  HIPCHK(hipMemcpyAsync(ctr, dctr, sizeof(ctr), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(norms, dnorm, (size_t)R * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (sweeps) *sweeps = ctr[CT_SWTOT];
  if (ctr[CT_ERR] & ERR_ABORT) return fail(NZE_EHIP, "rowortho aborted at a barrier");
  if (ctr[CT_ERR] & ERR_NOCONV) return fail(NZE_ENOCONV, "rowortho hit the sweep cap");
  return NZE_OK;
}

int rowortho_args(int32_t precision, int32_t R, int32_t C, const void* X, const void* W,
                  const double* norms, int32_t max_sweeps) {
  if (precision != NZE_FP64 && precision != NZE_MIXED) return fail(NZE_EINVAL, "precision");
  if (R < 1 || R > 4 * CHI_LIMIT || C < 4 || (C & 3) || !X || !W || !norms || max_sweeps < 1 || max_sweeps > MAXSW)
    return fail(NZE_EINVAL, "bad rowortho arguments (1 <= R <= 2048, C a positive multiple of 4, sweeps 1..40)");
  return NZE_OK;
}

}  // namespace

extern "C" int nze_kernel_rowortho(int32_t precision, int32_t R, int32_t C,
                                   void* X, void* W, double tol_rel,
                                   double tol_abs, int32_t max_sweeps,
                                   double* norms, int32_t* sweeps,
                                   void* stream) {
  int rc = rowortho_args(precision, R, C, X, W, norms, max_sweeps);
  if (rc) return rc;
  char* scr;
  rc = hook_scratch(&scr);
  if (rc) return rc;
  return rowortho_impl(precision, R, C, X, W, tol_rel, tol_abs, max_sweeps, norms, sweeps,
                       reinterpret_cast<hipStream_t>(stream), scr);
}

namespace {

// Scratch of the allocation-free variant: one 64 KiB array in every GPU's
// memory for the life of the process.  In host code `scratch` names a host
// stand-in; its device address comes from hipGetSymbolAddress, once per
// device, and only that address is ever passed to a kernel or a copy.
__device__ __align__(256) char scratch[HOOK_BYTES];
std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;

int static_scratch(char** out) {
  int dev;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) { *out = it->second; return NZE_OK; }
  char* ptr = nullptr;
  HIPCHK(hipGetSymbolAddress(reinterpret_cast<void**>(&ptr), HIP_SYMBOL(scratch)));
  if (!ptr) return fail(NZE_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
  g_scratch_ptr[dev] = ptr;
  *out = ptr;
  return NZE_OK;
}

}  // namespace

extern "C" int nze_kernel_rowortho_static(int32_t precision, int32_t R, int32_t C,
                                          void* X, void* W, double tol_rel,
                                          double tol_abs, int32_t max_sweeps,
                                          double* norms, int32_t* sweeps,
                                          void* stream) {
  int rc = rowortho_args(precision, R, C, X, W, norms, max_sweeps);
  if (rc) return rc;
  char* scr;
  rc = static_scratch(&scr);
  if (rc) return rc;
  return rowortho_impl(precision, R, C, X, W, tol_rel, tol_abs, max_sweeps, norms, sweeps,
                       reinterpret_cast<hipStream_t>(stream), scr);
}

