// Device-side building blocks for gfx950 (CDNA4, wave64): MFMA wrappers,
// per-MPO workgroup-group barriers, the block one-sided Jacobi pair step, and
// the tiled contraction / gather routines used by the persistent layer kernel.
#ifndef NZE_DEVICE_H
#define NZE_DEVICE_H

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nze {

constexpr int NT = 256;          // threads per workgroup (4 waves)
constexpr int BW = 16;           // Jacobi row-block width b
constexpr int PR = 32;           // rows of one block pair (2b)
constexpr int GLD = 33;          // LDS leading dimension of 32x32 fp64 tiles
constexpr int MAXSW = 40;        // sweep-counter slots
constexpr int CHI_LIMIT = 512;   // largest chi_max (select sorts 4*chi keys)
constexpr int SMEM_DOUBLES = 6400;

enum { OP_NONE = 0, OP_GATE_LR = 1, OP_GATE_RL = 2, OP_MOVE_LR = 3,
       OP_MOVE_RL = 4, OP_JACOBI = 5 };   // OP_JACOBI: SVD of X alone (tuning)

// per-MPO float64 scalars
enum { SC_LOG = 0, SC_FID = 1, SC_MAXDISC = 2, SC_MINGAP = 3, SC_F2 = 4,
       SC_KEPT = 5, SC_FLOPS = 6, SC_CAPQ = 7, SC_TOT = 8, SC_ABOVE = 9,
       SC_COUNT = 10 };
// SC_TOT: ||X||^2 of the block entering the last Jacobi; SC_ABOVE: number of
// singular values above tau s_1 at the last selection
// per-MPO int counters
enum { CT_RANK = 0, CT_ERR = 1, CT_MAXSW = 2, CT_UPD = 3, CT_SWTOT = 4,
       CT_OFFMAX = 5, CT_CAPHIT = 6, CT_NSMAX = 7, CT_ROT = 8, CT_BVER = 8 + MAXSW,
       CT_WVER = CT_BVER + 136, CT_NSFB = CT_WVER + 136, CT_COUNT = CT_NSFB + 1 };
// CT_NSFB: orthonormalisations that needed the scaled (slow) iteration
// CT_BVER / CT_WVER: per row block (<= 136), visits whose data rows / whose
// accumulator rows (kernel hook) are final
enum { ERR_NOCONV = 1, ERR_NAN = 2, ERR_ABORT = 4 };

// Everything one MPO (one noise level of one job) owns on the device.
struct Slot {
  void* sites;      // [n][site_cap] path precision; site k is (chi_l, 4, chi_r)
  int* dims;        // [n + 1] bond dimensions, dims[0] = dims[n] = 1
  double* scal;     // [SC_COUNT]
  int* ctr;         // [CT_COUNT]
  void* X;          // [m_cap * m_cap] two-site block / Jacobi data
  void* W;          // [m_cap * m_cap] layer kernel: copy of the unrotated
                    // block for the refinement; kernel hook: Jacobi
                    // accumulator (rows)
  double* norms;    // [m_cap] squared row norms
  int* perm;        // [m_cap] kept rows, in decreasing norm
  double* sval;     // [m_cap] kept singular values
  int n, chi, site_cap, m_cap;
  double tau, tie, tol_rel, tol_abs;
  int max_sweeps;
  int no_acc;       // 1 (the layer kernel's MPOs): the Jacobi keeps no
                    // accumulator, the float64 refinement builds the
                    // orthonormal factor from the rows; 0 (kernel hook): the
                    // rotations accumulate in W
  double* prof;     // [PROF_N] constant-rate clock ticks per phase (WG 0)
  // Jacobi schedule: the first cross_sweeps sweeps of problems with at least
  // cross_min_blocks row blocks take cross-block inner steps only
  int cross_sweeps, cross_min_blocks;
  // float64 refinement workspace (both precisions):
  // [(chi + 16) * m_cap] + [max((chi + 16)^2, 1088)] + [(chi + 16) * m_cap] doubles
  double* R64;
};

// phase timers of workgroup 0 of each MPO
enum { PF_THETA = 0, PF_GRAM, PF_CHECK, PF_EIGH, PF_ROTX, PF_ROTW, PF_WAIT,
       PF_NORMS, PF_SELECT, PF_ABSORB, PF_MOVE_PREP, PF_MOVE_GEMM, PF_SWEEP,
       PF_PAIRS, PF_WAIT_ALL, PF_N = 16 };

struct PhaseClock {
  bool on;
  uint64_t t;
  __device__ __forceinline__ PhaseClock(bool active) : on(active), t(active ? wall_clock64() : 0) {}
  __device__ __forceinline__ void lap(double* prof, int slot) {
    if (!on) return;
    const uint64_t now = wall_clock64();
    if (threadIdx.x == 0) prof[slot] += double(now - t);
    t = now;
  }
};

struct Step {
  int op;    // OP_*
  int k;     // gate: left site; move: site the centre leaves; jacobi: rows
  int ptm;   // gate: index of its 16x16 PTM in the launch's PTM array;
             // jacobi: columns
  int pad;
};

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct AccT;
template <> struct AccT<float> { typedef f32x4 type; };
template <> struct AccT<double> { typedef f64x4 type; };

// D(16x16) += A(16x4) B(4x16).  Lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator element r of lane l is D[mrow<T>(l/16, r)][l%16]
// (float32: row 4*(l/16) + r; float64: row l/16 + 4*r).
__device__ inline f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f64x4 mfma4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T> __device__ inline int mrow(int kq, int r);
template <> __device__ inline int mrow<float>(int kq, int r) { return 4 * kq + r; }
template <> __device__ inline int mrow<double>(int kq, int r) { return kq + 4 * r; }

// Row data lives in device (global) memory, but its pointers come out of the
// slot records as generic pointers; these accessors cast them to the global
// address space so that the accesses are global, not flat, instructions
// (flat accesses also count against the LDS wait counter, so every LDS wait
// of the pair phases would wait for them too).
typedef float nze_v4f __attribute__((ext_vector_type(4)));
typedef float nze_v2f __attribute__((ext_vector_type(2)));
typedef double nze_v2d __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const nze_v4f g_cv4f;
typedef __attribute__((address_space(1))) const nze_v2d g_cv2d;
typedef __attribute__((address_space(1))) nze_v2f g_v2f;
typedef __attribute__((address_space(1))) nze_v2d g_v2d;

template <typename T>
__device__ inline T load1(const T* p) {
  return *(__attribute__((address_space(1))) const T*)p;
}
template <typename T>
__device__ inline void store1(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}
__device__ inline void load4(const float* p, float v[4]) {
  const nze_v4f x = *(g_cv4f*)p;
  v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
}
__device__ inline void load4(const double* p, double v[4]) {
  const nze_v2d a = *(g_cv2d*)p;
  const nze_v2d b = *(g_cv2d*)(p + 2);
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ inline void store2(float* p, float a, float b) {
  nze_v2f x;
  x.x = a; x.y = b;
  *(g_v2f*)p = x;
}
__device__ inline void store2(double* p, double a, double b) {
  nze_v2d x;
  x.x = a; x.y = b;
  *(g_v2d*)p = x;
}

// Raw buffer resource over `bytes` bytes at `base` (gfx9 descriptor word 3).
// A load at an offset outside [0, bytes) returns zeros and a store there is
// dropped, so lanes whose row or column is out of range need no branch
// around their accesses; with no branches the compiler counts the loads in
// flight exactly and can wait for the older ones only.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr uint32_t OOB = 0x80000000u;   // an offset beyond every buffer here
// base and bytes must be the same in every lane of the wave: they are read
// from the first lane, so that the descriptor sits in scalar registers.
__device__ inline rsrc_t make_rsrc(const void* base, size_t bytes) {
  const uint64_t p = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)p);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(p >> 32));
  const uint32_t n = __builtin_amdgcn_readfirstlane(
      (uint32_t)(bytes < 0x7fffffffu ? bytes : 0x7fffffffu));
  return __builtin_amdgcn_make_buffer_rsrc(
      reinterpret_cast<void*>(((uint64_t)hi << 32) | lo), (short)0, (int)n, 0x00020000);
}
__device__ inline void bload4(rsrc_t r, uint32_t off, float v[4]) {
  const nze_v4f x = __builtin_bit_cast(nze_v4f, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
}
__device__ inline void bload4(rsrc_t r, uint32_t off, double v[4]) {
  const nze_v2d a = __builtin_bit_cast(nze_v2d, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  const nze_v2d b = __builtin_bit_cast(nze_v2d, __builtin_amdgcn_raw_buffer_load_b128(r, off + 16, 0, 0));
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}

typedef unsigned nze_v2u __attribute__((ext_vector_type(2)));
typedef unsigned nze_v4u __attribute__((ext_vector_type(4)));
__device__ inline void bstore2(rsrc_t r, uint32_t off, float a, float b) {
  nze_v2f x;
  x.x = a; x.y = b;
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(nze_v2u, x), r, off, 0, 0);
}
__device__ inline void bstore2(rsrc_t r, uint32_t off, double a, double b) {
  nze_v2d x;
  x.x = a; x.y = b;
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(nze_v4u, x), r, off, 0, 0);
}

// Largest value over the wave, in every lane, without LDS: DPP exchanges
// inside each row of 16 lanes (quad swaps, half-row mirror, row mirror), then
// the four row maxima through scalar registers.  max is exact, so the result
// does not depend on the order of the exchanges.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float wave_max(float v) {
  v = fmaxf(v, dpp_f32<0xB1>(v));    // quad_perm [1, 0, 3, 2]
  v = fmaxf(v, dpp_f32<0x4E>(v));    // quad_perm [2, 3, 0, 1]
  v = fmaxf(v, dpp_f32<0x141>(v));   // row_half_mirror
  v = fmaxf(v, dpp_f32<0x140>(v));   // row_mirror
  const int b = __float_as_int(v);
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(b, 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(b, 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(b, 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(b, 48));
  return fmaxf(fmaxf(r0, r1), fmaxf(r2, r3));
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x141>(v));
  v = fmax(v, dpp_f64<0x140>(v));
  double r[4];
  for (int k = 0; k < 4; ++k)
    r[k] = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 16 * k),
                            __builtin_amdgcn_readlane(__double2loint(v), 16 * k));
  return fmax(fmax(r[0], r[1]), fmax(r[2], r[3]));
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the workgroup; every thread gets the result.  red needs 4 doubles.
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double s = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return s;
}

// ------------------------------------------------------------ group sync

// Barrier across the G workgroups that serve one MPO.  The counter grows
// monotonically within one launch and is cleared by a fill kernel before the
// launch.  The wait is bounded: past `timeout` ticks of the constant-rate
// clock the launch-wide abort flag is raised and every waiter returns false.
struct Group {
  int* bar;
  int* abort_flag;
  int G;
  int nbar;
  uint64_t timeout;
  int* sflag;   // one LDS int
  int local;    // every workgroup of the group runs on one XCD
};

// XCD (accelerator complex die) this wave runs on.
__device__ inline int xcc_id() {
  unsigned v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return (int)(v & 7u);
}

__device__ inline bool group_sync(Group& grp) {
  // every wave's global stores have completed before the workgroup barrier;
  // thread 0 then publishes them (release), arrives, waits, and acquires (the
  // vector L1 it invalidates is shared by the whole workgroup).  A group on
  // one XCD shares that XCD's L2, where the completed stores already are:
  // release is the store wait alone and acquire invalidates the L1 only,
  // instead of writing back and invalidating the whole L2.
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  grp.nbar += 1;
  if (threadIdx.x == 0) {
    if (!grp.local) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    atomicAdd(grp.bar, 1);
    const int target = grp.nbar * grp.G;
    int ok = 1;
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(grp.bar, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(grp.abort_flag, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
      if (wall_clock64() - t0 > grp.timeout) {
        atomicExch(grp.abort_flag, 1);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (grp.local) asm volatile("buffer_inv sc1\n\ts_waitcnt vmcnt(0)" ::: "memory");
    else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *grp.sflag = ok;
  }
  __syncthreads();
  const int ok = *grp.sflag;
  __syncthreads();
  return ok != 0;
}

// Dataflow between the pair visits of a Jacobi sweep: ver[b] counts the
// visits of row block b.  A visit of round t may start once both of its
// blocks have completed round t - 1 (ver >= base + t), instead of waiting
// for every pair of the round.  In the kernel hook, which accumulates the
// rotations, accumulator rows have counters of their own, so the
// accumulator rotation of one visit overlaps the next visits of the blocks.
__device__ inline bool blocks_wait(Group& grp, const int* ver, int I, int J,
                                   int target) {
  if (threadIdx.x == 0) {
    int ok = 1;
    // both counters are loaded together (one round trip to L2, not two)
    auto ready = [&]() {
      const int vi = __hip_atomic_load(ver + I, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int vj = __hip_atomic_load(ver + J, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return (vi >= target) & (vj >= target);
    };
    if (!ready()) {
      const uint64_t t0 = wall_clock64();
      while (!ready()) {
        if (__hip_atomic_load(grp.abort_flag, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
        if (wall_clock64() - t0 > grp.timeout) {
          atomicExch(grp.abort_flag, 1);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    // the rows may be cached from an earlier visit of this workgroup
    if (grp.local) asm volatile("buffer_inv sc1\n\ts_waitcnt vmcnt(0)" ::: "memory");
    else __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *grp.sflag = ok;
  }
  __syncthreads();
  const int ok = *grp.sflag;
  // after a successful wait the next write of sflag follows the barriers of
  // the visit (or of blocks_release); a failed one returns through paths
  // without them
  if (!ok) __syncthreads();
  return ok != 0;
}

// Publishes the visit's row updates, then counts the visit on both blocks.
__device__ inline void blocks_release(const Group& grp, int* ver, int I, int J) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    if (!grp.local) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    atomicAdd(ver + I, 1);
    atomicAdd(ver + J, 1);
  }
}

}  // namespace nze

#endif
