// HIP kernels (gfx950, wave64) of the imaginary-time FDTD library.
//
// The hot kernel is k_step: one pass over the lattice that applies the update
// of Eq. (updateeq) (Strickland & Yager-Elorriaga, Sec. III) to every site and,
// in the same pass, reduces the norm, the kinetic and potential energy sums of
// Eq. (energysum) and the r^2 moment of the state it reads, plus the norm of
// the state it writes.  It is HBM-bound (about 1.7 flop per byte in FP32), so
// the design is about bytes, not flops:
//   * z is the contiguous axis; each lane owns VZ consecutive z sites of
//     RY (y, z) vectors and streams them along x, keeping planes x-1, x, x+1 in
//     registers, so every psi value comes from HBM once per step;
//   * the y +- 1 and z +- 1 neighbours are re-read from the plane the
//     work-group (and its XCD neighbours, see the work-item order built on the
//     host) has just streamed, i.e. from L1/L2, not HBM;
//   * the update is written in increment form psi' = s (psi + B (c lap - dt V
//     psi)) with B = 1/(1 + dt V/2) computed in registers from V (algebraically
//     A psi + B c lap with A = 2B - 1), so V is the only stored coefficient;
//   * the Laplacian is summed from neighbour differences in mirror-symmetric
//     pairs, so a parity-symmetric state stays exactly symmetric;
//   * reductions accumulate in FP64 per lane, then wave shuffle, LDS and a
//     fixed-order sum of per-work-item partials by the last work-group to
//     finish a member (deterministic run to run);
//   * the renormalisation scale of step t is computed from the output norm of
//     step t - 1 and folded into the update (the update is linear), so no
//     extra pass and no host round trip is needed.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "fdtd_internal.h"

// No implicit fused multiply-adds anywhere in this file: every fma is written
// out (fma_c), so a site's arithmetic is the same whichever kernel it is
// inlined into.  The one-step, persistent and two-step kernels then give the
// same bits for the same step.
#pragma clang fp contract(off)

namespace fdtd {
namespace {

// ---------------------------------------------------------------- types ----
template <int DT>
struct Types;
template <>
struct Types<kF64> {
  using S = double;  // storage
  using V = double;  // potential storage
  using C = double;  // arithmetic
  static constexpr int kVec = 2;
};
template <>
struct Types<kF32> {
  using S = float;
  using V = float;
  using C = float;
  static constexpr int kVec = 4;
};
template <>
struct Types<kBF16> {
  using S = uint16_t;
  using V = float;
  using C = float;
  static constexpr int kVec = 8;
};

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Round to nearest even; NaN stays a (quiet) NaN.  Acts on the magnitude
// bits only, so it commutes with negation.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t rne = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  return (uint16_t)(((u & 0x7fffffffu) > 0x7f800000u) ? ((u >> 16) | 0x40u) : rne);  // quiet NaN
}

template <typename S, typename C>
__device__ __forceinline__ C to_c(S v) {
  if constexpr (sizeof(S) == 2) {
    return (C)bf16_to_f32(v);
  } else {
    return (C)v;
  }
}

template <typename S, typename C>
__device__ __forceinline__ S from_c(C v) {
  if constexpr (sizeof(S) == 2) {
    return f32_to_bf16((float)v);
  } else {
    return (S)v;
  }
}

template <typename S, int VZ>
struct alignas(sizeof(S) * VZ) Pack {
  S v[VZ];
};

template <typename S, int VZ, typename C>
__device__ __forceinline__ void load_vec(const S* __restrict__ p, C (&o)[VZ]) {
  const Pack<S, VZ> t = *reinterpret_cast<const Pack<S, VZ>*>(p);
#pragma unroll
  for (int j = 0; j < VZ; ++j) o[j] = to_c<S, C>(t.v[j]);
}

template <typename S, int VZ>
__device__ __forceinline__ void store_vec(S* __restrict__ p, const Pack<S, VZ>& t) {
  *reinterpret_cast<Pack<S, VZ>*>(p) = t;
}

template <typename C, int VZ>
__device__ __forceinline__ void zero_vec(C (&o)[VZ]) {
#pragma unroll
  for (int j = 0; j < VZ; ++j) o[j] = C(0);
}

__device__ __forceinline__ float rcp_c(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_c(double x) { return 1.0 / x; }
__device__ __forceinline__ float fma_c(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_c(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum NV values over the work-group; the result is valid in thread 0.
// Fixed order: lanes by butterfly, then waves 0..3 left to right.
template <int NV, int NW = kBlock / 64>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*red)[NV]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if ((tid & 63) == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[tid >> 6][k] = v[k];
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double t = red[0][k];
#pragma unroll
      for (int w = 1; w < NW; ++w) t += red[w][k];
      v[k] = t;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ bool finite_d(double x) { return !(isnan(x) || isinf(x)); }

// Values the work-group shares (work-item fields, member constants) kept in
// scalar registers: buffer descriptors built from them must be uniform, or
// every buffer access becomes a per-lane loop.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned uni(unsigned v) {
  return (unsigned)__builtin_amdgcn_readfirstlane((int)v);
}
template <typename T>
__device__ __forceinline__ T* uni(T* p) {
  const unsigned long long u = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
  return reinterpret_cast<T*>(((unsigned long long)hi << 32) | lo);
}

// ------------------------------------------------------- buffer access ----
// Raw buffer loads return 0 and raw buffer stores are dropped for offsets at
// or beyond the resource's size.  Each x-plane gets its own resource, sized
// to the plane (or to 0 for the ghost planes x = -1 and x = N), so the
// Dirichlet ghosts around the lattice, the y = -1 / y = N rows and the
// ragged tail of a work item cost no branches and no HBM traffic.
constexpr int kRsrcWord3 = 0x00020000;  // gfx9-family raw buffer descriptor
constexpr unsigned kDeadLane = 1u << 28;  // element offset used by lanes past the plane

// Resource for plane x of a field whose planes are `bytes` long; planes
// outside [0, N) get an empty resource (every access reads 0 / is dropped).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, int x, int N,
                                                            unsigned bytes) {
  const bool in = x >= 0 && x < N;
  char* p = const_cast<char*>(static_cast<const char*>(base)) + (in ? (long long)x * bytes : 0);
  return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, in ? (int)bytes : 0, kRsrcWord3);
}

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Cache policy bits of buffer accesses: kNT streams past the caches (data
// used once: V, and the written state); kKeep leaves the default policy
// (psi, whose lines are re-read as neighbours by adjacent lanes).
constexpr int kKeep = 0;
constexpr int kNT = 2;
// Stores written through at system scope (sc0 sc1): the written state stays in
// the last-level cache (MALL) for the next step's reads.  Measured per FP32
// step: 256^3 51.7 -> 42.5 us, 320^3 101.9 -> 88.5 us, but 384^3 158.6 -> 162.0
// and 512^3 282.1 -> 283.3 us, where the lattice does not fit.
constexpr int kWriteThrough = 1 | 16;
// Build-time choice of the policies of the four streams of the step kernel.
#ifndef FDTD_AUX_PSI
#define FDTD_AUX_PSI 0  // own-site psi loads (first touch of each plane)
#endif
#ifndef FDTD_AUX_NBR
#define FDTD_AUX_NBR 0  // y / z neighbour loads (re-reads, meant to hit L2)
#endif
#ifndef FDTD_AUX_V
#define FDTD_AUX_V 2    // V loads (used once): non-temporal
#endif
#ifndef FDTD_AUX_OUT
#define FDTD_AUX_OUT 2  // psi' stores (read back only by the next launch): non-temporal
#endif

// Load VZ consecutive elements of S at byte offset `off`, converted to C.
template <typename S, int VZ, typename C, int AUX = kKeep>
__device__ __forceinline__ void bload(__amdgpu_buffer_rsrc_t r, unsigned off, C (&o)[VZ]) {
  constexpr int kBytes = (int)sizeof(S) * VZ;
  if constexpr (kBytes == 16) {
    const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, AUX);
    const Pack<S, VZ> t = __builtin_bit_cast(Pack<S, VZ>, w);
#pragma unroll
    for (int j = 0; j < VZ; ++j) o[j] = to_c<S, C>(t.v[j]);
  } else if constexpr (kBytes == 32) {
    const u32x4 w0 = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, AUX);
    const u32x4 w1 = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off + 16, 0, AUX);
    const Pack<S, VZ / 2> t0 = __builtin_bit_cast(Pack<S, VZ / 2>, w0);
    const Pack<S, VZ / 2> t1 = __builtin_bit_cast(Pack<S, VZ / 2>, w1);
#pragma unroll
    for (int j = 0; j < VZ / 2; ++j) {
      o[j] = to_c<S, C>(t0.v[j]);
      o[j + VZ / 2] = to_c<S, C>(t1.v[j]);
    }
  } else if constexpr (kBytes == 8) {
    const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, AUX);
    const Pack<S, VZ> t = __builtin_bit_cast(Pack<S, VZ>, w);
#pragma unroll
    for (int j = 0; j < VZ; ++j) o[j] = to_c<S, C>(t.v[j]);
  } else if constexpr (kBytes == 4) {
    const unsigned w = __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, AUX);
    const Pack<S, VZ> t = __builtin_bit_cast(Pack<S, VZ>, w);
#pragma unroll
    for (int j = 0; j < VZ; ++j) o[j] = to_c<S, C>(t.v[j]);
  } else {
    static_assert(kBytes == 2, "unsupported vector width");
    const unsigned short w = __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, AUX);
    o[0] = to_c<S, C>(__builtin_bit_cast(S, w));
  }
}

template <typename S, int VZ, int AUX = kKeep>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, unsigned off, const Pack<S, VZ>& t) {
  constexpr int kBytes = (int)sizeof(S) * VZ;
  if constexpr (kBytes == 32) {
    Pack<S, VZ / 2> lo, hi;
#pragma unroll
    for (int j = 0; j < VZ / 2; ++j) {
      lo.v[j] = t.v[j];
      hi.v[j] = t.v[j + VZ / 2];
    }
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, lo), r, (int)off, 0, AUX);
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, hi), r, (int)off + 16, 0, AUX);
  } else if constexpr (kBytes == 16) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, t), r, (int)off, 0, AUX);
  } else if constexpr (kBytes == 8) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, t), r, (int)off, 0, AUX);
  } else if constexpr (kBytes == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, t), r, (int)off, 0, AUX);
  } else {
    static_assert(kBytes == 2, "unsupported vector width");
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, t), r, (int)off, 0, AUX);
  }
}

// Stochastic rounding to BF16 (used for the stored state of BF16 lattices):
// add 16 random bits to the magnitude and truncate.  The result is unbiased,
// E[round(v)] = v, so increments far below one BF16 ulp still move the state
// on average instead of being rounded away.  Acts on the magnitude only, so
// mirror sites given the same random bits round to exactly opposite values.
// Branch-free: Inf keeps its all-zero low half, so adding r16 < 2^16 leaves
// it Inf; a NaN magnitude is first replaced by the quiet NaN 0x7fc00000,
// which the addition cannot carry out of the NaN range.
__device__ __forceinline__ uint16_t f32_to_bf16_sr(float f, uint32_t r16) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t mag = min(u & 0x7fffffffu, 0x7fc00000u);
  return (uint16_t)(((u & 0x80000000u) | (mag + r16)) >> 16);
}

// 32-bit integer hash (lowbias32, C. Wellons): random bits of the rounding.
// The 32 bits of a site are hash32(q ^ kSaltYZ) ^ hash32(cx + hash32(step)),
// with cx = min(x, N - 1 - x) and q its mirror-canonical (y, z) index k
// (odd N) or k >> 1 (even N).  The first factor is fixed per lane for a whole
// work item, the second is uniform over the work-group (scalar unit), so a
// site costs one XOR.  On even N one 32-bit draw serves two sites: the site
// takes half k & 1; the z-pair {2i, 2i+1} always shares k >> 1 (on one side
// of the centre the two indices differ in the last bit only; a pair across
// the centre is one canonical site).  The bits depend on the canonical
// (x, y, z) and the step only, never on the launch shape, and mirror sites
// share them.
__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
constexpr uint32_t kSaltYZ = 0x68e31da4u;

// Device-scope relaxed load of member state that other work-groups of the
// same launch may have written (a vector load, never the scalar cache).
template <typename T>
__device__ __forceinline__ T ld_agent(const T& x) {
  return __hip_atomic_load(const_cast<T*>(&x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A work item hands its partial sums to the member's last work-group within
// one launch.  Only the partials cross work-groups inside a launch (the
// updated state is read by the next launch), so instead of a release fence,
// which writes back the whole L2 of this XCD, the partials are stored as
// agent-scope atomic stores (written through to the coherence point), the
// wave waits until they have completed (vmcnt(0)), and only then counts the
// item on the member's counter; the last work-group reads them with
// agent-scope atomic loads.  Returns the counter's previous value.
template <int NV>
__device__ __forceinline__ unsigned publish_partials(double* const (&dst)[NV], const double (&v)[NV][5],
                                                     unsigned* counter) {
#pragma unroll
  for (int i = 0; i < NV; ++i)
#pragma unroll
    for (int q = 0; q < 5; ++q)
      __hip_atomic_store(&dst[i][q], v[i][q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt, lgkmcnt unconstrained
  return __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last work-group of member m: record the step's sums, set the scale of the
// next update, advance the step counter, flag non-finite sums, re-arm the
// completion counter and, last, publish the step as finalised (release).
// rn: -1 the renorm_every rule (rescale when the new step count is a
// multiple of renorm_every); 0 no rescale; 1 the rule applied to this step or
// the one before (the second step of a temporally blocked pass: a rescale due
// after the first is deferred to it).
__device__ __forceinline__ void finalize(const StepArgs& A, const MemberDev& M, int m,
                                      const double (&tot)[5], bool upd, int rn = -1) {
  MemberState& st = A.states[m];
  const double kin = -M.kin_scale * tot[1];
  const long long t = ld_agent(st.step);
  double rec[kRec] = {tot[0], kin, tot[2], tot[3], tot[4], (double)t, ld_agent(st.scale), 0.0};
  if (upd) {
    double* dst = A.ring + ((long long)m * A.ring_cap + (t % A.ring_cap)) * kRec;
#pragma unroll
    for (int k = 0; k < kRec; ++k) dst[k] = rec[k];
    const long long nt = t + 1;
    const bool renorm = A.renorm_every > 0 && rn != 0 &&
                        ((nt % A.renorm_every) == 0 || (rn == 1 && ((nt - 1) % A.renorm_every) == 0));
    st.scale = renorm ? 1.0 / sqrt(M.a3 * tot[4]) : 1.0;
    st.step = nt;
    if (!(finite_d(tot[0]) && finite_d(tot[4]) && finite_d(kin) && finite_d(tot[2])) &&
        !ld_agent(st.bad)) {
      st.bad = 1;
      st.bad_step = t;
    }
  } else {
    // reduction-only pass: the host inspects the sums itself
    double* dst = A.obs_out + (long long)m * kRec;
#pragma unroll
    for (int k = 0; k < kRec; ++k) dst[k] = rec[k];
    if (A.set_scale) st.scale = 1.0 / sqrt(M.a3 * tot[0]);
  }
  st.counter = 0u;
  if (upd) __hip_atomic_fetch_add(&st.fin, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Cross-lane read within the wave (ds_bpermute through the LDS crossbar,
// no memory traffic); src must be in [0, 64) for the lanes whose result is used.
__device__ __forceinline__ float shfl_c(float v, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute((src & 63) << 2, __float_as_int(v)));
}
__device__ __forceinline__ double shfl_c(double v, int src) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute((src & 63) << 2, (int)u);
  const int hi = __builtin_amdgcn_ds_bpermute((src & 63) << 2, (int)(u >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

#ifndef FDTD_SHUFFLE_Z
#define FDTD_SHUFFLE_Z 1
#endif
constexpr bool kShuffleZ = FDTD_SHUFFLE_Z != 0;

// ------------------------------------------------------- fused step kernel --
// Per-lane state of one work item: RY vectors of VZ sites at fixed (y, z).
template <int RY, int VZ, typename C>
struct Lane {
  unsigned off[RY];       // byte offset of the vector in a plane (storage dtype)
  unsigned voff[RY];      // byte offset of the vector in a plane of V
  unsigned offm[RY];      // y - 1 neighbour vector (may wrap: then out of range)
  unsigned offp[RY];      // y + 1 neighbour vector (out of range past the plane)
  unsigned offzm[RY];     // z - 1 site, for the wave's first lane only (else out of range)
  unsigned offzp[RY];     // z + 1 site, for the wave's last lane only (else out of range)
  float zmask_lo[RY];     // 0 where the vector starts at z = 0 (its z - 1 is a ghost)
  float zmask_hi[RY];     // 0 where the vector ends at z = N - 1
  C w2[RY][VZ];           // y^2 + z^2 of each site
  uint32_t hk[RY][VZ > 1 ? VZ / 2 : 1];  // (y, z) part of the rounding bits (BF16)
  uint32_t hsh[RY][VZ];   // which half of the 32 bits a site takes: 0 or 16
  C vl[RY][VZ];           // (y, z) part of a potential evaluated in the kernel
};

// Data of one plane that the update of that plane needs besides the planes
// x-1, x, x+1 of the lane's own sites: V and the y / z neighbours.
template <int RY, int VZ, typename C>
struct PlaneIn {
  C ym[RY][VZ], yp[RY][VZ], zm[RY], zp[RY];
};

// Analytic potentials the step can evaluate itself (FP32 arithmetic) instead
// of streaming V from HBM; the numbering is that of the C ABI.
enum VKind { kVConst = 0, kVHO = 1, kVCoulomb = 2, kVCoulombReg = 3, kVCornell = 4 };

// FV: the potential is evaluated in the kernel from the site coordinates
// (member kinds kVConst..kVCornell) instead of read from the V table.
template <int DT, int VZ, int RY, bool UPD, bool FV = false, int OUT = FDTD_AUX_OUT>
struct StepBody {
  using S = typename Types<DT>::S;
  using TV = typename Types<DT>::V;
  using C = typename Types<DT>::C;
  static constexpr unsigned kES = sizeof(S);
  // z neighbours across vector boundaries by cross-lane reads (measured
  // faster for FP32 and FP64; BF16 lanes hold 8 sites and gain nothing)
  static constexpr bool kSHZ = kShuffleZ && DT != kBF16;

  struct Ctx {
    const void* in;
    void* out;
    const TV* Vf;
    unsigned pbytes, vbytes;
    int N;
    int xe;  // end of the work item: planes the item never reads get empty resources
    C c, dt, eps, sc;
    double ha, cN;
    uint32_t smix;  // hash32(step): the step's part of the rounding bits
    // FV only: one branch-free form for every analytic kind,
    //   V = q1 / r + q2 r + hx x^2 + vl(y, z),  0 where r < va,
    // with 1/r taken of r^2 + ve (ve = 1 for kinds without 1/r, so r = 0
    // gives 0 * finite there; ve = 0 keeps Coulomb's singularity):
    //   CONST       vl = p0
    //   HO          hx = p0^2 / 2, vl = (p1^2 y^2 + p2^2 z^2) / 2
    //   COULOMB     q1 = -p0
    //   COULOMB_REG q1 = -p0, vl = p0 / a, va = a
    //   CORNELL     q1 = -p0, q2 = p1, vl = p2 z^2
    C q1, q2, hx, ve, va;
  };

  // Per-kind coefficients of the in-kernel potential (FV).
  static __device__ __forceinline__ void vcoef(Ctx& k, int kind, const double* vp, double a) {
    k.q1 = (kind == kVCoulomb || kind == kVCoulombReg || kind == kVCornell) ? (C)(-vp[0]) : C(0);
    k.q2 = kind == kVCornell ? (C)vp[1] : C(0);
    k.hx = kind == kVHO ? (C)(0.5 * vp[0] * vp[0]) : C(0);
    k.ve = (kind == kVCoulomb || kind == kVCoulombReg || kind == kVCornell) ? C(0) : C(1);
    k.va = kind == kVCoulombReg ? (C)a : C(0);
  }

  // (y, z) part vl of the in-kernel potential of site j of vector r, from
  // its mirror-exact coordinates yc, zc.
  static __device__ __forceinline__ void vlane(Lane<RY, VZ, C>& ln, int r, int j, int kind,
                                               const double* vp, double a, double yc,
                                               double zc) {
    if constexpr (FV) {
      double v = 0.0;
      if (kind == kVConst) v = vp[0];
      else if (kind == kVHO) v = 0.5 * (vp[1] * vp[1] * yc * yc + vp[2] * vp[2] * zc * zc);
      else if (kind == kVCoulombReg) v = vp[0] / a;
      else if (kind == kVCornell) v = vp[2] * zc * zc;
      ln.vl[r][j] = (C)v;
    }
  }

  // The (y, z) part of the rounding bits of vector r (BF16 stores only),
  // from the mirror-canonical (y, z) index of each of its sites.
  static __device__ __forceinline__ void hash_lane(Lane<RY, VZ, C>& ln, int r, int N,
                                                   const uint32_t (&key)[VZ]) {
    if constexpr (sizeof(S) == 2) {
#pragma unroll
      for (int j = 0; j < VZ; j += 2) {
        const uint32_t q = (N & 1) ? key[j] : key[j] >> 1;
        ln.hk[r][j / 2] = hash32(q ^ kSaltYZ);
      }
#pragma unroll
      for (int j = 0; j < VZ; ++j) ln.hsh[r][j] = (N & 1) ? 0u : (key[j] & 1u) << 4;
    }
  }

  // Issue the loads of the y and z neighbours of plane x (needed for x < xe).
  static __device__ __forceinline__ void fetch(const Ctx& k, const Lane<RY, VZ, C>& ln, int x,
                                               PlaneIn<RY, VZ, C>& d) {
    const __amdgpu_buffer_rsrc_t rc = plane_rsrc(k.in, x, min(k.N, k.xe), k.pbytes);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      C zz[1];
      bload<S, VZ, C, FDTD_AUX_NBR>(rc, ln.offm[r], d.ym[r]);
      bload<S, VZ, C, FDTD_AUX_NBR>(rc, ln.offp[r], d.yp[r]);
      bload<S, 1, C, FDTD_AUX_NBR>(rc, ln.offzm[r], zz);
      d.zm[r] = zz[0];
      bload<S, 1, C, FDTD_AUX_NBR>(rc, ln.offzp[r], zz);
      d.zp[r] = zz[0];
    }
  }

  // V of the lane's sites of plane x (needed for x < xe): loaded from the
  // table, or (FV) evaluated from the coordinates.  r^2 = x^2 + (y^2 + z^2)
  // and the other terms are mirror-symmetric bit for bit, as in the table.
  // VAUX: cache policy of the V table loads.
  template <int VAUX = FDTD_AUX_V>
  static __device__ __forceinline__ void fetch_v(const Ctx& k, const Lane<RY, VZ, C>& ln, int x,
                                                 C (&v)[RY][VZ]) {
    if constexpr (FV) {
      const double xd = (2.0 * x - k.cN) * k.ha;
      const C x2 = (C)(xd * xd);
#pragma unroll
      for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int j = 0; j < VZ; ++j) {
          const C r2 = x2 + ln.w2[r][j];
          const C inv = __builtin_amdgcn_rsqf(r2 + k.ve);  // 1/r, hardware (~1 ulp)
          const C rr = r2 * inv;
          const C vv = fma_c(k.q1, inv, fma_c(k.q2, rr, fma_c(k.hx, x2, ln.vl[r][j])));
          v[r][j] = rr < k.va ? C(0) : vv;
        }
    } else {
      const __amdgpu_buffer_rsrc_t rv = plane_rsrc(k.Vf, x, min(k.N, k.xe), k.vbytes);
#pragma unroll
      for (int r = 0; r < RY; ++r) bload<TV, VZ, C, VAUX>(rv, ln.voff[r], v[r]);
    }
  }

  // Own sites of plane x (needed for x <= xe).
  static __device__ __forceinline__ void fetch_own(const Ctx& k, const Lane<RY, VZ, C>& ln, int x,
                                                   C (&q)[RY][VZ]) {
    const __amdgpu_buffer_rsrc_t r0 = plane_rsrc(k.in, x, min(k.N, k.xe + 1), k.pbytes);
#pragma unroll
    for (int r = 0; r < RY; ++r) bload<S, VZ, C, FDTD_AUX_PSI>(r0, ln.off[r], q[r]);
  }

  // Update plane x from pm (x-1), pc (x), pn (x+1) and d; accumulate the
  // reductions of plane x into acc.  SHZ: the z neighbours across a vector
  // boundary come from the adjacent lanes, d.zm / d.zp hold them for the
  // wave's edge lanes only; otherwise d.zm / d.zp hold them for every lane.
  template <bool SHZ = kSHZ, int RYL = RY>
  static __device__ __forceinline__ void update(const Ctx& k, const Lane<RYL, VZ, C>& ln, int x,
                                                const C (&pm)[RY][VZ], const C (&pc)[RY][VZ],
                                                const C (&pn)[RY][VZ], const C (&vv)[RY][VZ],
                                                const PlaneIn<RY, VZ, C>& d, double (&acc)[5],
                                                bool live = true) {
    C unused[1][VZ];
    update_core<SHZ, false, RY>(k, ln, x, pm, pc, pn, vv, d, acc, live, unused);
  }

  // The update of plane x.  TOREG: instead of storing the new values to
  // HBM, return them (as stored: rounded to the storage type) in outv.  Only
  // the first NRED vectors enter the reductions (the two-step kernel's halo
  // sites, NRED = 0, belong to another work item).  The lane may carry more
  // vectors than RY (RYL >= RY): the first RY are updated.
  template <bool SHZ, bool TOREG, int NRED, int NO, int RYL>
  static __device__ __forceinline__ void update_core(const Ctx& k, const Lane<RYL, VZ, C>& ln,
                                                     int x, const C (&pm)[RY][VZ],
                                                     const C (&pc)[RY][VZ],
                                                     const C (&pn)[RY][VZ],
                                                     const C (&vv)[RY][VZ],
                                                     const PlaneIn<RY, VZ, C>& d,
                                                     double (&acc)[5], bool live,
                                                     C (&outv)[NO][VZ]) {
    const double xc = (2.0 * x - k.cN) * k.ha;
    const C rx2 = (C)(xc * xc);
    const __amdgpu_buffer_rsrc_t ro = plane_rsrc(k.out, x, k.N, k.pbytes);
    const uint32_t hx = hash32((uint32_t)min(x, k.N - 1 - x) + k.smix);  // uniform
    C s0 = 0, kin = 0, pot = 0, r2 = 0, s1 = 0;
    const int lane = __lane_id();
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      Pack<S, VZ> o;
      // z - 1 of the first site and z + 1 of the last come from the adjacent
      // lanes (consecutive lanes hold consecutive vectors of the flattened
      // plane); only the wave's edge lanes took them from memory
      C lo, hi;
      if constexpr (SHZ) {
        const C fl = shfl_c(pc[r][VZ - 1], lane - 1);
        const C fr = shfl_c(pc[r][0], lane + 1);
        lo = (lane == 0 ? d.zm[r] : fl) * (C)ln.zmask_lo[r];
        hi = (lane == 63 ? d.zp[r] : fr) * (C)ln.zmask_hi[r];
      } else {
        lo = d.zm[r] * (C)ln.zmask_lo[r];
        hi = d.zp[r] * (C)ln.zmask_hi[r];
      }
      uint32_t rb[VZ];  // 16 random bits per site (BF16 stores)
      if constexpr (UPD && sizeof(S) == 2) {
#pragma unroll
        for (int j = 0; j < VZ; ++j) {
          const uint32_t h = ln.hk[r][j / 2] ^ hx;  // the pair {2i, 2i+1} shares h
          rb[j] = __builtin_amdgcn_ubfe(h, ln.hsh[r][j], 16);
        }
      }
#pragma unroll
      for (int j = 0; j < VZ; ++j) {
        const C p = pc[r][j];
        C lft = lo, rgt = hi;
        if (j > 0) lft = pc[r][j - 1];
        if (j < VZ - 1) rgt = pc[r][j + 1];
        // a^2 * Laplacian, neighbours summed in mirror-symmetric pairs so a
        // mirrored or negated state gives the mirrored or negated result bit
        // for bit.  FP32/FP64 states: from neighbour differences (no
        // cancellation against 6 p).  BF16 states: 8-bit significands, so the
        // pair sums and the subtraction of 6 p are exact in FP32 whenever
        // the seven values lie within a factor 2^12 of each other, and the
        // plain sum equals the difference form with five fewer operations.
        C lap;
        if constexpr (sizeof(S) == 2) {
          lap = __builtin_fmaf(-6.f, p, ((pm[r][j] + pn[r][j]) + (d.ym[r][j] + d.yp[r][j])) + (lft + rgt));
        } else {
          lap = (((pm[r][j] - p) + (pn[r][j] - p)) + ((d.ym[r][j] - p) + (d.yp[r][j] - p))) +
                ((lft - p) + (rgt - p));
        }
        const C p2 = p * p;
        const C v = vv[r][j];
        if (r < NRED) {
          s0 += p2;
          kin = fma_c(p, lap, kin);
          pot = fma_c(v, p2, pot);
          r2 = fma_c(ln.w2[r][j], p2, r2);
        }
        if constexpr (UPD) {
          const C B = rcp_c(fma_c(k.eps, v, C(1)));
          const C g = fma_c(k.c, lap, -((k.dt * v) * p));  // c lap - dt V psi
          const C nv = k.sc * fma_c(B, g, p);
          if constexpr (sizeof(S) == 2) {
            o.v[j] = f32_to_bf16_sr((float)nv, rb[j]);
          } else {
            o.v[j] = (S)nv;
          }
          const C od = to_c<S, C>(o.v[j]);
          if (r < NRED) s1 = live ? fma_c(od, od, s1) : s1;
          if constexpr (TOREG) outv[r][j] = od;
        }
      }
      if constexpr (UPD && !TOREG) bstore<S, VZ, OUT>(ro, ln.off[r], o);
    }
    acc[0] += (double)s0;
    acc[1] += (double)kin;
    acc[2] += (double)pot;
    acc[3] += (double)r2 + (double)rx2 * (double)s0;
    acc[4] += (double)s1;
  }

  // Update plane X = xb + 6 i + SL of a work item whose planes live in rings
  // of six register slots: psi(p) in slot (p - xb + 1) % 6, V(p) and the
  // neighbour set of p in slot (p - xb) % 6.  The stage first issues every
  // load D planes ahead (psi(X + 1 + D), V(X + D), neighbours of X + D), then
  // updates plane X from data fetched D stages earlier.  All streams use the
  // same distance because the vector-memory counter retires loads in issue
  // order: a nearer load issued after a farther one would make the wait for
  // it wait for the farther one too.
  template <int D, int SL>
  static __device__ __forceinline__ void stage(const Ctx& k, const Lane<RY, VZ, C>& ln, int X,
                                               C (&qs)[6][RY][VZ], C (&vs)[6][RY][VZ],
                                               PlaneIn<RY, VZ, C> (&nb)[6], double (&acc)[5]) {
    fetch_own(k, ln, X + 1 + D, qs[(SL + 2 + D) % 6]);
    fetch_v(k, ln, X + D, vs[(SL + D) % 6]);
    fetch(k, ln, X + D, nb[(SL + D) % 6]);
    update(k, ln, X, qs[SL % 6], qs[(SL + 1) % 6], qs[(SL + 2) % 6], vs[SL % 6], nb[SL % 6], acc);
  }
};

#ifndef FDTD_STEP_MIN_WAVES
#define FDTD_STEP_MIN_WAVES 1  // waves per SIMD the register budget must allow
#endif

// One work item of the fused step: update (UPD) the item's sites of the
// member's buffer src into src ^ 1, reduce, and let the member's last
// work-group finalise the step.  Member state is read with atomic loads: in
// the persistent kernel another work-group may have changed it since this
// one last looked, and the loads must not come from a stale scalar cache.
// FENCE: the persistent kernel, where the next step's work items (on any
// XCD) read this item's updated state within the same launch, publishes with
// a full release fence; one launch per step only needs the partials to cross.
template <int DT, int VZ, int RY, bool UPD, int D, int BT, bool FV = false, int OUT = FDTD_AUX_OUT,
          bool FENCE = false>
__device__ __forceinline__ void run_item(const StepArgs& A, const Item& item, int src,
                                         double (&s_red)[BT / 64][5], int& s_last) {
  using Body = StepBody<DT, VZ, RY, UPD, FV, OUT>;
  using S = typename Body::S;
  using TV = typename Body::TV;
  using C = typename Body::C;
  constexpr unsigned kES = sizeof(S);
  const int tid = threadIdx.x;
  {
    const int m = item.member;
    const MemberDev& M = A.members[m];
    const int N = M.N;
    const unsigned P = (unsigned)M.plane;
    const void* in = M.psi[src];
    void* out = M.psi[src ^ 1];
    const TV* Vf = static_cast<const TV*>(M.V);
    const unsigned pbytes = P * kES, vbytes = P * (unsigned)sizeof(TV);
    const C c = (C)M.c;
    const C dt = (C)M.dt;
    const C eps = (C)(0.5 * M.dt);
    const C sc = (C)ld_agent(A.states[m].scale);
    const uint32_t smix = hash32((uint32_t)ld_agent(A.states[m].step));
    const double ha = M.ha;
    const double cN = (double)(N - 1);

    Lane<RY, VZ, C> ln;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const unsigned f = (unsigned)item.f0 + (unsigned)(r * BT + tid) * VZ;
      const bool ok = f < P;
      const unsigned fe = ok ? f : kDeadLane;
      const int y = ok ? (int)(f / (unsigned)N) : 0;
      const int z0 = ok ? (int)(f - (unsigned)y * N) : 0;
      ln.off[r] = fe * kES;
      ln.voff[r] = fe * (unsigned)sizeof(TV);
      ln.offm[r] = (fe - (unsigned)N) * kES;  // wraps below row 0: out of range
      ln.offp[r] = (fe + (unsigned)N) * kES;
      const int lane = __lane_id();
      if constexpr (Body::kSHZ) {
        ln.offzm[r] = (ok && lane == 0 && z0 > 0) ? (f - 1u) * kES : kDeadLane * kES;
        ln.offzp[r] = (ok && lane == 63 && z0 + VZ < N) ? (f + VZ) * kES : kDeadLane * kES;
      } else {
        ln.offzm[r] = fe * kES - kES;
        ln.offzp[r] = fe * kES + VZ * kES;
      }
      ln.zmask_lo[r] = (ok && z0 > 0) ? 1.f : 0.f;
      ln.zmask_hi[r] = (ok && z0 + VZ < N) ? 1.f : 0.f;
      const double yc = (2.0 * y - cN) * ha;
      const int cy = min(y, N - 1 - y);
      uint32_t key[VZ];  // mirror-canonical (y, z) index
#pragma unroll
      for (int j = 0; j < VZ; ++j) {
        const double zc = (2.0 * (z0 + j) - cN) * ha;
        ln.w2[r][j] = (C)(yc * yc + zc * zc);
        Body::vlane(ln, r, j, M.vkind, M.vp, M.a, yc, zc);
        const int z = z0 + j;
        key[j] = (uint32_t)cy * (uint32_t)N + (uint32_t)min(z, N - 1 - z);
      }
      Body::hash_lane(ln, r, N, key);
    }

    typename Body::Ctx k;
    if constexpr (FV) Body::vcoef(k, M.vkind, M.vp, M.a);
    k.in = in;
    k.out = out;
    k.Vf = Vf;
    k.pbytes = pbytes;
    k.vbytes = vbytes;
    k.N = N;
    k.c = c;
    k.dt = dt;
    k.eps = eps;
    k.sc = sc;
    k.ha = ha;
    k.cN = cN;
    k.smix = smix;
    k.xe = item.xe;

    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    C qs[6][RY][VZ], vs[6][RY][VZ];
    PlaneIn<RY, VZ, C> nb[6];
    const int xb = item.xb, xe = item.xe;
#pragma unroll
    for (int i = 0; i < D + 2; ++i) Body::fetch_own(k, ln, xb - 1 + i, qs[i]);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      Body::fetch_v(k, ln, xb + i, vs[i]);
      Body::fetch(k, ln, xb + i, nb[i]);
    }
    // six stages per trip, so the ring slots are compile-time constants;
    // full trips carry no branches between stages (a join would make the
    // load-counter waits conservative), the tail of < 6 planes is guarded
    int x = xb;
    for (; x + 6 <= xe; x += 6) {
      Body::template stage<D, 0>(k, ln, x, qs, vs, nb, acc);
      Body::template stage<D, 1>(k, ln, x + 1, qs, vs, nb, acc);
      Body::template stage<D, 2>(k, ln, x + 2, qs, vs, nb, acc);
      Body::template stage<D, 3>(k, ln, x + 3, qs, vs, nb, acc);
      Body::template stage<D, 4>(k, ln, x + 4, qs, vs, nb, acc);
      Body::template stage<D, 5>(k, ln, x + 5, qs, vs, nb, acc);
    }
    if (x < xe) Body::template stage<D, 0>(k, ln, x, qs, vs, nb, acc);
    if (x + 1 < xe) Body::template stage<D, 1>(k, ln, x + 1, qs, vs, nb, acc);
    if (x + 2 < xe) Body::template stage<D, 2>(k, ln, x + 2, qs, vs, nb, acc);
    if (x + 3 < xe) Body::template stage<D, 3>(k, ln, x + 3, qs, vs, nb, acc);
    if (x + 4 < xe) Body::template stage<D, 4>(k, ln, x + 4, qs, vs, nb, acc);

    // ---- per-item partials, then the last work-group of the member sums them
    block_sum<5, BT / 64>(acc, s_red);
    if (tid == 0) {
      double* part = A.partials + (long long)item.slot * kRec;
      unsigned int done;
      if constexpr (FENCE) {
#pragma unroll
        for (int k = 0; k < 5; ++k) part[k] = acc[k];
        __threadfence();
        done = atomicAdd(&A.states[m].counter, 1u);
      } else {
        double* const dst[1] = {part};
        const double v[1][5] = {{acc[0], acc[1], acc[2], acc[3], acc[4]}};
        done = publish_partials<1>(dst, v, &A.states[m].counter);
      }
      s_last = (done + 1u == (unsigned int)(M.item_end - M.item_begin));
    }
    __syncthreads();
    if (s_last) {
      if constexpr (FENCE) __threadfence();
      double tot[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      for (int i = M.item_begin + tid; i < M.item_end; i += BT) {
        const double* part = A.partials + (long long)i * kRec;
#pragma unroll
        for (int k = 0; k < 5; ++k) tot[k] += FENCE ? part[k] : ld_agent(part[k]);
      }
      block_sum<5, BT / 64>(tot, s_red);
      if (tid == 0) finalize(A, M, m, tot, UPD);
    }
    __syncthreads();
  }
}

// WT: the updated state is stored written through (kWriteThrough) instead of
// streamed past the caches.
template <int DT, int VZ, int RY, bool UPD, int D, int BT, bool FV, bool WT = false>
__global__ __launch_bounds__(BT, FDTD_STEP_MIN_WAVES) void k_step(StepArgs A) {
  __shared__ double s_red[BT / 64][5];
  __shared__ int s_last;
  for (int li = blockIdx.x; li < A.n_items; li += gridDim.x)
    run_item<DT, VZ, RY, UPD, D, BT, FV, WT ? kWriteThrough : FDTD_AUX_OUT>(
        A, A.items[A.item_offset + li], A.src, s_red, s_last);
}

// Persistent fused step: A.steps steps of every member in one launch.  Each
// work-group takes tickets k = t * n_items + i in increasing order (item i in
// processing order, step t; buffers alternate with t).  Before item i of
// step t, thread 0 polls until the item's member has finalised step t - 1
// (its `fin` counter, reset to 0 before the launch), which the member's last
// work-group of that step raises after the step's data, scale and record.
// Every wait ends: the items waited on hold smaller tickets, taken by running
// work-groups, and the smallest unfinished ticket never waits on anything
// unfinished.  As a guard the poll gives up after A.spin_limit rounds,
// raising ctrl->abort, which every work-group checks: the launch then drains
// and the host reports the results invalid.
template <int DT, int VZ, int RY, int D, int BT, bool FV>
__global__ __launch_bounds__(BT, FDTD_STEP_MIN_WAVES) void k_step_persist(StepArgs A) {
  __shared__ double s_red[BT / 64][5];
  __shared__ int s_last;
  __shared__ int s_tk;
  const int tid = threadIdx.x;
  const int total = A.steps * A.n_items;
  for (;;) {
    if (tid == 0) {
      int tk = (int)atomicAdd(&A.ctrl->ticket, 1u);
      if (tk < total) {
        const unsigned need = (unsigned)(tk / A.n_items);
        unsigned int* fin = &A.states[A.items[tk % A.n_items].member].fin;
        unsigned polls = 0;
        while (__hip_atomic_load(fin, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
          if (__hip_atomic_load(&A.ctrl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
              ++polls > A.spin_limit) {
            __hip_atomic_store(&A.ctrl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            tk = total;
            break;
          }
          __builtin_amdgcn_s_sleep(4);
        }
      }
      s_tk = tk;
    }
    __syncthreads();
    const int tk = s_tk;
    if (tk >= total) break;
    const int t = tk / A.n_items;
    run_item<DT, VZ, RY, true, D, BT, FV, FDTD_AUX_OUT, true>(A, A.items[tk % A.n_items], A.src ^ (t & 1), s_red,
                                          s_last);
  }
}

// -------------------------------------- temporal blocking: two steps ----
// k_step2 advances every member two steps per pass over HBM (psi and V read
// once, psi'' written once).  A work item owns a tile of kTbRows(DT) x
// kTbCols(DT) sites of the (y, z) plane and streams x; each lane holds one
// vector of VZ consecutive z sites (a tile row is 256 bytes of F32 / F64; BF16
// lattices use the F32 tile, 4 sites per lane).
// Step t runs on the tile's own vectors and on a frame of single halo sites
// (the rows y0 - 1 and y0 + rows, the columns z0 - 1 and z0 + cols), with the
// loads and arithmetic of the one-step kernel; its results stay in registers
// (planes x - 1, x, x + 1 of the own vectors) and go to an LDS copy of the
// framed tile for the y / z neighbours.  Step t + 1 follows one plane behind,
// from registers and LDS.  Per-site arithmetic is that of the one-step
// kernel, so with the rescale off the states are the same bits; the
// reductions group their sums by tile instead of by flattened chunk (FP64
// summation order only).  Step t never rescales; step t + 1 takes a rescale
// due after either step.
// Work-group barrier fenced on LDS only: outstanding global loads (the
// prefetched planes) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// V of a tile's sites is read again as the halo frame of its neighbours, so
// the two-step kernel keeps V loads in the caches.
#ifndef FDTD_TB_AUX_V
#define FDTD_TB_AUX_V 0
#endif
constexpr int kTbVAux = FDTD_TB_AUX_V;

template <int DT, int VZ, int D, bool FV>
struct Step2 {
  static constexpr int BT = 256;
  static constexpr int TZ = kTbCols(DT);            // tile columns (z sites)
  static constexpr int LPR = TZ / VZ;               // lanes per tile row
  static constexpr int TY = BT / LPR;               // tile rows
  static constexpr int NH = 2 * TZ + 2 * TY;        // halo sites, one per lane
  static constexpr int NHW = (NH + 63) / 64;        // waves that carry halo sites
  static constexpr int RP = TZ + 8;                 // LDS row pitch: own z at 4 .. 4 + TZ - 1
  static constexpr int TS = (TY + 2) * RP;          // LDS plane: rows y0 - 1 .. y0 + TY
  static_assert(TY == kTbRows(DT) && TZ % VZ == 0, "tile shape");
  static_assert(NH <= BT, "one halo site per lane");
  using B = StepBody<DT, VZ, 1, true, FV>;  // own vectors
  using H = StepBody<DT, 1, 1, true, FV>;   // halo sites
  using C = typename B::C;

  struct Rings {
    C qs[6][1][VZ];          // psi_t of planes, own vectors
    C vs[6][1][VZ];          // V of planes
    PlaneIn<1, VZ, C> nb[6]; // y / z neighbours of psi_t planes
    C qh[6][1][1];           // the same for the lane's halo site
    C vh[6][1][1];
    PlaneIn<1, 1, C> nh[6];
    C us[3][1][VZ];          // step-t results, own vectors
  };

  // Stage X (slot SL = (X - base) % 6, base = xb - 1): prefetch, step t at
  // plane X into registers and LDS buffer X & 1, then (STEP2) step t + 1 at
  // plane X - 1, then the work-group barrier.
  template <int SL, bool STEP2>
  static __device__ __forceinline__ void stage(const typename B::Ctx& kb,
                                               const typename H::Ctx& kh,
                                               const typename B::Ctx& k2,
                                               const Lane<1, VZ, C>& lb, const Lane<1, 1, C>& lh,
                                               bool own, bool halo_wave, int obase, int hidx,
                                               int X, int xb, int xe, unsigned N, C* tile,
                                               Rings& g, double (&acc1)[5], double (&acc2)[5]) {
    B::fetch_own(kb, lb, X + 1 + D, g.qs[(SL + 2 + D) % 6]);
    B::template fetch_v<kTbVAux>(kb, lb, X + D, g.vs[(SL + D) % 6]);
    B::fetch(kb, lb, X + D, g.nb[(SL + D) % 6]);
    if (halo_wave) {
      H::fetch_own(kh, lh, X + 1 + D, g.qh[(SL + 2 + D) % 6]);
      H::template fetch_v<kTbVAux>(kh, lh, X + D, g.vh[(SL + D) % 6]);
      H::fetch(kh, lh, X + D, g.nh[(SL + D) % 6]);
    }
    // planes -1 and N lie outside the lattice: psi_{t+1} = 0 there (the
    // one-step kernel drops their stores; here they feed step t + 1)
    const bool inx = (unsigned)X < N;
    C* t = tile + (X & 1) * TS;
    {
      // step t, own vectors: the work item's planes [xb, xe) count in the
      // reductions, the halo planes xb - 1 and xe do not
      double tmp[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      C un[1][VZ];
      B::template update_core<false, true, 1>(kb, lb, X, g.qs[SL % 6], g.qs[(SL + 1) % 6],
                                              g.qs[(SL + 2) % 6], g.vs[SL % 6], g.nb[SL % 6],
                                              tmp, true, un);
      if (X >= xb && X < xe) {
#pragma unroll
        for (int q = 0; q < 5; ++q) acc1[q] += tmp[q];
      }
      Pack<C, VZ> pk;
#pragma unroll
      for (int j = 0; j < VZ; ++j) {
        pk.v[j] = inx ? un[0][j] : C(0);
        g.us[SL % 3][0][j] = pk.v[j];
      }
      *reinterpret_cast<Pack<C, VZ>*>(t + obase) = pk;
    }
    if (halo_wave) {
      // step t, halo site (no reductions: another work item owns it)
      double tmp[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      C uh[1][1];
      H::template update_core<false, true, 0>(kh, lh, X, g.qh[SL % 6], g.qh[(SL + 1) % 6],
                                              g.qh[(SL + 2) % 6], g.vh[SL % 6], g.nh[SL % 6],
                                              tmp, true, uh);
      if ((int)threadIdx.x < NH) t[hidx] = inx ? uh[0][0] : C(0);
    }
    if constexpr (STEP2) {
      // step t + 1 at plane X - 1: psi_{t+1} planes X - 2, X - 1, X in
      // registers, the y / z neighbours of plane X - 1 from LDS.  A vector
      // outside the lattice gets zero neighbours, as its loads in the
      // one-step kernel: its result is not stored, but it enters the norm.
      const C* tp = tile + ((X - 1) & 1) * TS;
      PlaneIn<1, VZ, C> d;
      const Pack<C, VZ> pm = *reinterpret_cast<const Pack<C, VZ>*>(tp + obase - RP);
      const Pack<C, VZ> pp = *reinterpret_cast<const Pack<C, VZ>*>(tp + obase + RP);
#pragma unroll
      for (int j = 0; j < VZ; ++j) {
        d.ym[0][j] = own ? pm.v[j] : C(0);
        d.yp[0][j] = own ? pp.v[j] : C(0);
      }
      d.zm[0] = own ? tp[obase - 1] : C(0);
      d.zp[0] = own ? tp[obase + VZ] : C(0);
      B::template update<false>(k2, lb, X - 1, g.us[(SL + 1) % 3], g.us[(SL + 2) % 3],
                                g.us[SL % 3], g.vs[(SL + 5) % 6], d, acc2);
    }
    lds_barrier();
  }
};

// Lane vector r of a temporally blocked work item: site f of the flattened
// plane (ok: a lattice site), with every offset the one-step loads use.
template <typename Body, int RYL, int VZ, typename C>
__device__ __forceinline__ void tb_lane(Lane<RYL, VZ, C>& ln, int r, unsigned f, bool ok,
                                        const MemberDev& M, int N, double cN, double ha) {
  constexpr unsigned kES = sizeof(typename Body::S);
  using TV = typename Body::TV;
  const unsigned fe = ok ? f : kDeadLane;
  const int y = ok ? (int)(f / (unsigned)N) : 0;
  const int z0 = ok ? (int)(f - (unsigned)y * N) : 0;
  ln.off[r] = fe * kES;
  ln.voff[r] = fe * (unsigned)sizeof(TV);
  ln.offm[r] = (fe - (unsigned)N) * kES;
  ln.offp[r] = (fe + (unsigned)N) * kES;
  ln.offzm[r] = fe * kES - kES;
  ln.offzp[r] = fe * kES + VZ * kES;
  ln.zmask_lo[r] = (ok && z0 > 0) ? 1.f : 0.f;
  ln.zmask_hi[r] = (ok && z0 + VZ < N) ? 1.f : 0.f;
  const double yc = (2.0 * y - cN) * ha;
  const int cy = min(y, N - 1 - y);
  uint32_t key[VZ];
#pragma unroll
  for (int j = 0; j < VZ; ++j) {
    const double zc = (2.0 * (z0 + j) - cN) * ha;
    ln.w2[r][j] = (C)(yc * yc + zc * zc);
    Body::vlane(ln, r, j, M.vkind, M.vp, M.a, yc, zc);
    const int z = z0 + j;
    key[j] = (uint32_t)cy * (uint32_t)N + (uint32_t)min(z, N - 1 - z);
  }
  Body::hash_lane(ln, r, N, key);
}

#ifndef FDTD_TB_MIN_WAVES
#define FDTD_TB_MIN_WAVES 1  // waves per SIMD the register budget must allow
#endif

template <int DT, int VZ, int D, bool FV>
__global__ __launch_bounds__(256, FDTD_TB_MIN_WAVES) void k_step2(StepArgs A) {
  using T = Step2<DT, VZ, D, FV>;
  using B = typename T::B;
  using H = typename T::H;
  using C = typename T::C;
  using TV = typename B::TV;
  constexpr int BT = 256;
  constexpr unsigned kES = sizeof(typename B::S);
  __shared__ __align__(16) C tile[2 * T::TS];
  __shared__ double s_red[BT / 64][5];
  __shared__ int s_last;
  const int tid = threadIdx.x;
  // the waves that carry halo sites (uniform per wave)
  const bool halo_wave = __builtin_amdgcn_readfirstlane(tid >> 6) < T::NHW;

  for (int li = blockIdx.x; li < A.n_items; li += gridDim.x) {
    const Item item = A.items[A.item_offset + li];
    const int m = item.member;
    const MemberDev& M = A.members[m];
    const int N = M.N;
    const unsigned P = (unsigned)M.plane;
    const double cN = (double)(N - 1), ha = M.ha;
    const long long step = ld_agent(A.states[m].step);
    const int y0 = item.f0 / N, z0 = item.f0 - y0 * N;  // tile origin

    typename B::Ctx kb;
    kb.in = M.psi[A.src];
    kb.out = M.psi[A.src ^ 1];  // unused: step t goes to registers
    kb.Vf = static_cast<const TV*>(M.V);
    kb.pbytes = P * kES;
    kb.vbytes = P * (unsigned)sizeof(TV);
    kb.N = N;
    kb.xe = item.xe + 1;  // step t also runs on plane xe (the halo plane)
    kb.c = (C)M.c;
    kb.dt = (C)M.dt;
    kb.eps = (C)(0.5 * M.dt);
    kb.sc = (C)ld_agent(A.states[m].scale);
    kb.ha = ha;
    kb.cN = cN;
    kb.smix = hash32((uint32_t)step);
    if constexpr (FV) B::vcoef(kb, M.vkind, M.vp, M.a);
    typename H::Ctx kh;
    kh.in = kb.in;
    kh.out = kb.out;
    kh.Vf = kb.Vf;
    kh.pbytes = kb.pbytes;
    kh.vbytes = kb.vbytes;
    kh.N = N;
    kh.xe = kb.xe;
    kh.c = kb.c;
    kh.dt = kb.dt;
    kh.eps = kb.eps;
    kh.sc = kb.sc;
    kh.ha = ha;
    kh.cN = cN;
    kh.smix = kb.smix;
    if constexpr (FV) H::vcoef(kh, M.vkind, M.vp, M.a);
    typename B::Ctx k2 = kb;
    k2.xe = item.xe;
    k2.sc = C(1);  // no rescale between the two steps of a pass
    k2.smix = hash32((uint32_t)(step + 1));

    // own vector: row tid / LPR, columns (tid % LPR) * VZ of the tile
    const int ly = tid / T::LPR, lz = (tid % T::LPR) * VZ;
    const int yo = y0 + ly, zo = z0 + lz;
    const bool own = yo < N && zo < N;
    const int obase = (ly + 1) * T::RP + 4 + lz;
    Lane<1, VZ, C> lb;
    tb_lane<B>(lb, 0, (unsigned)(yo * N + zo), own, M, N, cN, ha);
    // halo site of lanes below NH: row y0 - 1, row y0 + TY, column z0 - 1,
    // column z0 + TZ
    int hy, hz, hidx;
    if (tid < T::TZ) {
      hy = y0 - 1, hz = z0 + tid, hidx = 4 + tid;
    } else if (tid < 2 * T::TZ) {
      hy = y0 + T::TY, hz = z0 + tid - T::TZ, hidx = (T::TY + 1) * T::RP + 4 + tid - T::TZ;
    } else if (tid < 2 * T::TZ + T::TY) {
      hy = y0 + tid - 2 * T::TZ, hz = z0 - 1, hidx = (tid - 2 * T::TZ + 1) * T::RP + 3;
    } else {
      hy = y0 + tid - 2 * T::TZ - T::TY, hz = z0 + T::TZ;
      hidx = (tid - 2 * T::TZ - T::TY + 1) * T::RP + 4 + T::TZ;
    }
    const bool hok = tid < T::NH && hy >= 0 && hy < N && hz >= 0 && hz < N;
    Lane<1, 1, C> lh;
    tb_lane<H>(lh, 0, hok ? (unsigned)(hy * N + hz) : 0u, hok, M, N, cN, ha);

    double acc1[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, acc2[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    typename T::Rings g;
    const int xb = item.xb, xe = item.xe, base = xb - 1;
#pragma unroll
    for (int i = 0; i < D + 2; ++i) B::fetch_own(kb, lb, base - 1 + i, g.qs[i]);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      B::template fetch_v<kTbVAux>(kb, lb, base + i, g.vs[i]);
      B::fetch(kb, lb, base + i, g.nb[i]);
    }
    if (halo_wave) {
#pragma unroll
      for (int i = 0; i < D + 2; ++i) H::fetch_own(kh, lh, base - 1 + i, g.qh[i]);
#pragma unroll
      for (int i = 0; i < D; ++i) {
        H::template fetch_v<kTbVAux>(kh, lh, base + i, g.vh[i]);
        H::fetch(kh, lh, base + i, g.nh[i]);
      }
    }
#define FDTD_STAGE2(SL, S2, XX)                                                                  \
  T::template stage<SL, S2>(kb, kh, k2, lb, lh, own, halo_wave, obase, hidx, XX, xb, xe,         \
                            (unsigned)N, tile, g, acc1, acc2)
    // planes xb - 1 and xb: step t only; then both steps, six stages a trip
    FDTD_STAGE2(0, false, base);
    FDTD_STAGE2(1, false, base + 1);
    int X = xb + 1;
    for (; X + 6 <= xe + 1; X += 6) {
      FDTD_STAGE2(2, true, X);
      FDTD_STAGE2(3, true, X + 1);
      FDTD_STAGE2(4, true, X + 2);
      FDTD_STAGE2(5, true, X + 3);
      FDTD_STAGE2(0, true, X + 4);
      FDTD_STAGE2(1, true, X + 5);
    }
    if (X <= xe) FDTD_STAGE2(2, true, X);
    if (X + 1 <= xe) FDTD_STAGE2(3, true, X + 1);
    if (X + 2 <= xe) FDTD_STAGE2(4, true, X + 2);
    if (X + 3 <= xe) FDTD_STAGE2(5, true, X + 3);
    if (X + 4 <= xe) FDTD_STAGE2(0, true, X + 4);
#undef FDTD_STAGE2

    // ---- partials of both steps; the member's last work-group finalises them
    block_sum<5, BT / 64>(acc1, s_red);
    block_sum<5, BT / 64>(acc2, s_red);
    if (tid == 0) {
      double* p1 = A.partials + (long long)item.slot * kRec;
      double* p2 = A.partials + (long long)(A.slot_stride + item.slot) * kRec;
      double* const dst[2] = {p1, p2};
      const double v[2][5] = {{acc1[0], acc1[1], acc1[2], acc1[3], acc1[4]},
                              {acc2[0], acc2[1], acc2[2], acc2[3], acc2[4]}};
      const unsigned int done = publish_partials<2>(dst, v, &A.states[m].counter);
      s_last = (done + 1u == (unsigned int)(M.tb_end - M.tb_begin));
    }
    __syncthreads();
    if (s_last) {
      double t1[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, t2[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      for (int i = M.tb_begin + tid; i < M.tb_end; i += BT) {
        const double* p1 = A.partials + (long long)i * kRec;
        const double* p2 = A.partials + (long long)(A.slot_stride + i) * kRec;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          t1[q] += ld_agent(p1[q]);
          t2[q] += ld_agent(p2[q]);
        }
      }
      block_sum<5, BT / 64>(t1, s_red);
      block_sum<5, BT / 64>(t2, s_red);
      if (tid == 0) {
        finalize(A, M, m, t1, true, 0);  // never rescales: step t + 1 already ran
        finalize(A, M, m, t2, true, 1);
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------- fused step, LDS plane tiles ----
// Variant of k_step for large work-groups: each lane owns one vector of VZ
// sites, the work-group a chunk of kTB * VZ consecutive sites of the
// flattened (y, z) plane.  Planes stream along x as before (own sites of
// x-1, x, x+1 in a register ring, loads D planes ahead), but the y and z
// neighbours come from an LDS copy of plane x: the chunk plus one row above
// and below it (the halo rows, loaded by the first 2N/VZ lanes).  Two LDS
// buffers alternate between planes; one work-group barrier per plane, fenced
// on LDS only so the prefetched global loads stay in flight.  Per lane and
// plane this issues 2 (+1 halo) vector loads instead of 6, and keeps no
// neighbour registers, so 16 waves fit on a CU.
template <int DT>
struct TileShape {
  static constexpr int kTB = DT == kBF16 ? 512 : 1024;  // threads per work-group
};


template <int DT, int VZ, bool UPD, int D>
struct TileBody {
  using Body = StepBody<DT, VZ, 1, UPD>;
  using S = typename Body::S;
  using C = typename Body::C;
  using Ctx = typename Body::Ctx;

  static __device__ __forceinline__ void fetch_halo(const Ctx& k, int x, unsigned hoff,
                                                    C (&h)[VZ]) {
    const __amdgpu_buffer_rsrc_t r = plane_rsrc(k.in, x, min(k.N, k.xe + 1), k.pbytes);
    bload<S, VZ, C, FDTD_AUX_PSI>(r, hoff, h);
  }

  static __device__ __forceinline__ void put(C* tile, unsigned TS, int b, unsigned rel,
                                             bool has_halo, unsigned hidx, const C (&q)[1][VZ],
                                             const C (&h)[VZ]) {
    C* t = tile + (unsigned)b * TS;
    Pack<C, VZ> pq, ph;
#pragma unroll
    for (int j = 0; j < VZ; ++j) {
      pq.v[j] = q[0][j];
      ph.v[j] = h[j];
    }
    *reinterpret_cast<Pack<C, VZ>*>(t + rel) = pq;
    if (has_halo) *reinterpret_cast<Pack<C, VZ>*>(t + hidx) = ph;
  }

  // Update plane X from LDS buffer SL & 1, then stage plane X + 1 into the
  // other buffer.
  template <int SL>
  static __device__ __forceinline__ void stage(const Ctx& k, const Lane<1, VZ, C>& ln, int X,
                                               C* tile, unsigned TS, unsigned rel, bool has_halo,
                                               unsigned hidx, unsigned hoff, bool ok,
                                               C (&qs)[6][1][VZ], C (&vs)[6][1][VZ],
                                               C (&hs)[6][VZ], double (&acc)[5]) {
    constexpr int b = SL & 1;
    Body::fetch_own(k, ln, X + 1 + D, qs[(SL + 2 + D) % 6]);
    Body::fetch_v(k, ln, X + D, vs[(SL + D) % 6]);
    fetch_halo(k, X + 1 + D, hoff, hs[(SL + 2 + D) % 6]);
    PlaneIn<1, VZ, C> nb;
    const C* t = tile + (unsigned)b * TS;
    const unsigned N = (unsigned)k.N;
    const Pack<C, VZ> pm = *reinterpret_cast<const Pack<C, VZ>*>(t + rel - N);
    const Pack<C, VZ> pp = *reinterpret_cast<const Pack<C, VZ>*>(t + rel + N);
#pragma unroll
    for (int j = 0; j < VZ; ++j) {
      nb.ym[0][j] = pm.v[j];
      nb.yp[0][j] = pp.v[j];
    }
    nb.zm[0] = t[rel - 1];
    nb.zp[0] = t[rel + VZ];
    Body::template update<false>(k, ln, X, qs[SL % 6], qs[(SL + 1) % 6], qs[(SL + 2) % 6],
                                 vs[SL % 6], nb, acc, ok);
    put(tile, TS, b ^ 1, rel, has_halo, hidx, qs[(SL + 2) % 6], hs[(SL + 2) % 6]);
    lds_barrier();
  }
};

template <int DT, int VZ, bool UPD, int D>
__global__ __launch_bounds__(TileShape<DT>::kTB) void k_step_tile(StepArgs A) {
  using Body = StepBody<DT, VZ, 1, UPD>;
  using S = typename Body::S;
  using TV = typename Body::TV;
  using C = typename Body::C;
  constexpr int kTB = TileShape<DT>::kTB;
  constexpr unsigned kES = sizeof(S);
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_red[kTB / 64][5];
  __shared__ int s_last;
  const int tid = threadIdx.x;

  for (int li = blockIdx.x; li < A.n_items; li += gridDim.x) {
    const int it = A.item_offset + li;
    const Item item0 = A.items[it];
    Item item;
    item.member = uni(item0.member);
    item.f0 = uni(item0.f0);
    item.xb = uni(item0.xb);
    item.xe = uni(item0.xe);
    item.slot = uni(item0.slot);
    const int m = item.member;
    const MemberDev& M = A.members[m];
    const int N = uni(M.N);
    const unsigned P = uni((unsigned)M.plane);
    const unsigned F = (unsigned)kTB * VZ;
    const unsigned TS = F + 2u * (unsigned)N;  // tile elements per buffer
    C* tile = reinterpret_cast<C*>(smem);       // [2][TS]

    typename Body::Ctx k;
    k.in = uni(M.psi[A.src]);
    k.out = uni(M.psi[A.src ^ 1]);
    k.Vf = uni(static_cast<const TV*>(M.V));
    k.pbytes = P * kES;
    k.vbytes = P * (unsigned)sizeof(TV);
    k.N = N;
    k.c = (C)M.c;
    k.dt = (C)M.dt;
    k.eps = (C)(0.5 * M.dt);
    k.sc = (C)A.states[m].scale;
    k.ha = M.ha;
    k.cN = (double)(N - 1);
    k.smix = hash32((uint32_t)A.states[m].step);
    k.xe = item.xe;

    // own vector
    Lane<1, VZ, C> ln;
    const unsigned f = (unsigned)item.f0 + (unsigned)tid * VZ;
    const bool ok = f < P;
    {
      const unsigned fe = ok ? f : kDeadLane;
      const int y = ok ? (int)(f / (unsigned)N) : 0;
      const int z0 = ok ? (int)(f - (unsigned)y * N) : 0;
      ln.off[0] = fe * kES;
      ln.voff[0] = fe * (unsigned)sizeof(TV);
      ln.offm[0] = 0;
      ln.offp[0] = 0;
      ln.zmask_lo[0] = (ok && z0 > 0) ? 1.f : 0.f;
      ln.zmask_hi[0] = (ok && z0 + VZ < N) ? 1.f : 0.f;
      const double yc = (2.0 * y - k.cN) * k.ha;
      const int cy = min(y, N - 1 - y);
      uint32_t key[VZ];  // mirror-canonical (y, z) index
#pragma unroll
      for (int j = 0; j < VZ; ++j) {
        const double zc = (2.0 * (z0 + j) - k.cN) * k.ha;
        ln.w2[0][j] = (C)(yc * yc + zc * zc);
        const int z = z0 + j;
        key[j] = (uint32_t)cy * (uint32_t)N + (uint32_t)min(z, N - 1 - z);
      }
      Body::hash_lane(ln, 0, N, key);
    }
    const unsigned rel = (unsigned)tid * VZ + (unsigned)N;  // own vector in the tile
    // halo: lanes below 2N/VZ fetch one vector of the row above / below the chunk
    const unsigned nh = 2u * (unsigned)N / VZ;
    const bool has_halo = (unsigned)tid < nh;
    unsigned hoff = kDeadLane * kES, hidx = 0;
    if (has_halo) {
      const unsigned half = (unsigned)N / VZ;
      const bool above = (unsigned)tid < half;
      const unsigned t = above ? (unsigned)tid : (unsigned)tid - half;
      const unsigned hf = above ? (unsigned)item.f0 - (unsigned)N + t * VZ
                                : (unsigned)item.f0 + F + t * VZ;  // may wrap: out of range
      hoff = hf * kES;
      hidx = above ? t * VZ : F + (unsigned)N + t * VZ;
    }

    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    C qs[6][1][VZ], vs[6][1][VZ], hs[6][VZ];
    const int xb = item.xb, xe = item.xe;
    using TB = TileBody<DT, VZ, UPD, D>;
#pragma unroll
    for (int i = 0; i < D + 2; ++i) Body::fetch_own(k, ln, xb - 1 + i, qs[i]);
#pragma unroll
    for (int i = 1; i < D + 2; ++i) TB::fetch_halo(k, xb - 1 + i, hoff, hs[i]);
#pragma unroll
    for (int i = 0; i < D; ++i) Body::fetch_v(k, ln, xb + i, vs[i]);
    TB::put(tile, TS, 0, rel, has_halo, hidx, qs[1], hs[1]);
    lds_barrier();
    int x = xb;
    for (; x + 6 <= xe; x += 6) {
      TB::template stage<0>(k, ln, x, tile, TS, rel, has_halo, hidx, hoff, ok, qs, vs, hs, acc);
      TB::template stage<1>(k, ln, x + 1, tile, TS, rel, has_halo, hidx, hoff, ok, qs, vs, hs, acc);
      TB::template stage<2>(k, ln, x + 2, tile, TS, rel, has_halo, hidx, hoff, ok, qs, vs, hs, acc);
      TB::template stage<3>(k, ln, x + 3, tile, TS, rel, has_halo, hidx, hoff, ok, qs, vs, hs, acc);
      TB::template stage<4>(k, ln, x + 4, tile, TS, rel, has_halo, hidx, hoff, ok, qs, vs, hs, acc);
      TB::template stage<5>(k, ln, x + 5, tile, TS, rel, has_halo, hidx, hoff, ok, qs, vs, hs, acc);
    }
    // tail: x is uniform, so every lane takes the same branches (barriers)
    if (x < xe) TB::template stage<0>(k, ln, x, tile, TS, rel, has_halo, hidx, hoff, ok, qs, vs, hs, acc);
    if (x + 1 < xe) TB::template stage<1>(k, ln, x + 1, tile, TS, rel, has_halo, hidx, hoff, ok, qs, vs, hs, acc);
    if (x + 2 < xe) TB::template stage<2>(k, ln, x + 2, tile, TS, rel, has_halo, hidx, hoff, ok, qs, vs, hs, acc);
    if (x + 3 < xe) TB::template stage<3>(k, ln, x + 3, tile, TS, rel, has_halo, hidx, hoff, ok, qs, vs, hs, acc);
    if (x + 4 < xe) TB::template stage<4>(k, ln, x + 4, tile, TS, rel, has_halo, hidx, hoff, ok, qs, vs, hs, acc);

    block_sum<5, kTB / 64>(acc, s_red);
    if (tid == 0) {
      double* part = A.partials + (long long)item.slot * kRec;
      double* const dst[1] = {part};
      const double v[1][5] = {{acc[0], acc[1], acc[2], acc[3], acc[4]}};
      const unsigned int done = publish_partials<1>(dst, v, &A.states[m].counter);
      s_last = (done + 1u == (unsigned int)(M.item_end - M.item_begin));
    }
    __syncthreads();
    if (s_last) {
      double tot[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      for (int i = M.item_begin + tid; i < M.item_end; i += kTB) {
        const double* part = A.partials + (long long)i * kRec;
#pragma unroll
        for (int kk = 0; kk < 5; ++kk) tot[kk] += ld_agent(part[kk]);
      }
      block_sum<5, kTB / 64>(tot, s_red);
      if (tid == 0) finalize(A, M, m, tot, UPD);
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------- potentials ----
// Regular dodecahedron of Sec. VII.E in lattice units u = x / ((N - 1) a / 2)
// (the first and last sites of each axis at u = -1 and 1): vertices
// (+-1, +-1, +-1)/phi, (0, +-1/phi^2, +-1), (+-1/phi^2, +-1, 0),
// (+-1, 0, +-1/phi^2); faces perpendicular to (0, +-phi, +-1), (+-1, 0, +-phi),
// (+-phi, +-1, 0), each at the largest projection of the vertices on its unit
// normal.  Closed, with a relative slack of 1e-12 so that sites exactly on a
// face are inside whatever the last bit; FP64 without fused multiply-adds.
__device__ bool dodeca_inside(double ux, double uy, double uz) {
#pragma clang fp contract(off)
  const double phi = 0.5 * (1.0 + sqrt(5.0));
  const double ip = 1.0 / phi, ip2 = 1.0 / (phi * phi);
  double vtx[20][3];
  int nv = 0;
  for (int sx = -1; sx <= 1; sx += 2)
    for (int sy = -1; sy <= 1; sy += 2)
      for (int sz = -1; sz <= 1; sz += 2) {
        vtx[nv][0] = sx * ip;
        vtx[nv][1] = sy * ip;
        vtx[nv][2] = sz * ip;
        ++nv;
      }
  for (int s1 = -1; s1 <= 1; s1 += 2)
    for (int s2 = -1; s2 <= 1; s2 += 2) {
      vtx[nv][0] = 0.0; vtx[nv][1] = s1 * ip2; vtx[nv][2] = s2 * 1.0; ++nv;
      vtx[nv][0] = s1 * ip2; vtx[nv][1] = s2 * 1.0; vtx[nv][2] = 0.0; ++nv;
      vtx[nv][0] = s1 * 1.0; vtx[nv][1] = 0.0; vtx[nv][2] = s2 * ip2; ++nv;
    }
  const double nrm[6][3] = {{0, phi, 1}, {0, phi, -1}, {1, 0, phi},
                            {-1, 0, phi}, {phi, 1, 0}, {phi, -1, 0}};
  for (int f = 0; f < 6; ++f) {
    const double len = sqrt(nrm[f][0] * nrm[f][0] + nrm[f][1] * nrm[f][1] + nrm[f][2] * nrm[f][2]);
    double d = 0.0;
    for (int v = 0; v < 20; ++v) {
      const double pr = (vtx[v][0] * nrm[f][0] + vtx[v][1] * nrm[f][1] + vtx[v][2] * nrm[f][2]) / len;
      d = pr > d ? pr : d;
    }
    const double q = (ux * nrm[f][0] + uy * nrm[f][1] + uz * nrm[f][2]) / len;
    if (fabs(q) > d * (1.0 + 1e-12)) return false;
  }
  return true;
}

template <typename TV>
__global__ __launch_bounds__(kBlock) void k_potential(TV* __restrict__ V, int N, double ha,
                                                      double a, int kind,
                                                      const double* __restrict__ p, int np) {
  const long long n3 = (long long)N * N * N;
  const double cN = (double)(N - 1);
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n3;
       s += (long long)gridDim.x * blockDim.x) {
    const int iz = (int)(s % N);
    const long long q = s / N;
    const int iy = (int)(q % N);
    const int ix = (int)(q / N);
    const double x = (2.0 * ix - cN) * ha, y = (2.0 * iy - cN) * ha, z = (2.0 * iz - cN) * ha;
    const double r = sqrt(x * x + y * y + z * z);
    double v = 0.0;
    switch (kind) {
      case 0: v = p[0]; break;
      case 1: v = 0.5 * (p[0] * p[0] * x * x + p[1] * p[1] * y * y + p[2] * p[2] * z * z); break;
      case 2: v = -p[0] / r; break;
      case 3: v = (r < a) ? 0.0 : (-p[0] / r + p[0] / a); break;
      case 4: v = -p[0] / r + p[1] * r + p[2] * z * z; break;
      case 5: {
        v = 0.5 * (p[0] * p[0] * x * x + p[1] * p[1] * y * y + p[2] * p[2] * z * z);
        for (int k = 3; k + 4 < np; k += 5) {
          const double dx = x - p[k + 1], dy = y - p[k + 2], dz = z - p[k + 3];
          const double d2 = dx * dx + dy * dy + dz * dz;
          v -= p[k] * exp(-d2 / (2.0 * p[k + 4] * p[k + 4]));
        }
        break;
      }
      case 6: {
        const double half = 0.5 * (double)(N - 1) * a;
        v = (N > 1 && dodeca_inside(x / half, y / half, z / half)) ? p[0] : 0.0;
        break;
      }
      default: v = 0.0;
    }
    V[s] = (TV)v;
  }
}

// -------------------------------------------------------- initial state ----
__device__ __forceinline__ uint64_t splitmix(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double unit53(uint64_t r) {
  return (double)(r >> 11) * (1.0 / 9007199254740992.0);
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_initial(S* __restrict__ psi, int N, uint64_t seed,
                                                    uint32_t member, int kind, uint32_t parity) {
  const long long n3 = (long long)N * N * N;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n3;
       s += (long long)gridDim.x * blockDim.x) {
    int c[3];
    c[2] = (int)(s % N);
    const long long q = s / N;
    c[1] = (int)(q % N);
    c[0] = (int)(q / N);
    double sign = 1.0;
    bool zero = false;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const uint32_t mode = (parity >> (2 * ax)) & 3u;
      if (mode == 0u) continue;
      const int mir = N - 1 - c[ax];
      if (c[ax] > mir) {  // upper half takes the value of its mirror site
        c[ax] = mir;
        if (mode == 2u) sign = -sign;
      } else if (c[ax] == mir && mode == 2u) {
        zero = true;
      }
    }
    const long long src = ((long long)c[0] * N + c[1]) * N + c[2];
    const uint64_t ctr = ((uint64_t)member << 36) + 2ull * (uint64_t)src;
    double val;
    if (kind == 0) {
      val = 2.0 * unit53(splitmix(seed, ctr)) - 1.0;
    } else {
      const double u1 = unit53(splitmix(seed, ctr)) + 1.0 / 9007199254740992.0;
      const double u2 = unit53(splitmix(seed, ctr + 1ull));
      val = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
    }
    val = zero ? 0.0 : sign * val;
    if constexpr (sizeof(S) == 2) psi[s] = f32_to_bf16((float)val);
    else psi[s] = (S)val;
  }
}

// ----------------------------------------------------------- conversion ----
template <typename SS, typename DS>
__global__ __launch_bounds__(kBlock) void k_convert(const SS* __restrict__ src,
                                                    DS* __restrict__ dst, long long n,
                                                    double scale) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double v;
    if constexpr (sizeof(SS) == 2) v = (double)bf16_to_f32(src[i]);
    else v = (double)src[i];
    v *= scale;
    if constexpr (sizeof(DS) == 2) dst[i] = f32_to_bf16((float)v);
    else dst[i] = (DS)v;
  }
}

// ------------------------------------------------------------- upsample ----
template <typename CS>
__device__ __forceinline__ double fetch_c(const CS* __restrict__ pc, int N, int x, int y, int z) {
  if (x < 0 || y < 0 || z < 0 || x >= N || y >= N || z >= N) return 0.0;  // ghost
  const CS v = pc[((long long)x * N + y) * N + z];
  if constexpr (sizeof(CS) == 2) return (double)bf16_to_f32(v);
  else return (double)v;
}

// Trilinear spread of a coarse state onto a finer lattice of the same box
// (Sec. VI).  Interpolates along z, then y, then x; each 1-d step adds the
// two weighted ends, so mirrored fine sites see the same sums.
// A thread owns kUpVZ consecutive fine z sites of one fine row y and streams
// kUpXC fine planes.  The (z, y) interpolation of a coarse plane at the
// thread's sites does not depend on the fine x, so it is formed once per
// coarse plane and serves every fine plane between that coarse plane and the
// next: a fine site then costs one lerp along x (and, at a 2x ratio, half of
// a plane's two z lerps and one y lerp).  The fine coordinate of an axis maps
// into coarse index space as ((2 j - (Nf - 1)) haf) / ac + (Nc - 1) / 2; the
// plane weights of the block's x-range are formed once, in LDS.
constexpr int kUpVZ = 4;   // fine z sites per thread
constexpr int kUpXC = 32;  // fine planes per thread

// Fine index j of an axis -> lower coarse index i0 and the weights of coarse
// sites i0 (wlo) and i0 + 1 (whi).  The map is evaluated at the
// mirror-canonical index min(j, Nf - 1 - j); the mirrored half takes the
// mirrored coarse pair with the two weights swapped, so sites j and
// Nf - 1 - j add the same two products: the interpolation maps a mirror-odd
// (even) state to a mirror-odd (even) one bit for bit, whatever the spacings
// (the sums (Nc - 1) / 2 + u and (Nc - 1) / 2 - u need not round alike).
__device__ __forceinline__ void up_weight(int j, int Nf, int Nc, double cNf, double haf, double ac,
                                          double halfc, int& i0, double& wlo, double& whi) {
  const int jm = min(j, Nf - 1 - j);
  const double t = ((2.0 * jm - cNf) * haf) / ac + halfc;
  const double fl = floor(t);
  const double w = t - fl;
  if (j == jm) {
    i0 = (int)fl;
    wlo = 1.0 - w;
    whi = w;
  } else {
    i0 = Nc - 2 - (int)fl;
    wlo = w;
    whi = 1.0 - w;
  }
}

// Coarse planes whose loads a thread issues together (FP64 coarse states:
// half as many, for registers).
#ifndef FDTD_UP_GROUP
#define FDTD_UP_GROUP 4
#endif

// PAIR: a BF16 coarse lattice of even side under a fine side at least twice
// as large.  A thread's coarse z indices then lie within six consecutive
// values from an even start, read as three dwords per coarse row (a dword
// holds an aligned pair of sites and never straddles a row), 6 loads per
// coarse plane instead of 16 single-site loads.  Single-site loads are what
// bound the kernel: they keep the texture addresser busy.
template <typename CS, typename FS, bool PAIR>
__global__ __launch_bounds__(kBlock) void k_upsample(const CS* __restrict__ pc, int Nc, double ac,
                                                     FS* __restrict__ pf, int Nf, double haf) {
  static_assert(!PAIR || sizeof(CS) == 2, "pair loads are for BF16 coarse states");
  __shared__ int s_i0[kUpXC];
  __shared__ double s_w[kUpXC], s_w1[kUpXC];  // weights of coarse planes i0 + 1, i0
  const double cNf = (double)(Nf - 1), halfc = 0.5 * (double)(Nc - 1);
  const int x0 = blockIdx.y * kUpXC;
  const int nx = min(kUpXC, Nf - x0);
  if ((int)threadIdx.x < nx) {
    int i0;
    double wlo, whi;
    up_weight(x0 + threadIdx.x, Nf, Nc, cNf, haf, ac, halfc, i0, wlo, whi);
    s_i0[threadIdx.x] = i0;
    s_w[threadIdx.x] = whi;
    s_w1[threadIdx.x] = wlo;
  }
  __syncthreads();
  const int nzv = (Nf + kUpVZ - 1) / kUpVZ;
  const long long col = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= (long long)Nf * nzv) return;
  const int y = (int)(col / nzv);
  const int z0 = (int)(col - (long long)y * nzv) * kUpVZ;
  int iy, iz[kUpVZ];
  double wy, wy1, wz[kUpVZ], wz1[kUpVZ];
  up_weight(y, Nf, Nc, cNf, haf, ac, halfc, iy, wy1, wy);
#pragma unroll
  for (int j = 0; j < kUpVZ; ++j)
    up_weight(min(z0 + j, Nf - 1), Nf, Nc, cNf, haf, ac, halfc, iz[j], wz1[j], wz[j]);
  // (z, y) interpolation of coarse plane c at the thread's sites.  Plane c
  // is one buffer resource (empty outside the lattice); a coarse site whose
  // row or column lies outside the lattice gets an offset past the plane.
  // Both read 0: the zero ghosts cost no branches and no traffic.
  const unsigned dead = kDeadLane * (unsigned)sizeof(CS);
  unsigned off[2][kUpVZ][2];
#pragma unroll
  for (int cy = 0; cy < 2; ++cy) {
    const int yy = iy + cy;
#pragma unroll
    for (int j = 0; j < kUpVZ; ++j)
#pragma unroll
      for (int cz = 0; cz < 2; ++cz) {
        const int zz = iz[j] + cz;
        const bool ok = yy >= 0 && yy < Nc && zz >= 0 && zz < Nc;
        off[cy][j][cz] = ok ? (unsigned)(yy * Nc + zz) * (unsigned)sizeof(CS) : dead;
      }
  }
  const unsigned pbytes = (unsigned)Nc * (unsigned)Nc * (unsigned)sizeof(CS);
  // PAIR: dword m of row cy holds coarse sites zs + 2m, zs + 2m + 1; site j
  // takes its two coarse values at dz[j], dz[j] + 1 of those six (<= 4 + 1:
  // the fine sites of a thread span at most 1.5 coarse spacings)
  unsigned poff[2][3];
  int dz[kUpVZ];
  if constexpr (PAIR) {
    const int zs = iz[0] - (iz[0] & 1);  // down to even (iz[0] >= -1)
#pragma unroll
    for (int cy = 0; cy < 2; ++cy) {
      const int yy = iy + cy;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const int zz = zs + 2 * m;  // even: the pair lies wholly inside or outside [0, Nc)
        const bool ok = yy >= 0 && yy < Nc && zz >= 0 && zz < Nc;
        poff[cy][m] = ok ? (unsigned)(yy * Nc + zz) * 2u : dead;
      }
    }
#pragma unroll
    for (int j = 0; j < kUpVZ; ++j) dz[j] = iz[j] - zs;
  }
  // coarse values as loaded (FP64 coarse states stay FP64)
  using CE = typename std::conditional<sizeof(CS) == 8, double, float>::type;
  // loads of coarse plane c at the thread's sites, and their (z, y) lerps
  auto load_plane = [&](int c, CE (&e)[2][kUpVZ][2]) {
    const __amdgpu_buffer_rsrc_t rp = plane_rsrc(pc, c, Nc, pbytes);
    if constexpr (PAIR) {
#pragma unroll
      for (int cy = 0; cy < 2; ++cy) {
        float v[6];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const unsigned wd = __builtin_amdgcn_raw_buffer_load_b32(rp, (int)poff[cy][m], 0, 0);
          v[2 * m] = __uint_as_float(wd << 16);
          v[2 * m + 1] = __uint_as_float(wd & 0xffff0000u);
        }
#pragma unroll
        for (int j = 0; j < kUpVZ; ++j)
#pragma unroll
          for (int cz = 0; cz < 2; ++cz) {
            const int k = dz[j] + cz;
            float r = v[0];
#pragma unroll
            for (int q = 1; q < 6; ++q) r = k == q ? v[q] : r;
            e[cy][j][cz] = r;
          }
      }
    } else {
#pragma unroll
      for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int j = 0; j < kUpVZ; ++j)
#pragma unroll
          for (int cz = 0; cz < 2; ++cz) {
            CE q[1];
            bload<CS, 1, CE>(rp, off[cy][j][cz], q);
            e[cy][j][cz] = q[0];
          }
    }
  };
  auto interp = [&](const CE (&e)[2][kUpVZ][2], double (&o)[kUpVZ]) {
    double v[2][kUpVZ];
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int j = 0; j < kUpVZ; ++j)
        v[cy][j] = wz1[j] * (double)e[cy][j][0] + wz[j] * (double)e[cy][j][1];
#pragma unroll
    for (int j = 0; j < kUpVZ; ++j) o[j] = wy1 * v[0][j] + wy * v[1][j];
  };
  // A window of G + 1 consecutive coarse planes, base .. base + G (w[k] is
  // plane base + k), advanced G planes at a time: the loads of the G new
  // planes are issued together, one memory round trip per G coarse planes.
  // Fine planes are emitted in order; fine plane i lies between coarse
  // planes s_i0[i] and s_i0[i] + 1 (non-decreasing in i; uniform).
  constexpr int G = sizeof(CE) == 8 ? (FDTD_UP_GROUP + 1) / 2 : FDTD_UP_GROUP;
  const bool full = z0 + kUpVZ <= Nf && (Nf % kUpVZ) == 0;
  auto emit = [&](int i, const double (&lo)[kUpVZ], const double (&hi)[kUpVZ]) {
    const double wx = s_w[i], wx1 = s_w1[i];
    Pack<FS, kUpVZ> o;
#pragma unroll
    for (int j = 0; j < kUpVZ; ++j) {
      const double v = wx1 * lo[j] + wx * hi[j];
      if constexpr (sizeof(FS) == 2) o.v[j] = f32_to_bf16((float)v);
      else o.v[j] = (FS)v;
    }
    FS* dst = pf + ((long long)(x0 + i) * Nf + y) * Nf + z0;
    if (full) {
      *reinterpret_cast<Pack<FS, kUpVZ>*>(dst) = o;
    } else {
#pragma unroll
      for (int j = 0; j < kUpVZ; ++j)
        if (z0 + j < Nf) dst[j] = o.v[j];
    }
  };
  double w[G + 1][kUpVZ];
  int base = uni(s_i0[0]);  // the block's planes: uniform
  {
    CE e[G + 1][2][kUpVZ][2];
#pragma unroll
    for (int k = 0; k <= G; ++k) load_plane(base + k, e[k]);
#pragma unroll
    for (int k = 0; k <= G; ++k) interp(e[k], w[k]);
  }
  int i = 0;
  while (true) {
#pragma unroll
    for (int k = 0; k < G; ++k)
      while (i < nx && uni(s_i0[i]) == base + k) {
        emit(i, w[k], w[k + 1]);
        ++i;
      }
    if (i >= nx) break;
    base += G;
#pragma unroll
    for (int j = 0; j < kUpVZ; ++j) w[0][j] = w[G][j];
    CE e[G][2][kUpVZ][2];
#pragma unroll
    for (int k = 0; k < G; ++k) load_plane(base + 1 + k, e[k]);
#pragma unroll
    for (int k = 0; k < G; ++k) interp(e[k], w[k + 1]);
  }
}

// ----------------------------------------------------- parity reimposed ----
template <typename S>
__global__ __launch_bounds__(kBlock) void k_reimpose(S* __restrict__ psi, int N, uint32_t parity) {
  const long long n3 = (long long)N * N * N;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n3;
       s += (long long)gridDim.x * blockDim.x) {
    int c[3];
    c[2] = (int)(s % N);
    const long long q = s / N;
    c[1] = (int)(q % N);
    c[0] = (int)(q / N);
    bool neg = false, zero = false, moved = false;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const uint32_t mode = (parity >> (2 * ax)) & 3u;
      if (mode == 0u) continue;
      const int mir = N - 1 - c[ax];
      if (c[ax] > mir) {
        c[ax] = mir;
        moved = true;
        if (mode == 2u) neg = !neg;
      } else if (c[ax] == mir && mode == 2u) {
        zero = true;
      }
    }
    if (zero) {
      psi[s] = S(0);
    } else if (moved) {
      // the source lies in the lower half of every masked axis: never written here
      const S v = psi[((long long)c[0] * N + c[1]) * N + c[2]];
      if constexpr (sizeof(S) == 2) psi[s] = neg ? (uint16_t)(v ^ 0x8000u) : v;
      else psi[s] = neg ? -v : v;
    }
  }
}

__global__ void k_set_state(MemberState* st, int member, double scale, long long step,
                            int reset_bad) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    MemberState& s = st[member];
    s.scale = scale;
    s.step = step;
    s.counter = 0u;
    if (reset_bad) {
      s.bad = 0;
      s.bad_step = -1;
    }
  }
}

// -------------------------------------------------------------- adjoint ----
// One step of the adjoint recurrence of the renormalised update
// psi_{t+1} = s_t M psi_t,  M = I + diag(B) (c Lap - dt diag(V)):
//   lambda_t = s_t M^T lambda_{t+1},
//   (M^T l)_j = l_j + c (Lap w)_j - dt V_j w_j,   w = B l,
//   G_j += lambda_{t+1,j} (-(dt/2) B_j) (s_t psi_{t,j} + psi_{t+1,j}),
// the last line being d psi_{t+1,j} / dV_j (through A_j and B_j) times the
// adjoint.  Streamed along x like the forward step: a work item is a chunk of
// 256 x VZ consecutive sites of the flattened (y, z) plane and an x-range;
// each lane keeps w of its sites for planes x - 1, x, x + 1 in registers (so
// lambda and V come from HBM once), and forms the y / z neighbours' w from
// loads the adjacent rows and lanes also make (served by L1 / L2).  Out-of-
// range loads read 0 (zero ghosts).  Per site: lambda, V, psi_t, psi_{t+1}
// and G read, lambda_t and G written.
template <typename S, int VZ, int BT>
__global__ __launch_bounds__(BT) void k_adjoint_step(AdjArgs a) {
  using C = typename std::conditional<sizeof(S) == 8, double, float>::type;
  constexpr unsigned kES = sizeof(S);
  const int N = a.N;
  const unsigned P = (unsigned)N * (unsigned)N, pb = P * kES;
  const unsigned F = (unsigned)BT * VZ;
  const int nchunk = (int)((P + F - 1) / F), nx = a.nx;
  const C c = (C)a.c, dt = (C)a.dt, eps = (C)(0.5 * a.dt), st = (C)a.s_t;
  const double hdt = -0.5 * a.dt, std_ = (double)st;
  const int tid = threadIdx.x;
  auto wof = [&](C l, C v) -> C { return l * rcp_c(C(1) + eps * v); };
  for (int it = blockIdx.x; it < nchunk * nx; it += gridDim.x) {
    const int ch = it % nchunk, xr = it / nchunk;
    const int xb = (int)(((long long)xr * N) / nx), xe = (int)(((long long)(xr + 1) * N) / nx);
    const unsigned f = (unsigned)ch * F + (unsigned)tid * VZ;
    const bool ok = f < P;
    const unsigned fe = ok ? f : kDeadLane;
    const int y = ok ? (int)(f / (unsigned)N) : 0;
    const int z0 = ok ? (int)(f - (unsigned)y * N) : 0;
    const bool zlo = ok && z0 > 0, zhi = ok && z0 + VZ < N;
    const unsigned off = fe * kES, offm = (fe - (unsigned)N) * kES, offp = (fe + (unsigned)N) * kES;
    const unsigned offzm = fe * kES - kES, offzp = fe * kES + VZ * kES;
    // w of the lane's sites on planes x - 1 (wm) and x (wc); lambda, V on x
    C wm[VZ], wc[VZ], lc[VZ], vc[VZ];
    {
      C l0[VZ], v0[VZ];
      bload<S, VZ, C>(plane_rsrc(a.lam_in, xb - 1, N, pb), off, l0);
      bload<S, VZ, C>(plane_rsrc(a.V, xb - 1, N, pb), off, v0);
      bload<S, VZ, C>(plane_rsrc(a.lam_in, xb, N, pb), off, lc);
      bload<S, VZ, C>(plane_rsrc(a.V, xb, N, pb), off, vc);
#pragma unroll
      for (int j = 0; j < VZ; ++j) {
        wm[j] = wof(l0[j], v0[j]);
        wc[j] = wof(lc[j], vc[j]);
      }
    }
    for (int x = xb; x < xe; ++x) {
      C lp[VZ], vp[VZ], lym[VZ], vym[VZ], lyp[VZ], vyp[VZ], pt[VZ], pt1[VZ];
      C lzm[1], vzm[1], lzp[1], vzp[1];
      const __amdgpu_buffer_rsrc_t rl1 = plane_rsrc(a.lam_in, x + 1, N, pb);
      const __amdgpu_buffer_rsrc_t rv1 = plane_rsrc(a.V, x + 1, N, pb);
      const __amdgpu_buffer_rsrc_t rl = plane_rsrc(a.lam_in, x, N, pb);
      const __amdgpu_buffer_rsrc_t rv = plane_rsrc(a.V, x, N, pb);
      bload<S, VZ, C>(rl1, off, lp);
      bload<S, VZ, C>(rv1, off, vp);
      bload<S, VZ, C>(rl, offm, lym);
      bload<S, VZ, C>(rv, offm, vym);
      bload<S, VZ, C>(rl, offp, lyp);
      bload<S, VZ, C>(rv, offp, vyp);
      bload<S, 1, C>(rl, offzm, lzm);
      bload<S, 1, C>(rv, offzm, vzm);
      bload<S, 1, C>(rl, offzp, lzp);
      bload<S, 1, C>(rv, offzp, vzp);
      // read once and written once: past the caches, which keep lambda and V
      // for the neighbour re-reads
      bload<S, VZ, C, kNT>(plane_rsrc(a.psi_t, x, N, pb), off, pt);
      bload<S, VZ, C, kNT>(plane_rsrc(a.psi_t1, x, N, pb), off, pt1);
      const __amdgpu_buffer_rsrc_t rg = plane_rsrc(a.G, x, N, P * 8u);
      double gv[VZ];
      bload<double, VZ, double, kNT>(rg, fe * 8u, gv);
      C wp[VZ];
      Pack<S, VZ> o;
#pragma unroll
      for (int j = 0; j < VZ; ++j) wp[j] = wof(lp[j], vp[j]);
      const C wzl = zlo ? wof(lzm[0], vzm[0]) : C(0), wzr = zhi ? wof(lzp[0], vzp[0]) : C(0);
#pragma unroll
      for (int j = 0; j < VZ; ++j) {
        const C w = wc[j];
        const C wym = wof(lym[j], vym[j]), wyp = wof(lyp[j], vyp[j]);
        const C wzm = j > 0 ? wc[j - 1] : wzl, wzp = j < VZ - 1 ? wc[j + 1] : wzr;
        const C lapw = (((wm[j] - w) + (wp[j] - w)) + ((wym - w) + (wyp - w))) + ((wzm - w) + (wzp - w));
        o.v[j] = (S)(st * (lc[j] + c * lapw - dt * vc[j] * w));
        const C B = rcp_c(C(1) + eps * vc[j]);
        gv[j] += (double)lc[j] * (hdt * (double)B) * (std_ * (double)pt[j] + (double)pt1[j]);
      }
      bstore<S, VZ, kNT>(plane_rsrc(a.lam_out, x, N, pb), off, o);
      Pack<double, VZ> go;
#pragma unroll
      for (int j = 0; j < VZ; ++j) go.v[j] = gv[j];
      bstore<double, VZ, kNT>(rg, fe * 8u, go);
#pragma unroll
      for (int j = 0; j < VZ; ++j) {
        wm[j] = wc[j];
        wc[j] = wp[j];
        lc[j] = lp[j];
        vc[j] = vp[j];
      }
    }
  }
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_adjoint_init(AdjInitArgs a) {
  const S* __restrict__ V = static_cast<const S*>(a.V);
  const S* __restrict__ p = static_cast<const S*>(a.psi);
  S* __restrict__ lam = static_cast<S*>(a.lam);
  const int N = a.N;
  const long long P = (long long)N * N, n3 = P * N;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n3;
       s += (long long)gridDim.x * blockDim.x) {
    const int iz = (int)(s % N);
    const long long q = s / N;
    const int iy = (int)(q % N);
    const int ix = (int)(q / N);
    const double c0 = (double)p[s];
    auto at = [&](bool okk, long long k) -> double { return okk ? (double)p[k] : 0.0; };
    const double lap = (((at(ix > 0, s - P) - c0) + (at(ix < N - 1, s + P) - c0)) +
                        ((at(iy > 0, s - N) - c0) + (at(iy < N - 1, s + N) - c0))) +
                       ((at(iz > 0, s - 1) - c0) + (at(iz < N - 1, s + 1) - c0));
    const double hp = -a.kin_scale * lap + (double)V[s] * c0;
    lam[s] = (S)(2.0 * (hp - a.E * c0) / a.S0);
    a.G[s] = c0 * c0 / a.S0;
  }
}

// Contraction of dE/dV with the analytic derivatives of the potential's
// parameters (kinds numbered as in k_potential, which defines each V):
//   CONST 1; HO p_d x_d^2; COULOMB -1/r; COULOMB_REG 1/a - 1/r (0 for r < a);
//   CORNELL -1/r, r, z^2; WELLS p_d x_d^2 for the oscillator (j < 3), and for
//   well k with e = exp(-d^2 / 2 s^2): A -e, centre c_d -A e (x_d - c_d) / s^2,
//   width s -A e d^2 / s^3; DODECA 1 inside the solid.
constexpr int kMaxWrt = 64;

__device__ __forceinline__ double param_dv(int kind, const double* __restrict__ p, int j,
                                           const double (&xs)[3], double r, double a, int N,
                                           double half) {
  switch (kind) {
    case 0: return 1.0;
    case 1: return p[j] * xs[j] * xs[j];
    case 2: return -1.0 / r;
    case 3: return (r < a) ? 0.0 : (1.0 / a - 1.0 / r);
    case 4: return j == 0 ? -1.0 / r : (j == 1 ? r : xs[2] * xs[2]);
    case 5: {
      if (j < 3) return p[j] * xs[j] * xs[j];
      const double* w = p + 3 + 5 * ((j - 3) / 5);
      const int q = (j - 3) % 5;
      const double dx = xs[0] - w[1], dy = xs[1] - w[2], dz = xs[2] - w[3];
      const double d2 = dx * dx + dy * dy + dz * dz;
      const double e = exp(-d2 / (2.0 * w[4] * w[4]));
      if (q == 0) return -e;
      if (q == 4) return -w[0] * e * d2 / (w[4] * w[4] * w[4]);
      return -w[0] * e * (xs[q - 1] - w[q]) / (w[4] * w[4]);
    }
    case 6: return (N > 1 && dodeca_inside(xs[0] / half, xs[1] / half, xs[2] / half)) ? 1.0 : 0.0;
    default: return 0.0;
  }
}

__global__ __launch_bounds__(kBlock) void k_param_contract(const double* __restrict__ G, int N,
                                                           double ha, double a, int kind,
                                                           const double* __restrict__ p,
                                                           const int* __restrict__ wrt, int nwrt,
                                                           double* __restrict__ partials) {
  __shared__ double red[kBlock / 64][8];
  const long long n3 = (long long)N * N * N;
  const double cN = (double)(N - 1), half = 0.5 * (double)(N - 1) * a;
  for (int k0 = 0; k0 < nwrt; k0 += 8) {
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n3;
         s += (long long)gridDim.x * blockDim.x) {
      const int iz = (int)(s % N);
      const long long q = s / N;
      const int iy = (int)(q % N);
      const int ix = (int)(q / N);
      const double xs[3] = {(2.0 * ix - cN) * ha, (2.0 * iy - cN) * ha, (2.0 * iz - cN) * ha};
      const double r = sqrt(xs[0] * xs[0] + xs[1] * xs[1] + xs[2] * xs[2]);
      const double g = G[s];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const int k = k0 + kk;
        if (k >= nwrt) break;
        acc[kk] += g * param_dv(kind, p, wrt[k], xs, r, a, N, half);
      }
    }
    block_sum<8>(acc, red);
    if (threadIdx.x == 0) {
      for (int kk = 0; kk < 8 && k0 + kk < nwrt; ++kk)
        partials[(long long)blockIdx.x * kMaxWrt + k0 + kk] = acc[kk];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_sum_partials(const double* __restrict__ partials,
                                                         int nblocks, int nwrt,
                                                         double* __restrict__ out) {
  const int k = threadIdx.x;
  if (k < nwrt) {
    double t = 0.0;
    for (int b = 0; b < nblocks; ++b) t += partials[(long long)b * kMaxWrt + k];
    out[k] = t;
  }
}

// ----------------------------------------------------------- projection ----
// Excited states by projection (Sec. III): psi <- psi - phi <phi|psi> /
// <phi|phi>.  Three launches per state, no host round trip: FP64 partial sums
// of <phi|phi> and <phi|psi> per work-group (grid-stride, fixed grid), one
// work-group summing them in a fixed order into the coefficient (device
// memory), then the update reading it.
constexpr int kProjGrid = 1024;

template <typename S, typename B>
__global__ __launch_bounds__(kBlock) void k_proj_partials(const S* __restrict__ psi,
                                                          const B* __restrict__ phi,
                                                          long long n3, double* partials) {
  __shared__ double red[kBlock / 64][2];
  double pp = 0.0, pq = 0.0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n3;
       i += (long long)gridDim.x * kBlock) {
    const double f = (double)phi[i];
    pp += f * f;
    pq += f * to_c<S, double>(psi[i]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    pp += __shfl_down(pp, o);
    pq += __shfl_down(pq, o);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[w][0] = pp;
    red[w][1] = pq;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < kBlock / 64; ++k) {
      a += red[k][0];
      b += red[k][1];
    }
    partials[2 * blockIdx.x] = a;
    partials[2 * blockIdx.x + 1] = b;
  }
}

__global__ void k_proj_coef(const double* __restrict__ partials, int nblocks, double* coef) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double pp = 0.0, pq = 0.0;
    for (int b = 0; b < nblocks; ++b) {
      pp += partials[2 * b];
      pq += partials[2 * b + 1];
    }
    coef[0] = pp > 0.0 ? pq / pp : 0.0;
  }
}

template <typename S, typename B>
__global__ __launch_bounds__(kBlock) void k_proj_update(S* __restrict__ psi,
                                                        const B* __restrict__ phi, long long n3,
                                                        const double* __restrict__ coef) {
  const double c = coef[0];
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n3;
       i += (long long)gridDim.x * kBlock) {
    if constexpr (sizeof(S) == 8) {
      psi[i] = psi[i] - c * (double)phi[i];
    } else {
      const float v = to_c<S, float>(psi[i]) - (float)c * (float)phi[i];
      psi[i] = from_c<S, float>(v);
    }
  }
}

// ------------------------------------------------------------- dispatch ----
int grid_for(long long n) {
  long long g = (n + kBlock - 1) / kBlock;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

// Launch shapes holding more than 32 bytes of arithmetic-type state per
// lane and plane (8 FP32 or 4 FP64 sites) spill registers and are not
// instantiated; the scalar-lane fallback (VZ = 1) and the reduction-only
// pass use prefetch distance 1 only.
template <int DT, int VZ, int RY, bool UPD, int D>
hipError_t step_one(int grid, int bt, bool fv, bool wt, const StepArgs& a, hipStream_t s) {
  if constexpr (VZ * RY * (int)sizeof(typename Types<DT>::C) <= 32 && (D == 1 || (UPD && VZ > 1))) {
    // written-through stores: 256-lane groups, full vectors, one or two per lane
    if constexpr (UPD && VZ == Types<DT>::kVec && RY <= 2) {
      if (wt && bt == 256) {
        if constexpr (DT != kF64) {
          if (fv) {
            hipLaunchKernelGGL((k_step<DT, VZ, RY, UPD, D, 256, true, true>), dim3(grid), dim3(256), 0, s, a);
            return hipGetLastError();
          }
        }
        if (fv) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_step<DT, VZ, RY, UPD, D, 256, false, true>), dim3(grid), dim3(256), 0, s, a);
        return hipGetLastError();
      }
    }
    if (wt && UPD) return hipErrorInvalidValue;
    if (fv) {
      // in-kernel potential: FP32 arithmetic lattices
      if constexpr (DT != kF64) {
        if (bt == 256) {
          hipLaunchKernelGGL((k_step<DT, VZ, RY, UPD, D, 256, true>), dim3(grid), dim3(256), 0, s, a);
          return hipGetLastError();
        }
        if constexpr (RY == 1 && VZ * sizeof(typename Types<DT>::C) <= 16) {
          if (bt == 512) {
            hipLaunchKernelGGL((k_step<DT, VZ, 1, UPD, D, 512, true>), dim3(grid), dim3(512), 0, s, a);
            return hipGetLastError();
          }
        }
      }
      return hipErrorInvalidValue;
    }
    if (bt == 256) {
      hipLaunchKernelGGL((k_step<DT, VZ, RY, UPD, D, 256, false>), dim3(grid), dim3(256), 0, s, a);
      return hipGetLastError();
    }
    // 512-lane groups cap registers at 256: one vector of <= 16 bytes of
    // arithmetic-type state per lane, and no deep prefetch for FP64
    if constexpr (RY == 1 && VZ * sizeof(typename Types<DT>::C) <= 16 &&
                  (D == 1 || sizeof(typename Types<DT>::C) == 4)) {
      if (bt == 512) {
        hipLaunchKernelGGL((k_step<DT, VZ, 1, UPD, D, 512, false>), dim3(grid), dim3(512), 0, s, a);
        return hipGetLastError();
      }
    }
    return hipErrorInvalidValue;
  } else {
    return hipErrorInvalidValue;
  }
}

template <int DT, int VZ, bool UPD, int D>
hipError_t step_ry(int ry, int grid, int bt, bool fv, bool wt, const StepArgs& a, hipStream_t s) {
  switch (ry) {
    case 1: return step_one<DT, VZ, 1, UPD, D>(grid, bt, fv, wt, a, s);
    case 2: return step_one<DT, VZ, 2, UPD, D>(grid, bt, fv, wt, a, s);
    case 4: return step_one<DT, VZ, 4, UPD, D>(grid, bt, fv, wt, a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int DT, int VZ, int RY, int D>
hipError_t persist_one(int grid, bool fv, const StepArgs& a, hipStream_t s) {
  if constexpr (VZ * RY * (int)sizeof(typename Types<DT>::C) <= 32 && (D == 1 || VZ > 1)) {
    if (fv) {
      if constexpr (DT != kF64) {
        hipLaunchKernelGGL((k_step_persist<DT, VZ, RY, D, 256, true>), dim3(grid), dim3(256), 0, s, a);
        return hipGetLastError();
      }
      return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((k_step_persist<DT, VZ, RY, D, 256, false>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int DT, int VZ, int D>
hipError_t persist_ry(int ry, int grid, bool fv, const StepArgs& a, hipStream_t s) {
  switch (ry) {
    case 1: return persist_one<DT, VZ, 1, D>(grid, fv, a, s);
    case 2: return persist_one<DT, VZ, 2, D>(grid, fv, a, s);
    case 4: return persist_one<DT, VZ, 4, D>(grid, fv, a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int DT, int VZ>
hipError_t persist_d(int depth, int ry, int grid, bool fv, const StepArgs& a, hipStream_t s) {
  switch (depth) {
    case 1: return persist_ry<DT, VZ, 1>(ry, grid, fv, a, s);
    case 2: return persist_ry<DT, VZ, 2>(ry, grid, fv, a, s);
    case 3: return persist_ry<DT, VZ, 3>(ry, grid, fv, a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int DT>
hipError_t persist_dt(int vz, int depth, int ry, int grid, bool fv, const StepArgs& a,
                      hipStream_t s) {
  if (vz == 1) return persist_d<DT, 1>(1, ry, grid, fv, a, s);
  if (vz == Types<DT>::kVec) return persist_d<DT, Types<DT>::kVec>(depth, ry, grid, fv, a, s);
  return hipErrorInvalidValue;
}

__global__ void k_persist_reset(Control* ctrl, MemberState* states, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) states[i].fin = 0u;
  if (i == 0) {
    ctrl->ticket = 0u;
    ctrl->abort = 0;
  }
}

template <int DT, int VZ, bool UPD>
hipError_t step_d(int depth, int ry, int grid, int bt, bool fv, bool wt, const StepArgs& a,
                  hipStream_t s) {
  switch (depth) {
    case 1: return step_ry<DT, VZ, UPD, 1>(ry, grid, bt, fv, wt, a, s);
    case 2: return step_ry<DT, VZ, UPD, 2>(ry, grid, bt, fv, wt, a, s);
    case 3: return step_ry<DT, VZ, UPD, 3>(ry, grid, bt, fv, wt, a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int DT, bool UPD>
hipError_t step_vz(int vz, int depth, int ry, int grid, int bt, bool fv, bool wt,
                   const StepArgs& a, hipStream_t s) {
  if (vz == 1) return step_d<DT, 1, UPD>(depth, ry, grid, bt, fv, wt, a, s);
  if (vz == Types<DT>::kVec)
    return step_d<DT, Types<DT>::kVec, UPD>(depth, ry, grid, bt, fv, wt, a, s);
  return hipErrorInvalidValue;
}

template <int DT>
hipError_t step_dt(int vz, int depth, int ry, bool upd, int grid, int bt, bool fv, bool wt,
                   const StepArgs& a, hipStream_t s) {
  // the reduction-only pass stores nothing
  return upd ? step_vz<DT, true>(vz, depth, ry, grid, bt, fv, wt, a, s)
             : step_vz<DT, false>(vz, 1, ry, grid, bt, fv, false, a, s);
}

template <int DT, bool UPD, int D>
hipError_t tile_d(int grid, unsigned lds, const StepArgs& a, hipStream_t s) {
  constexpr int VZ = Types<DT>::kVec;
  hipLaunchKernelGGL((k_step_tile<DT, VZ, UPD, D>), dim3(grid), dim3(TileShape<DT>::kTB), lds, s, a);
  return hipGetLastError();
}

template <int DT>
hipError_t tile_dt(int depth, bool upd, int grid, unsigned lds, const StepArgs& a, hipStream_t s) {
  if (!upd) return tile_d<DT, false, 1>(grid, lds, a, s);
  switch (depth) {
    case 1: return tile_d<DT, true, 1>(grid, lds, a, s);
    case 2: return tile_d<DT, true, 2>(grid, lds, a, s);
    case 3: return tile_d<DT, true, 3>(grid, lds, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int tile_threads(int dtype) { return dtype == kBF16 ? 512 : 1024; }

hipError_t launch_step_tile(int dtype, int depth, bool update, int grid, int max_n,
                            const StepArgs& a, hipStream_t s) {
  const unsigned vz = dtype == kF64 ? 2 : (dtype == kF32 ? 4 : 8);
  // the first 2N / vz lanes load the halo rows: 2N <= (lanes) vz
  if (grid < 1 || max_n < 1 || 2u * (unsigned)max_n > (unsigned)tile_threads(dtype) * vz)
    return hipErrorInvalidValue;
  const unsigned cs = dtype == kF64 ? 8 : 4;
  const unsigned lds = 2u * ((unsigned)tile_threads(dtype) * vz + 2u * (unsigned)max_n) * cs;
  switch (dtype) {
    case kF64: return tile_dt<kF64>(depth, update, grid, lds, a, s);
    case kF32: return tile_dt<kF32>(depth, update, grid, lds, a, s);
    case kBF16: return tile_dt<kBF16>(depth, update, grid, lds, a, s);
    default: return hipErrorInvalidValue;
  }
}

namespace {

template <int DT, int D, bool FV>
hipError_t step2_one(int grid, const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_step2<DT, kTbVec(DT), D, FV>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int DT, bool FV>
hipError_t step2_depth(int depth, int grid, const StepArgs& a, hipStream_t s) {
  switch (depth) {
    case 1: return step2_one<DT, 1, FV>(grid, a, s);
    case 2: return step2_one<DT, 2, FV>(grid, a, s);
    case 3: return step2_one<DT, 3, FV>(grid, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_step2(int dtype, int depth, bool fv, int grid, const StepArgs& a,
                        hipStream_t s) {
  if (grid < 1) return hipErrorInvalidValue;
  switch (dtype) {
    case kF64: return fv ? hipErrorInvalidValue : step2_depth<kF64, false>(depth, grid, a, s);
    case kF32: return fv ? step2_depth<kF32, true>(depth, grid, a, s)
                         : step2_depth<kF32, false>(depth, grid, a, s);
    case kBF16: return fv ? step2_depth<kBF16, true>(depth, grid, a, s)
                          : step2_depth<kBF16, false>(depth, grid, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_step_persist(int dtype, int vz, int ry, int depth, int grid, bool fv,
                               const StepArgs& a, hipStream_t s) {
  if (grid < 1 || a.steps < 1 || !a.ctrl) return hipErrorInvalidValue;
  switch (dtype) {
    case kF64: return persist_dt<kF64>(vz, depth, ry, grid, fv, a, s);
    case kF32: return persist_dt<kF32>(vz, depth, ry, grid, fv, a, s);
    case kBF16: return persist_dt<kBF16>(vz, depth, ry, grid, fv, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_persist_reset(Control* ctrl, MemberState* states, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_persist_reset, dim3((count + 255) / 256), dim3(256), 0, s, ctrl, states, count);
  return hipGetLastError();
}

hipError_t launch_step(int dtype, int vz, int ry, int depth, bool update, int grid, int bt,
                       bool fv, bool wt, const StepArgs& a, hipStream_t s) {
  if (grid < 1) return hipErrorInvalidValue;
  if (vz == 1) depth = 1;
  switch (dtype) {
    case kF64: return step_dt<kF64>(vz, depth, ry, update, grid, bt, fv, wt, a, s);
    case kF32: return step_dt<kF32>(vz, depth, ry, update, grid, bt, fv, wt, a, s);
    case kBF16: return step_dt<kBF16>(vz, depth, ry, update, grid, bt, fv, wt, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_potential(int vdtype, void* V, int N, double ha, double a, int kind,
                            const double* p_dev, int np, hipStream_t s) {
  const int g = grid_for((long long)N * N * N);
  if (vdtype == kF64)
    hipLaunchKernelGGL(k_potential<double>, dim3(g), dim3(kBlock), 0, s, (double*)V, N, ha, a,
                       kind, p_dev, np);
  else
    hipLaunchKernelGGL(k_potential<float>, dim3(g), dim3(kBlock), 0, s, (float*)V, N, ha, a, kind,
                       p_dev, np);
  return hipGetLastError();
}

hipError_t launch_initial(int dtype, void* psi, int N, uint64_t seed, uint32_t member, int kind,
                          uint32_t parity, hipStream_t s) {
  const int g = grid_for((long long)N * N * N);
  switch (dtype) {
    case kF64: hipLaunchKernelGGL(k_initial<double>, dim3(g), dim3(kBlock), 0, s, (double*)psi, N, seed, member, kind, parity); break;
    case kF32: hipLaunchKernelGGL(k_initial<float>, dim3(g), dim3(kBlock), 0, s, (float*)psi, N, seed, member, kind, parity); break;
    case kBF16: hipLaunchKernelGGL(k_initial<uint16_t>, dim3(g), dim3(kBlock), 0, s, (uint16_t*)psi, N, seed, member, kind, parity); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

namespace {
template <typename SS>
hipError_t convert_to(const SS* src, int ddtype, void* dst, long long n, double scale,
                      hipStream_t s) {
  const int g = grid_for(n);
  switch (ddtype) {
    case kF64: hipLaunchKernelGGL((k_convert<SS, double>), dim3(g), dim3(kBlock), 0, s, src, (double*)dst, n, scale); break;
    case kF32: hipLaunchKernelGGL((k_convert<SS, float>), dim3(g), dim3(kBlock), 0, s, src, (float*)dst, n, scale); break;
    case kBF16: hipLaunchKernelGGL((k_convert<SS, uint16_t>), dim3(g), dim3(kBlock), 0, s, src, (uint16_t*)dst, n, scale); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename CS>
hipError_t upsample_to(const CS* pc, int Nc, double hac, double ac, int fdtype, void* pf, int Nf,
                       double haf, hipStream_t s) {
  (void)hac;
  // (y, z-vector) columns of the fine lattice x fine x-ranges of kUpXC planes
  const long long cols = (long long)Nf * ((Nf + kUpVZ - 1) / kUpVZ);
  const dim3 g((unsigned)((cols + kBlock - 1) / kBlock), (unsigned)((Nf + kUpXC - 1) / kUpXC));
  if constexpr (sizeof(CS) == 2) {
    if (Nc % 2 == 0 && Nf >= 2 * Nc) {
      switch (fdtype) {
        case kF64: hipLaunchKernelGGL((k_upsample<CS, double, true>), g, dim3(kBlock), 0, s, pc, Nc, ac, (double*)pf, Nf, haf); break;
        case kF32: hipLaunchKernelGGL((k_upsample<CS, float, true>), g, dim3(kBlock), 0, s, pc, Nc, ac, (float*)pf, Nf, haf); break;
        case kBF16: hipLaunchKernelGGL((k_upsample<CS, uint16_t, true>), g, dim3(kBlock), 0, s, pc, Nc, ac, (uint16_t*)pf, Nf, haf); break;
        default: return hipErrorInvalidValue;
      }
      return hipGetLastError();
    }
  }
  switch (fdtype) {
    case kF64: hipLaunchKernelGGL((k_upsample<CS, double, false>), g, dim3(kBlock), 0, s, pc, Nc, ac, (double*)pf, Nf, haf); break;
    case kF32: hipLaunchKernelGGL((k_upsample<CS, float, false>), g, dim3(kBlock), 0, s, pc, Nc, ac, (float*)pf, Nf, haf); break;
    case kBF16: hipLaunchKernelGGL((k_upsample<CS, uint16_t, false>), g, dim3(kBlock), 0, s, pc, Nc, ac, (uint16_t*)pf, Nf, haf); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_convert(int sdtype, const void* src, int ddtype, void* dst, long long n,
                          double scale, hipStream_t s) {
  switch (sdtype) {
    case kF64: return convert_to((const double*)src, ddtype, dst, n, scale, s);
    case kF32: return convert_to((const float*)src, ddtype, dst, n, scale, s);
    case kBF16: return convert_to((const uint16_t*)src, ddtype, dst, n, scale, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_upsample(int cdtype, const void* pc, int Nc, double hac, double ac, int fdtype,
                           void* pf, int Nf, double haf, hipStream_t s) {
  switch (cdtype) {
    case kF64: return upsample_to((const double*)pc, Nc, hac, ac, fdtype, pf, Nf, haf, s);
    case kF32: return upsample_to((const float*)pc, Nc, hac, ac, fdtype, pf, Nf, haf, s);
    case kBF16: return upsample_to((const uint16_t*)pc, Nc, hac, ac, fdtype, pf, Nf, haf, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_project(int dtype, void* psi, const void* phi, long long n3, double* partials,
                          double* coef, hipStream_t s) {
  const int g = kProjGrid;
  switch (dtype) {
    case kF64:
      hipLaunchKernelGGL((k_proj_partials<double, double>), dim3(g), dim3(kBlock), 0, s,
                         (const double*)psi, (const double*)phi, n3, partials);
      break;
    case kF32:
      hipLaunchKernelGGL((k_proj_partials<float, float>), dim3(g), dim3(kBlock), 0, s,
                         (const float*)psi, (const float*)phi, n3, partials);
      break;
    case kBF16:
      hipLaunchKernelGGL((k_proj_partials<uint16_t, float>), dim3(g), dim3(kBlock), 0, s,
                         (const uint16_t*)psi, (const float*)phi, n3, partials);
      break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k_proj_coef, dim3(1), dim3(64), 0, s, (const double*)partials, g, coef);
  switch (dtype) {
    case kF64:
      hipLaunchKernelGGL((k_proj_update<double, double>), dim3(g), dim3(kBlock), 0, s,
                         (double*)psi, (const double*)phi, n3, (const double*)coef);
      break;
    case kF32:
      hipLaunchKernelGGL((k_proj_update<float, float>), dim3(g), dim3(kBlock), 0, s,
                         (float*)psi, (const float*)phi, n3, (const double*)coef);
      break;
    default:
      hipLaunchKernelGGL((k_proj_update<uint16_t, float>), dim3(g), dim3(kBlock), 0, s,
                         (uint16_t*)psi, (const float*)phi, n3, (const double*)coef);
  }
  return hipGetLastError();
}

int project_partials_doubles() { return 2 * kProjGrid; }

hipError_t launch_reimpose(int dtype, void* psi, int N, uint32_t parity, hipStream_t s) {
  const int g = grid_for((long long)N * N * N);
  switch (dtype) {
    case kF64: hipLaunchKernelGGL(k_reimpose<double>, dim3(g), dim3(kBlock), 0, s, (double*)psi, N, parity); break;
    case kF32: hipLaunchKernelGGL(k_reimpose<float>, dim3(g), dim3(kBlock), 0, s, (float*)psi, N, parity); break;
    case kBF16: hipLaunchKernelGGL(k_reimpose<uint16_t>, dim3(g), dim3(kBlock), 0, s, (uint16_t*)psi, N, parity); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_set_state(MemberState* st, int member, double scale, long long step,
                            int reset_bad, hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(1), dim3(64), 0, s, st, member, scale, step, reset_bad);
  return hipGetLastError();
}

hipError_t launch_adjoint_step(int dtype, const AdjArgs& a, hipStream_t s) {
  if (a.N < 1 || (dtype != kF64 && dtype != kF32)) return hipErrorInvalidValue;
  // VZ sites per lane when N allows (a lane's vector stays within a z-row),
  // else one
  const int vz = dtype == kF64 ? 2 : 4;
  const bool vec = a.N % vz == 0;
  const long long P = (long long)a.N * a.N, F = (long long)kBlock * (vec ? vz : 1);
  const long long nchunk = (P + F - 1) / F;
  AdjArgs b = a;
  // x split into ranges for about 2048 work items (measured at 256^3 FP32:
  // 256 to 4096 items and 256 to 1024 lanes per work-group within 3%)
  b.nx = (int)std::min<long long>(a.N, std::max<long long>(1, (2048 + nchunk - 1) / nchunk));
  const int g = (int)std::min<long long>(nchunk * b.nx, 1 << 20);
  if (dtype == kF64) {
    if (vec) hipLaunchKernelGGL((k_adjoint_step<double, 2, kBlock>), dim3(g), dim3(kBlock), 0, s, b);
    else hipLaunchKernelGGL((k_adjoint_step<double, 1, kBlock>), dim3(g), dim3(kBlock), 0, s, b);
  } else {
    if (vec) hipLaunchKernelGGL((k_adjoint_step<float, 4, kBlock>), dim3(g), dim3(kBlock), 0, s, b);
    else hipLaunchKernelGGL((k_adjoint_step<float, 1, kBlock>), dim3(g), dim3(kBlock), 0, s, b);
  }
  return hipGetLastError();
}

hipError_t launch_adjoint_init(int dtype, const AdjInitArgs& a, hipStream_t s) {
  const int g = grid_for((long long)a.N * a.N * a.N);
  if (dtype == kF64) hipLaunchKernelGGL(k_adjoint_init<double>, dim3(g), dim3(kBlock), 0, s, a);
  else if (dtype == kF32) hipLaunchKernelGGL(k_adjoint_init<float>, dim3(g), dim3(kBlock), 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_param_contract(const double* G, int N, double ha, double a, int kind,
                                 const double* p_dev, int np, const int* wrt_dev, int nwrt,
                                 double* partials, int nblocks, double* out_dev, hipStream_t s) {
  if (nwrt < 1 || nwrt > kMaxWrt || nblocks < 1 || kind < 0 || kind > 6 || np < 1)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_param_contract, dim3(nblocks), dim3(kBlock), 0, s, G, N, ha, a, kind, p_dev,
                     wrt_dev, nwrt, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kMaxWrt), 0, s, partials, nblocks, nwrt,
                     out_dev);
  return hipGetLastError();
}

}  // namespace fdtd
