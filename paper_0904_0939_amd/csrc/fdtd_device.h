// Device-side helpers shared by the step kernels (fdtd_step.hip) and the
// set-up, upsample, adjoint and projection kernels (fdtd_aux.hip): number
// types, raw buffer loads and stores, BF16 rounding, the site hash, FP64
// block reductions and the last-work-group finalisation of a step.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "fdtd_internal.h"

// No implicit fused multiply-adds in any kernel source: every fma is written
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

// The same for a plane index held in a scalar register (a loop counter):
// the select is on the index, not on the product, so it stays a scalar
// select.  The select of the product becomes a uniform branch, and the
// branches split an unrolled plane loop into blocks into which the compiler
// sinks earlier stages' arithmetic, keeping its operands live.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc_u(const void* base, int x, int N,
                                                              unsigned bytes) {
  const bool in = x >= 0 && x < N;
  const unsigned xs = in ? (unsigned)x : 0u;
  char* p = const_cast<char*>(static_cast<const char*>(base)) + (unsigned long long)xs * bytes;
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
// Returns the rounded value as an FP32 bit pattern whose low 16 bits are
// zero: the high half is the BF16 value, and the whole is its FP32 value, so
// the stored bits and the value the norm sums come from one mask-and-or.
__device__ __forceinline__ uint32_t f32_to_bf16_sr_bits(float f, uint32_t r16) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t mag = min(u & 0x7fffffffu, 0x7fc00000u);
  return ((mag + r16) & 0x7fff0000u) | (u & 0x80000000u);
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

}  // namespace
}  // namespace fdtd
