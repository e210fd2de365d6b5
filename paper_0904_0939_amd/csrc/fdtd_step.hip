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
#include "fdtd_stepbody.h"

#pragma clang fp contract(off)

namespace fdtd {
namespace {

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

}  // namespace fdtd
