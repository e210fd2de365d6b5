// The per-site update and reductions of the fused step (Eq. (updateeq),
// Eq. (energysum)) and the streaming of one work item along x, shared by the
// one-step kernels (fdtd_step.hip) and the two-step kernels (fdtd_step2.hip).
#pragma once

#include "fdtd_device.h"

#pragma clang fp contract(off)

namespace fdtd {
namespace {

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
// USEL: plane indices are loop counters in scalar registers (the one-step
// kernels), so the resources take the branch-free form (plane_rsrc_u).
template <int DT, int VZ, int RY, bool UPD, bool FV = false, int OUT = FDTD_AUX_OUT,
          bool USEL = false>
struct StepBody {
  using S = typename Types<DT>::S;
  using TV = typename Types<DT>::V;
  using C = typename Types<DT>::C;
  static constexpr unsigned kES = sizeof(S);
  // z neighbours across vector boundaries by cross-lane reads (measured
  // faster for FP32 and FP64; BF16 lanes hold 8 sites and gain nothing)
  static constexpr bool kSHZ = kShuffleZ && DT != kBF16;
  static constexpr bool kPinSums = DT != kF64;

  static __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, int x, int N,
                                                                unsigned bytes) {
    if constexpr (USEL) return plane_rsrc_u(base, x, N, bytes);
    else return plane_rsrc(base, x, N, bytes);
  }

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
    const __amdgpu_buffer_rsrc_t rc = rsrc(k.in, x, min(k.N, k.xe), k.pbytes);
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
      const __amdgpu_buffer_rsrc_t rv = rsrc(k.Vf, x, min(k.N, k.xe), k.vbytes);
#pragma unroll
      for (int r = 0; r < RY; ++r) bload<TV, VZ, C, VAUX>(rv, ln.voff[r], v[r]);
    }
  }

  // Own sites of plane x (needed for x <= xe).
  static __device__ __forceinline__ void fetch_own(const Ctx& k, const Lane<RY, VZ, C>& ln, int x,
                                                   C (&q)[RY][VZ]) {
    const __amdgpu_buffer_rsrc_t r0 = rsrc(k.in, x, min(k.N, k.xe + 1), k.pbytes);
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
    const __amdgpu_buffer_rsrc_t ro = rsrc(k.out, x, k.N, k.pbytes);
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
          C od;
          if constexpr (sizeof(S) == 2) {
            uint32_t ob = f32_to_bf16_sr_bits((float)nv, rb[j]);
            // one register for the stored bits and the value the norm sums
            // (else both are built, by two different instructions)
            asm volatile("" : "+v"(ob));
            o.v[j] = (S)(ob >> 16);
            od = __uint_as_float(ob);
          } else {
            o.v[j] = (S)nv;
            od = to_c<S, C>(o.v[j]);
          }
          if (r < NRED) s1 = live ? fma_c(od, od, s1) : s1;
          if constexpr (TOREG) outv[r][j] = od;
        }
      }
      if constexpr (UPD && !TOREG) bstore<S, VZ, OUT>(ro, ln.off[r], o);
    }
    if constexpr (NRED > 0) {
      acc[0] += (double)s0;
      acc[1] += (double)kin;
      acc[2] += (double)pot;
      acc[3] += (double)r2 + (double)rx2 * (double)s0;
      acc[4] += (double)s1;
      // FP32 arithmetic: keep this plane's sums here.  Without the pin the
      // compiler sinks the reductions of every stage to the end of the
      // unrolled trip, which keeps all their operands live at once (~90 more
      // registers per lane).  FP64 kernels are compiled without it.
      if constexpr (kPinSums)
        asm volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]));
    }
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
  // BF16 states: branch-free plane resources (in-kernel V, sums pinned: 512^3
  // 225.7 -> 221.4 us, 256^3 36.7 -> 34.9 us per step); FP32 states keep the
  // branch form (in-kernel V at 512^3: 215 us with it, 260 us without)
  using Body = StepBody<DT, VZ, RY, UPD, FV, OUT, DT == kBF16>;
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

// Work-group barrier fenced on LDS only: outstanding global loads (the
// prefetched planes) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

}  // namespace
}  // namespace fdtd
