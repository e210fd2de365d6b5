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

}  // namespace fdtd
