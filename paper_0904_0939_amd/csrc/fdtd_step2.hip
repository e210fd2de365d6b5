// Temporal blocking (two steps per pass over HBM) of the fused step: the
// k_step2 kernel and its dispatch.  The per-site arithmetic is the one-step
// kernel's (fdtd_stepbody.h), so with the rescale off a two-step pass
// stores the same bits as two one-step launches.
#include "fdtd_stepbody.h"

#pragma clang fp contract(off)

namespace fdtd {
namespace {

// -------------------------------------- temporal blocking: two steps ----
// k_step2 advances every member two steps per pass over HBM (psi and V read
// once, psi'' written once).  A work item owns a tile of kTbRows(DT, WIDE) x
// kTbCols(DT, WIDE) sites of the (y, z) plane and streams x; each lane holds
// one vector of VZ consecutive z sites (a tile row is 256 bytes of F32 / F64,
// 512 bytes for the wide F32 tile; BF16 lattices use the F32 tiles, 4 sites
// per lane).
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

// V of a tile's sites is read again as the halo frame of its neighbours, so
// the two-step kernel keeps V loads in the caches.
#ifndef FDTD_TB_AUX_V
#define FDTD_TB_AUX_V 0
#endif
constexpr int kTbVAux = FDTD_TB_AUX_V;

// FP32-arithmetic lattices (F32, BF16): step t's y / z neighbours of the
// tile's own vectors from an LDS copy of the framed psi_t plane, written one
// stage ahead from the lanes' own loads and the halo lanes' loads, instead of
// per-lane neighbour loads and their register ring (1); with it, and two
// waves per SIMD, a 512^3 F32 step takes 192 us (depth 3) against 225 us (one
// wave, the loads).  FP64 lattices keep the loads: with one wave the staging measured
// slower (485 against 433 us per step), and two waves would spill a hundred
// registers.  0: the loads for every dtype.
#ifndef FDTD_TB_LDS_PSI
#define FDTD_TB_LDS_PSI 1
#endif
constexpr bool tb_lds_psi(int dt) { return FDTD_TB_LDS_PSI != 0 && dt != kF64; }

// Step t's results of the planes step t + 1 reads (X - 2, X - 1, X) from a
// triple-buffered LDS tile (1) instead of a three-plane register ring (0);
// measured no faster (210 against 206 us per 512^3 F32 step): off.
#ifndef FDTD_TB_LDS_U
#define FDTD_TB_LDS_U 0
#endif
constexpr bool kTbLdsU = FDTD_TB_LDS_U != 0;
constexpr int kTbTileBufs = kTbLdsU ? 3 : 2;

// Waves per SIMD the two-step kernel's register budget must allow: two for
// FP32 arithmetic (F32 and BF16 states: 200-225 VGPRs with the reductions
// pinned per plane; a 512-lane tile per CU), one for FP64 (two would spill
// about a hundred).
#ifndef FDTD_TB_MIN_WAVES_F32
#define FDTD_TB_MIN_WAVES_F32 2
#endif
#ifndef FDTD_TB_MIN_WAVES_F64
#define FDTD_TB_MIN_WAVES_F64 1
#endif
constexpr int tb_min_waves(int dt) { return dt == kF64 ? FDTD_TB_MIN_WAVES_F64 : FDTD_TB_MIN_WAVES_F32; }

template <int DT, int VZ, int D, bool FV, bool WIDE>
struct Step2 {
  static constexpr int BT = kTbThreads(DT);
  static constexpr int TZ = kTbCols(DT, WIDE);      // tile columns (z sites)
  static constexpr int LPR = TZ / VZ;               // lanes per tile row
  static constexpr int TY = BT / LPR;               // tile rows
  static constexpr int NH = 2 * TZ + 2 * TY;        // halo sites, one per lane
  static constexpr int NHW = (NH + 63) / 64;        // waves that carry halo sites
  static constexpr int RP = TZ + 8;                 // LDS row pitch: own z at 4 .. 4 + TZ - 1
  static constexpr int TS = (TY + 2) * RP;          // LDS plane: rows y0 - 1 .. y0 + TY
  static constexpr bool kPsi = tb_lds_psi(DT);       // neighbours of step t from LDS
  // register rings: RS plane slots (an unrolled trip of RS stages; a load
  // D planes ahead needs D + 3 slots), US slots of step-t results
  static constexpr int RS = D <= 3 ? 6 : 8;
  static constexpr int US = D <= 3 ? 3 : 4;
  static_assert(D >= 1 && D + 3 <= RS, "prefetch depth 1..5");
  static_assert(TY == kTbRows(DT, WIDE) && TZ % VZ == 0, "tile shape");
  static_assert(NH <= BT, "one halo site per lane");
  using B = StepBody<DT, VZ, 1, true, FV>;  // own vectors
  using H = StepBody<DT, 1, 1, true, FV>;   // halo sites
  using C = typename B::C;

  struct Rings {
    C qs[RS][1][VZ];          // psi_t of planes, own vectors
    C vs[RS][1][VZ];          // V of planes
    PlaneIn<1, VZ, C> nb[RS]; // y / z neighbours of psi_t planes
    C qh[RS][1][1];           // the same for the lane's halo site
    C vh[RS][1][1];
    PlaneIn<1, 1, C> nh[RS];
    C us[kTbLdsU ? 1 : US][1][VZ];  // step-t results, own vectors (register ring form)
    // F32 states (kShare): the x-differences carried from plane to plane
    // (step t, step t + 1), and B, dt V of the own vectors of the last two
    // planes (written by step t, read by step t + 1 one plane later)
    C dx1[VZ], dx2[VZ];
    C bw[2][VZ], dw[2][VZ];
  };

  // F32 states share work between neighbouring sites and between the two
  // steps (update_tb); BF16 states sum the Laplacian without differences,
  // FP64 keeps the one-step body as it is.
  static constexpr bool kShare = DT == kF32 && !kTbLdsU;

  // update_core's arithmetic for the lane's own vector (F32 states), bit for
  // bit, with what a pass of two steps can share.  (1) A difference along x
  // or z is computed once per pair of sites: the one a site takes towards
  // x - 1 (z - 1) is the negation of the one its neighbour took towards
  // x + 1 (z + 1), the same value in round to nearest (an exact zero may
  // change sign, which no pair sum of the Laplacian keeps).  dxc carries
  // q(x) - q(x - 1) in and q(x + 1) - q(x) out.  (2) Step t computes B =
  // 1 / (1 + dt V / 2) and dt V of its own vectors and keeps them (BM = 1);
  // step t + 1 takes them one plane later (BM = 2).  TOREG: return the new
  // values (step t) instead of storing them (step t + 1).
  template <bool TOREG, int BM>
  static __device__ __forceinline__ void update_tb(const typename B::Ctx& k,
                                                   const Lane<1, VZ, C>& ln, int x,
                                                   const C (&pc)[VZ], const C (&pn)[VZ],
                                                   C (&dxc)[VZ], const C (&vv)[VZ],
                                                   const PlaneIn<1, VZ, C>& d, C (&bw)[VZ],
                                                   C (&dw)[VZ], double (&acc)[5], C (&outv)[VZ]) {
    static_assert(DT == kF32, "F32 states");
    const double xc = (2.0 * x - k.cN) * k.ha;
    const C rx2 = (C)(xc * xc);
    C s0 = 0, kin = 0, pot = 0, r2 = 0, s1 = 0;
    // d holds the LDS values unmasked: beyond the lattice's z ends they are
    // the frame's or the outside lanes' zeros, so no z mask is needed (an
    // outside vector has c = 0, see tb_item)
    const C lo = d.zm[0];
    const C hi = d.zp[0];
    // zd[j]: site j's difference towards z - 1; zd[VZ]: the last site's
    // towards z + 1
    C zd[VZ + 1];
    zd[0] = lo - pc[0];
#pragma unroll
    for (int j = 1; j < VZ; ++j) zd[j] = pc[j - 1] - pc[j];
    zd[VZ] = hi - pc[VZ - 1];
    Pack<C, VZ> o;
#pragma unroll
    for (int j = 0; j < VZ; ++j) {
      const C p = pc[j];
      const C dxm = -dxc[j];
      const C dxp = pn[j] - p;
      dxc[j] = dxp;
      const C dzr = j < VZ - 1 ? -zd[j + 1] : zd[VZ];
      const C lap = ((dxm + dxp) + ((d.ym[0][j] - p) + (d.yp[0][j] - p))) + (zd[j] + dzr);
      const C p2 = p * p;
      const C v = vv[j];
      s0 += p2;
      kin = fma_c(p, lap, kin);
      pot = fma_c(v, p2, pot);
      r2 = fma_c(ln.w2[0][j], p2, r2);
      if constexpr (BM != 2) {
        bw[j] = rcp_c(fma_c(k.eps, v, C(1)));
        dw[j] = k.dt * v;
      }
      const C g = fma_c(k.c, lap, -(dw[j] * p));  // c lap - dt V psi
      const C nv = k.sc * fma_c(bw[j], g, p);
      o.v[j] = nv;
      s1 = fma_c(nv, nv, s1);
      if constexpr (TOREG) outv[j] = nv;
    }
    if constexpr (!TOREG) bstore<C, VZ, FDTD_AUX_OUT>(plane_rsrc(k.out, x, k.N, k.pbytes), ln.off[0], o);
    acc[0] += (double)s0;
    acc[1] += (double)kin;
    acc[2] += (double)pot;
    acc[3] += (double)r2 + (double)rx2 * (double)s0;
    acc[4] += (double)s1;
    asm volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]));
  }

  // Stage X (slot SL = (X - base) % RS, base = xb - 1): prefetch, step t at
  // plane X into registers and LDS buffer X & 1, then (STEP2) step t + 1 at
  // plane X - 1, then the work-group barrier.
  // The y / z neighbours of the lane's own vector from an LDS plane, as
  // stored (FP32 arithmetic).  A vector outside the lattice reads whatever
  // its LDS neighbours hold: it takes c = 0 (tb_item), so its result, the
  // boundary value its neighbours read, is +0 all the same.  (Masking the
  // values instead cost about 20 VALU instructions per plane; FP64 lattices
  // keep zero neighbours for outside vectors, as a branch around the reads.)
  static __device__ __forceinline__ void lds_nbrs(const C* p, int obase, PlaneIn<1, VZ, C>& d) {
    static_assert(sizeof(C) == 4, "FP32 arithmetic");
    const Pack<C, VZ> pm = *reinterpret_cast<const Pack<C, VZ>*>(p + obase - RP);
    const Pack<C, VZ> pp = *reinterpret_cast<const Pack<C, VZ>*>(p + obase + RP);
#pragma unroll
    for (int j = 0; j < VZ; ++j) {
      d.ym[0][j] = pm.v[j];
      d.yp[0][j] = pp.v[j];
    }
    d.zm[0] = p[obase - 1];
    d.zp[0] = p[obase + VZ];
  }

  // Buffer of plane X (X >= -2) in the LDS tile of step-t results.
  static __device__ __forceinline__ int tbuf(int X) {
    return kTbLdsU ? (X + 3) % 3 : (X & 1);
  }

  // psi_t of plane X + 1 (slot SL + 2: own vector, halo site) into the LDS
  // copy `ptile` + ((X + 1) & 1) * TS, read by step t at plane X + 1 in the
  // next stage.
  template <int SL>
  static __device__ __forceinline__ void stage_psi(bool halo_wave, int obase, int hidx, int X,
                                                   C* ptile, const Rings& g) {
    C* p = ptile + ((X + 1) & 1) * TS;
    Pack<C, VZ> pk;
#pragma unroll
    for (int j = 0; j < VZ; ++j) pk.v[j] = g.qs[(SL + 2) % RS][0][j];
    *reinterpret_cast<Pack<C, VZ>*>(p + obase) = pk;
    if (halo_wave && (int)threadIdx.x < NH) p[hidx] = g.qh[(SL + 2) % RS][0][0];
  }

  template <int SL, bool STEP2>
  static __device__ __forceinline__ void stage(const typename B::Ctx& kb,
                                               const typename H::Ctx& kh,
                                               const typename B::Ctx& k2,
                                               const Lane<1, VZ, C>& lb, const Lane<1, 1, C>& lh,
                                               bool own, bool halo_wave, int obase, int hidx,
                                               int X, int xb, int xe, unsigned N, C* tile,
                                               C* ptile, Rings& g, double (&acc1)[5],
                                               double (&acc2)[5]) {
    B::fetch_own(kb, lb, X + 1 + D, g.qs[(SL + 2 + D) % RS]);
    B::template fetch_v<kTbVAux>(kb, lb, X + D, g.vs[(SL + D) % RS]);
    if constexpr (!kPsi) B::fetch(kb, lb, X + D, g.nb[(SL + D) % RS]);
    if (halo_wave) {
      H::fetch_own(kh, lh, X + 1 + D, g.qh[(SL + 2 + D) % RS]);
      H::template fetch_v<kTbVAux>(kh, lh, X + D, g.vh[(SL + D) % RS]);
      H::fetch(kh, lh, X + D, g.nh[(SL + D) % RS]);
    }
    // planes -1 and N lie outside the lattice: psi_{t+1} = 0 there (the
    // one-step kernel drops their stores; here they feed step t + 1)
    const bool inx = (unsigned)X < N;
    C* t = tile + tbuf(X) * TS;
    {
      // step t, own vectors: the work item's planes [xb, xe) count in the
      // reductions, the halo planes xb - 1 and xe do not.  FP32 arithmetic:
      // the sums start from -0, so the first addition folds away (x + -0 = x)
      constexpr double kZ = DT == kF64 ? 0.0 : -0.0;
      double tmp[5] = {kZ, kZ, kZ, kZ, kZ};
      C un[1][VZ];
      if constexpr (kPsi) {
        // y / z neighbours of plane X from the LDS copy written last stage
        PlaneIn<1, VZ, C> d;
        lds_nbrs(ptile + (X & 1) * TS, obase, d);
        if constexpr (kShare) {
          update_tb<true, 1>(kb, lb, X, g.qs[(SL + 1) % RS][0], g.qs[(SL + 2) % RS][0], g.dx1,
                             g.vs[SL % RS][0], d, g.bw[SL % 2], g.dw[SL % 2], tmp, un[0]);
        } else {
          B::template update_core<false, true, 1>(kb, lb, X, g.qs[SL % RS], g.qs[(SL + 1) % RS],
                                                  g.qs[(SL + 2) % RS], g.vs[SL % RS], d, tmp, true,
                                                  un);
        }
      } else {
        B::template update_core<false, true, 1>(kb, lb, X, g.qs[SL % RS], g.qs[(SL + 1) % RS],
                                                g.qs[(SL + 2) % RS], g.vs[SL % RS], g.nb[SL % RS],
                                                tmp, true, un);
      }
      if (X >= xb && X < xe) {
#pragma unroll
        for (int q = 0; q < 5; ++q) acc1[q] += tmp[q];
      }
      Pack<C, VZ> pk;
#pragma unroll
      for (int j = 0; j < VZ; ++j) {
        pk.v[j] = inx ? un[0][j] : C(0);
        if constexpr (!kTbLdsU) g.us[SL % US][0][j] = pk.v[j];
      }
      *reinterpret_cast<Pack<C, VZ>*>(t + obase) = pk;
    }
    if (halo_wave) {
      // step t, halo site (no reductions: another work item owns it)
      double tmp[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      C uh[1][1];
      H::template update_core<false, true, 0>(kh, lh, X, g.qh[SL % RS], g.qh[(SL + 1) % RS],
                                              g.qh[(SL + 2) % RS], g.vh[SL % RS], g.nh[SL % RS],
                                              tmp, true, uh);
      if ((int)threadIdx.x < NH) t[hidx] = inx ? uh[0][0] : C(0);
    }
    if constexpr (STEP2) {
      // step t + 1 at plane X - 1: psi_{t+1} planes X - 2, X - 1, X in
      // registers, the y / z neighbours of plane X - 1 from LDS.  A vector
      // outside the lattice must add nothing to the norm (its result is not
      // stored): FP64 gives it zero neighbours, as its loads in the one-step
      // kernel; FP32 arithmetic gives it c = 0.
      const C* tp = tile + tbuf(X - 1) * TS;
      PlaneIn<1, VZ, C> d;
      if constexpr (DT == kF64) {
        const Pack<C, VZ> pm = *reinterpret_cast<const Pack<C, VZ>*>(tp + obase - RP);
        const Pack<C, VZ> pp = *reinterpret_cast<const Pack<C, VZ>*>(tp + obase + RP);
#pragma unroll
        for (int j = 0; j < VZ; ++j) {
          d.ym[0][j] = own ? pm.v[j] : C(0);
          d.yp[0][j] = own ? pp.v[j] : C(0);
        }
        d.zm[0] = own ? tp[obase - 1] : C(0);
        d.zp[0] = own ? tp[obase + VZ] : C(0);
      } else {
        lds_nbrs(tp, obase, d);
      }
      if constexpr (kTbLdsU) {
        // planes X - 2, X - 1, X of the lane's own vector (X: written by this
        // lane in this stage, so no barrier is needed for it)
        C u0[1][VZ], u1[1][VZ], u2[1][VZ];
        const Pack<C, VZ> a0 = *reinterpret_cast<const Pack<C, VZ>*>(tile + tbuf(X - 2) * TS + obase);
        const Pack<C, VZ> a1 = *reinterpret_cast<const Pack<C, VZ>*>(tp + obase);
        const Pack<C, VZ> a2 = *reinterpret_cast<const Pack<C, VZ>*>(tile + tbuf(X) * TS + obase);
#pragma unroll
        for (int j = 0; j < VZ; ++j) {
          u0[0][j] = a0.v[j];
          u1[0][j] = a1.v[j];
          u2[0][j] = a2.v[j];
        }
        B::template update<false>(k2, lb, X - 1, u0, u1, u2, g.vs[(SL + RS - 1) % RS], d, acc2);
      } else if constexpr (kShare) {
        C unused[VZ];
        update_tb<false, 2>(k2, lb, X - 1, g.us[(SL + US - 1) % US][0], g.us[SL % US][0], g.dx2,
                            g.vs[(SL + RS - 1) % RS][0], d, g.bw[(SL + 1) % 2], g.dw[(SL + 1) % 2], acc2,
                            unused);
      } else {
        B::template update<false>(k2, lb, X - 1, g.us[(SL + US - 2) % US], g.us[(SL + US - 1) % US],
                                  g.us[SL % US], g.vs[(SL + RS - 1) % RS], d, acc2);
      }
    }
    if constexpr (kPsi) stage_psi<SL>(halo_wave, obase, hidx, X, ptile, g);
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


// One tile work item of a two-step pass reading buffer src (see k_step2).
// FENCE: the persistent form, where the next pass's tiles (on any XCD) read
// this pass's state within the same launch: the partials are published with
// a full release fence, as the persistent one-step kernel does.
template <int DT, int VZ, int D, bool FV, bool WIDE, bool FENCE>
__device__ __forceinline__ void tb_item(const StepArgs& A, const Item& item, int src,
                                        typename Step2<DT, VZ, D, FV, WIDE>::C* tile,
                                        typename Step2<DT, VZ, D, FV, WIDE>::C* ptile,
                                        double (&s_red)[kTbThreads(DT) / 64][5], int& s_last) {
  using T = Step2<DT, VZ, D, FV, WIDE>;
  using B = typename T::B;
  using H = typename T::H;
  using C = typename T::C;
  using TV = typename B::TV;
  constexpr int BT = kTbThreads(DT);
  constexpr unsigned kES = sizeof(typename B::S);
  const int tid = threadIdx.x;
  // the waves that carry halo sites (uniform per wave)
  const bool halo_wave = __builtin_amdgcn_readfirstlane(tid >> 6) < T::NHW;
  {
    const int m = item.member;
    const MemberDev& M = A.members[m];
    const int N = M.N;
    const unsigned P = (unsigned)M.plane;
    const double cN = (double)(N - 1), ha = M.ha;
    const long long step = ld_agent(A.states[m].step);
    const int y0 = item.f0 / N, z0 = item.f0 - y0 * N;  // tile origin

    typename B::Ctx kb;
    kb.in = M.psi[src];
    kb.out = M.psi[src ^ 1];  // unused: step t goes to registers
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
    kh.c = (C)M.c;
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
    if constexpr (DT != kF64) {
      // FP32 arithmetic: the own vectors' y / z neighbours of step t + 1 (and,
      // with the LDS copy of psi_t, of step t) come from LDS unmasked.  A
      // vector outside the lattice has psi = 0 (its loads read zeros) and
      // takes c = 0, so its result and its sums are +0 whatever its neighbours
      // hold, as with zero neighbours.  (The halo sites keep c.)
      kb.c = own ? kb.c : C(0);
      k2.c = kb.c;
    }
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
      if constexpr (!T::kPsi) B::fetch(kb, lb, base + i, g.nb[i]);
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
    if constexpr (T::kPsi) {
      // the LDS copy of plane base (slot 1), read by the first stage
      T::template stage_psi<T::RS - 1>(halo_wave, obase, hidx, base - 1, ptile, g);
      lds_barrier();
    }
#define FDTD_STAGE2(SL, S2, XX)                                                                  \
  T::template stage<SL, S2>(kb, kh, k2, lb, lh, own, halo_wave, obase, hidx, XX, xb, xe,         \
                            (unsigned)N, tile, ptile, g, acc1, acc2)
    // the x-difference step t carries into plane base: q(base) - q(base - 1)
    if constexpr (T::kShare) {
#pragma unroll
      for (int j = 0; j < VZ; ++j) g.dx1[j] = g.qs[1][0][j] - g.qs[0][0][j];
    }
    // planes xb - 1 and xb: step t only; then both steps, six stages a trip
    FDTD_STAGE2(0, false, base);
    FDTD_STAGE2(1, false, base + 1);
    // the x-difference step t + 1 carries into plane xb: u(xb) - u(xb - 1)
    if constexpr (T::kShare) {
#pragma unroll
      for (int j = 0; j < VZ; ++j) g.dx2[j] = g.us[1][0][j] - g.us[0][0][j];
    }
    int X = xb + 1;
    if constexpr (T::RS == 6) {
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
    } else {
      static_assert(T::RS == 8, "ring of 6 or 8 slots");
      for (; X + 8 <= xe + 1; X += 8) {
        FDTD_STAGE2(2, true, X);
        FDTD_STAGE2(3, true, X + 1);
        FDTD_STAGE2(4, true, X + 2);
        FDTD_STAGE2(5, true, X + 3);
        FDTD_STAGE2(6, true, X + 4);
        FDTD_STAGE2(7, true, X + 5);
        FDTD_STAGE2(0, true, X + 6);
        FDTD_STAGE2(1, true, X + 7);
      }
      if (X <= xe) FDTD_STAGE2(2, true, X);
      if (X + 1 <= xe) FDTD_STAGE2(3, true, X + 1);
      if (X + 2 <= xe) FDTD_STAGE2(4, true, X + 2);
      if (X + 3 <= xe) FDTD_STAGE2(5, true, X + 3);
      if (X + 4 <= xe) FDTD_STAGE2(6, true, X + 4);
      if (X + 5 <= xe) FDTD_STAGE2(7, true, X + 5);
      if (X + 6 <= xe) FDTD_STAGE2(0, true, X + 6);
    }
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
      unsigned int done;
      if constexpr (FENCE) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          p1[q] = v[0][q];
          p2[q] = v[1][q];
        }
        __threadfence();
        done = atomicAdd(&A.states[m].counter, 1u);
      } else {
        done = publish_partials<2>(dst, v, &A.states[m].counter);
      }
      s_last = (done + 1u == (unsigned int)(M.tb_end - M.tb_begin));
    }
    __syncthreads();
    if (s_last) {
      if constexpr (FENCE) __threadfence();
      double t1[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, t2[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      for (int i = M.tb_begin + tid; i < M.tb_end; i += BT) {
        const double* p1 = A.partials + (long long)i * kRec;
        const double* p2 = A.partials + (long long)(A.slot_stride + i) * kRec;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          t1[q] += FENCE ? p1[q] : ld_agent(p1[q]);
          t2[q] += FENCE ? p2[q] : ld_agent(p2[q]);
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

template <int DT, int VZ, int D, bool FV, bool WIDE>
__global__ __launch_bounds__(kTbThreads(DT), tb_min_waves(DT)) void k_step2(StepArgs A) {
  using T = Step2<DT, VZ, D, FV, WIDE>;
  __shared__ __align__(16) typename T::C tile[kTbTileBufs * T::TS];
  __shared__ __align__(16) typename T::C ptile[T::kPsi ? 2 * T::TS : 4];
  __shared__ double s_red[kTbThreads(DT) / 64][5];
  __shared__ int s_last;
  for (int li = blockIdx.x; li < A.n_items; li += gridDim.x)
    tb_item<DT, VZ, D, FV, WIDE, false>(A, A.items[A.item_offset + li], A.src, tile, ptile, s_red,
                                        s_last);
}

// Persistent two-step passes: A.steps passes (2 A.steps steps) of every
// member in one launch.  Work-groups take tickets k = p * n_items + i in
// increasing order (tile i in processing order, pass p; buffers alternate
// with p).  Before tile i of pass p, thread 0 polls until the tile's member
// has finalised both steps of pass p - 1 (its `fin` counter, reset to 0
// before the launch, reaches 2p; each finalised step raises it by one).  The
// waits end for the reason the persistent one-step kernel's do: the tiles
// waited on hold smaller tickets.  The same bounded poll and abort flag guard
// them.  Per-tile arithmetic, partial slots and summation order are those of
// k_step2: the same bits as one launch per pass.
template <int DT, int VZ, int D, bool FV, bool WIDE>
__global__ __launch_bounds__(kTbThreads(DT), tb_min_waves(DT)) void k_step2_persist(StepArgs A) {
  using T = Step2<DT, VZ, D, FV, WIDE>;
  __shared__ __align__(16) typename T::C tile[kTbTileBufs * T::TS];
  __shared__ __align__(16) typename T::C ptile[T::kPsi ? 2 * T::TS : 4];
  __shared__ double s_red[kTbThreads(DT) / 64][5];
  __shared__ int s_last;
  __shared__ int s_tk;
  const int tid = threadIdx.x;
  const int total = A.steps * A.n_items;
  for (;;) {
    if (tid == 0) {
      int tk = (int)atomicAdd(&A.ctrl->ticket, 1u);
      if (tk < total) {
        const unsigned need = 2u * (unsigned)(tk / A.n_items);
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
    const int pass = tk / A.n_items;
    tb_item<DT, VZ, D, FV, WIDE, true>(A, A.items[tk % A.n_items], A.src ^ (pass & 1), tile,
                                       ptile, s_red, s_last);
  }
}


template <int DT, int D, bool FV, bool WIDE>
hipError_t step2_one(int grid, bool persist, const StepArgs& a, hipStream_t s) {
  if (persist)
    hipLaunchKernelGGL((k_step2_persist<DT, kTbVec(DT), D, FV, WIDE>), dim3(grid), dim3(kTbThreads(DT)),
                       0, s, a);
  else
    hipLaunchKernelGGL((k_step2<DT, kTbVec(DT), D, FV, WIDE>), dim3(grid), dim3(kTbThreads(DT)), 0, s,
                       a);
  return hipGetLastError();
}

template <int DT, bool FV, bool WIDE>
hipError_t step2_depth(int depth, int grid, bool persist, const StepArgs& a, hipStream_t s) {
  switch (depth) {
    case 1: return step2_one<DT, 1, FV, WIDE>(grid, persist, a, s);
    case 2: return step2_one<DT, 2, FV, WIDE>(grid, persist, a, s);
    case 3: return step2_one<DT, 3, FV, WIDE>(grid, persist, a, s);
    case 4:  // FP32-arithmetic lattices only (a ring of 8 plane slots)
      if constexpr (DT != kF64) return step2_one<DT, 4, FV, WIDE>(grid, persist, a, s);
      else return hipErrorInvalidValue;
    case 5:  // the same ring, every slot in use
      if constexpr (DT != kF64) return step2_one<DT, 5, FV, WIDE>(grid, persist, a, s);
      else return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

// F32 / BF16 lattices: the tile shape (32 x 64, or 16 x 128 with wide)
template <int DT, bool FV>
hipError_t step2_tile(int depth, bool wide, int grid, bool persist, const StepArgs& a,
                      hipStream_t s) {
  return wide ? step2_depth<DT, FV, true>(depth, grid, persist, a, s)
              : step2_depth<DT, FV, false>(depth, grid, persist, a, s);
}

}  // namespace

hipError_t launch_step2(int dtype, int depth, bool fv, bool wide, int grid, bool persist,
                        const StepArgs& a, hipStream_t s) {
  if (grid < 1 || (persist && (a.steps < 1 || !a.ctrl))) return hipErrorInvalidValue;
  switch (dtype) {
    case kF64:
      return fv || wide ? hipErrorInvalidValue : step2_depth<kF64, false, false>(depth, grid, persist, a, s);
    case kF32: return fv ? step2_tile<kF32, true>(depth, wide, grid, persist, a, s)
                         : step2_tile<kF32, false>(depth, wide, grid, persist, a, s);
    case kBF16: return fv ? step2_tile<kBF16, true>(depth, wide, grid, persist, a, s)
                          : step2_tile<kBF16, false>(depth, wide, grid, persist, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fdtd
