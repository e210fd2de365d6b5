// Internal declarations shared by the HIP kernels and the host runtime of
// libfdtd.  Device-side descriptors, work items and kernel launch wrappers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdtd {

constexpr int kBlock = 256;  // threads per work-group: 4 wave64s
constexpr int kRec = 8;      // doubles per observable record

// Layout of one observable record (per member, per step).
enum RecordField {
  kS0 = 0,     // sum psi^2 of the state entering the step
  kKin = 1,    // kinetic energy sum: -(1/2m a^2) sum psi * (a^2 lap psi)
  kPot = 2,    // sum V psi^2
  kR2 = 3,     // sum r^2 psi^2
  kS0Out = 4,  // sum psi'^2 of the written state
  kStep = 5,   // step index
  kScale = 6,  // scale folded into this step's update
  kSpare = 7
};

// Read-only description of one lattice, resident on the device.
struct MemberDev {
  void* psi[2];       // ping-pong state buffers (storage dtype)
  const void* V;      // potential (double when psi is FP64, float otherwise)
  int N;
  int item_begin;     // this member's work items are [item_begin, item_end)
  int item_end;
  int tb_begin;       // its tiles of two-step passes are [tb_begin, tb_end)
  long long plane;    // N * N
  double ha;          // a / 2 (site coordinate = (2 i - (N - 1)) * ha)
  double c;           // dt / (2 m a^2)
  double dt;
  double kin_scale;   // 1 / (2 m a^2)
  double a3;          // a^3
  double a;           // lattice spacing
  double vp[3];       // parameters of an analytic potential (kind vkind)
  int vkind;          // analytic kind 0..4 the step may evaluate itself; -1: table only
  int tb_end;
};

// Mutable per-member state, resident on the device.
struct MemberState {
  double scale;         // multiplies the next step's update (deferred renormalisation)
  long long step;       // steps taken
  unsigned int counter; // work items finished in the current launch
  int bad;              // a reduction went non-finite
  long long bad_step;
  unsigned int fin;     // steps finalised since the last persistent-launch reset
  unsigned int pad0;
  double spare[2];
};

// Work dispenser of the persistent step kernel (in the workspace): tickets
// t * n_items + i hand out item i of step t in increasing order.
struct Control {
  unsigned int ticket;  // next ticket
  int abort;            // a dependency wait exceeded its bound: results invalid
  unsigned int pad[62];
};

// One work item: a chunk of a member's flattened (y, z) plane, for planes
// x in [xb, xe).  slot: where the item's partial sums go; a member's slots
// are [item_begin, item_end), whatever order the items are processed in.
struct Item {
  int member;
  int f0;
  int xb;
  int xe;
  int slot;
};

struct StepArgs {
  const MemberDev* members;
  MemberState* states;
  const Item* items;
  int item_offset;      // this launch processes items [item_offset, item_offset + n_items)
  int n_items;
  int src;              // input buffer index (0 / 1); the output is src ^ 1
  int renorm_every;     // > 0: rescale after every k-th step
  int set_scale;        // observe mode: set scale = 1 / sqrt(a^3 S0)
  double* partials;     // kRec doubles per item slot
  double* ring;         // history: n_members * ring_cap * kRec
  int ring_cap;
  double* obs_out;      // observe mode: n_members * kRec
  int slot_stride;      // two-step passes: step t + 1's partials at slot_stride + slot
  // persistent launches only
  int steps;            // steps this launch advances every member
  unsigned int spin_limit;  // polls of a dependency wait before it gives up
  Control* ctrl;
};

enum DType { kF64 = 0, kF32 = 1, kBF16 = 2 };

// Launch the fused step (update = true) or the reduction-only pass.
// depth: prefetch distance of the HBM streams, in planes (1..3).
// bt: threads per work-group, 256, or 512 for ry = 1.
// fv: evaluate the members' analytic potentials in the kernel (F32 / BF16,
// bt = 256; every member's vkind must be >= 0) instead of reading V.
// wt: store the updated state written through (it stays in the last-level
// cache for the next step) instead of streamed past the caches; update with
// 256-lane groups, vz = the dtype's vector width and ry <= 2 only.
hipError_t launch_step(int dtype, int vz, int ry, int depth, bool update, int grid, int bt,
                       bool fv, bool wt, const StepArgs& a, hipStream_t s);
// Two steps per pass (temporal blocking, update only): work items
// are tiles of kTbRows(dtype, wide) x kTbCols(dtype, wide) sites of the (y, z)
// plane, whose f0 is the tile origin y0 N + z0; one vector of kTbVec(dtype)
// sites per lane (kTbThreads(dtype) lanes); depth 1..5 (4 and 5: F32 / BF16);
// partials for 2 * slot_stride slots.
// persist: one persistent launch of a.steps passes (2 a.steps steps; `grid`
// work-groups take (pass, tile) tickets, a tile of pass p waiting until its
// member has finalised pass p - 1); launch_persist_reset must run first.
// Lanes of a two-step work-group: 512 for FP32-arithmetic lattices (a 32 x
// 64 tile: its one-site halo frame is 9% of its sites, against 16% for the
// 16 x 64 tile of 256 lanes; 512^3 F32 197 -> 175 us per step), 256 for F64.
// wide (F32 / BF16 only): 16 x 128 tiles instead of 32 x 64.  Their frame has
// half as many column sites, each a separate cache line that an L2 can miss,
// and more row sites, which are contiguous: fewer HBM bytes per pass (a 512^3
// F32 pass with the V table 176 -> 160 us per step at depth 4), but 288 halo
// sites on five waves instead of 192 on three (more arithmetic: slower where
// the pass is bound by it, as with the in-kernel potential).
#ifndef FDTD_TB_THREADS_F32
#define FDTD_TB_THREADS_F32 512
#endif
constexpr int kTbThreads(int dtype) { return dtype == kF64 ? 256 : FDTD_TB_THREADS_F32; }  // lanes
constexpr int kTbVec(int dtype) { return dtype == kF64 ? 2 : 4; }  // sites per lane
constexpr int kTbCols(int dtype, bool wide = false) { return dtype == kF64 ? 32 : (wide ? 128 : 64); }
constexpr int kTbRows(int dtype, bool wide = false) {
  return kTbThreads(dtype) * kTbVec(dtype) / kTbCols(dtype, wide);
}
hipError_t launch_step2(int dtype, int depth, bool fv, bool wide, int grid, bool persist,
                        const StepArgs& a, hipStream_t s);

// Persistent form of launch_step (update only): `grid` work-groups take
// (step, item) tickets in order and advance every member a.steps steps; an
// item of step t waits until its member has finalised step t - 1.
// launch_persist_reset must run first on the same stream.
hipError_t launch_step_persist(int dtype, int vz, int ry, int depth, int grid, bool fv,
                               const StepArgs& a, hipStream_t s);
hipError_t launch_persist_reset(Control* ctrl, MemberState* states, int count, hipStream_t s);

// psi (storage dtype, n3 values) <- psi - phi <phi|psi> / <phi|phi>, phi in
// the arithmetic type (F64 for F64 states, F32 otherwise); sums in FP64.
// partials: project_partials_doubles() doubles of scratch; coef: 1 double,
// receives the coefficient.
hipError_t launch_project(int dtype, void* psi, const void* phi, long long n3, double* partials,
                          double* coef, hipStream_t s);
int project_partials_doubles();

// LDS-tile variant: work-groups of tile_threads(dtype) lanes, one vector of
// the dtype's width per lane; max_n sizes the LDS tile (two planes of the
// chunk plus one row above and below).
int tile_threads(int dtype);
hipError_t launch_step_tile(int dtype, int depth, bool update, int grid, int max_n,
                            const StepArgs& a, hipStream_t s);

// One thread per site, member m only.
hipError_t launch_potential(int vdtype, void* V, int N, double ha, double a, int kind,
                            const double* p_dev, int np, hipStream_t s);
hipError_t launch_initial(int dtype, void* psi, int N, uint64_t seed, uint32_t member, int kind,
                          uint32_t parity, hipStream_t s);
hipError_t launch_convert(int sdtype, const void* src, int ddtype, void* dst, long long n,
                          double scale, hipStream_t s);
// Renormalisation done by the upsample kernel itself: per-work-group FP64
// partial sums (upsample_groups(Nf) of them) and the fine member's state and
// observable record.
struct UpNorm {
  double* partials;
  MemberState* st;   // its counter must be 0 on entry; receives the scale
  double* obs;       // kRec doubles: obs[kS0] receives sum psi^2
  double a3;         // fine a^3
};
constexpr int kUpSitesZ = 4;    // fine z sites per thread of the upsample kernel
constexpr int kUpPlanes = 32;   // fine planes per work-group
inline long long upsample_groups(int Nf) {
  const long long nzv = (Nf + kUpSitesZ - 1) / kUpSitesZ;
  return (((long long)Nf * nzv + kBlock - 1) / kBlock) * ((Nf + kUpPlanes - 1) / kUpPlanes);
}
hipError_t launch_upsample(int cdtype, const void* pc, int Nc, double hac, double ac, int fdtype,
                           void* pf, int Nf, double haf, const UpNorm& u, hipStream_t s);
hipError_t launch_reimpose(int dtype, void* psi, int N, uint32_t parity, hipStream_t s);
hipError_t launch_set_state(MemberState* st, int member, double scale, long long step,
                            int reset_bad, hipStream_t s);

// ---- adjoint (gradient) kernels ------------------------------------------------
struct AdjArgs {
  const void* V;        // float (F32 path) or double (F64 path)
  const void* lam_in;   // lambda_{t+1}
  void* lam_out;        // lambda_t
  const void* psi_t;    // psi_t  (as stored by the forward)
  const void* psi_t1;   // psi_{t+1}
  void* G;              // dE/dV accumulator: FP64 on the F64 path; on the F32
                        // path an FP32 accumulator of the current checkpoint
                        // segment, folded into the FP64 sum by launch_fold_grad
  int N;
  int nx;               // x-ranges per chunk column (set by launch_adjoint_step)
  double c, dt;
  double s_t;           // scale applied in forward step t
};
hipError_t launch_adjoint_step(int dtype, const AdjArgs& a, hipStream_t s);
// G64 += G32 and G32 = 0 over n sites (the end of a checkpoint segment).
hipError_t launch_fold_grad(double* G64, float* G32, long long n, hipStream_t s);

struct AdjInitArgs {
  const void* V;
  const void* psi;      // psi_T
  void* lam;            // out: 2 (H psi - E psi) / S0
  double* G;            // out: psi^2 / S0
  float* G32;           // F32 path: out: 0 (the segment accumulator); else null
  int N;
  int pad0;
  double kin_scale;     // 1 / (2 m a^2)
  double E, S0;
};
hipError_t launch_adjoint_init(int dtype, const AdjInitArgs& a, hipStream_t s);

// dE/dtheta_j = sum_i G_i dV_i/dtheta_j for the parameters of an analytic
// potential of kind `kind` (the FDTD_POT_* numbering), lattice spacing a.
hipError_t launch_param_contract(const double* G, int N, double ha, double a, int kind,
                                 const double* p_dev, int np, const int* wrt_dev, int nwrt,
                                 double* partials, int nblocks, double* out_dev, hipStream_t s);

}  // namespace fdtd
