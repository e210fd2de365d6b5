// Host runtime of libfdtd: handles, device memory layout, work items, the
// evolution loop (direct launches or a replayed HIP graph), observables,
// upsampling, the adjoint gradient driver and the launch-shape autotuner.
// Exposes the C ABI declared in include/fdtd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fdtd.h"
#include "fdtd_internal.h"

using namespace fdtd;

namespace {

thread_local std::string g_err;

fdtd_status fail(fdtd_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

fdtd_status hip_fail(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return FDTD_EHIP;
}

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);   \
  } while (0)

#define ST_TRY(expr)                 \
  do {                               \
    fdtd_status s_ = (expr);         \
    if (s_ != FDTD_OK) return s_;    \
  } while (0)

size_t elem_size(int dt) { return dt == kF64 ? 8 : (dt == kF32 ? 4 : 2); }
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
int vec_width(int dt) { return dt == kF64 ? 2 : (dt == kF32 ? 4 : 8); }

struct MemberHost {
  int N = 0;
  double L = 0, mass = 1, dt = 0, v_inf = 0;
  double a = 0, ha = 0, c = 0, kin_scale = 0, a3 = 0;
  long long n3 = 0;
  size_t off_psi[2] = {0, 0}, off_V = 0;
  bool pot_set = false, init_set = false;
  uint32_t parity = 0;
  int item_begin = 0, item_end = 0;
  int tb_begin = 0, tb_end = 0;  // tiles of two-step passes (member order)
  int vkind = -1;  // analytic kind the step may evaluate itself (0..4), -1: table only
  double vp[3] = {0, 0, 0};
  int pkind = -1;              // analytic kind V was set from (-1: a caller's array)
  std::vector<double> params;  // its parameters (for the gradient's contraction)
  long long hist_from = 0;  // first step whose record the history ring holds
  int nproj = 0;          // states kept for projection (Sec. III)
  void* proj = nullptr;   // nproj * n3 values of the arithmetic type (library-owned)
};

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  int K = 0, renorm = 0, src = 0;
  int dst = 0;  // buffer holding the state after the K steps (a two-step pass flips once)
  fdtd_tuning tun{};
};

}  // namespace

struct fdtd_ctx {
  int count = 0;
  int dtype = kF32;
  int vdtype = kF32;
  int device = 0;
  int ring_cap = 4096;
  hipStream_t stream = nullptr;
  hipStream_t capture_stream = nullptr;
  std::vector<MemberHost> mem;

  // device memory
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
  size_t off_members = 0, off_states = 0, off_ring = 0, off_obs = 0, off_params = 0, off_ctrl = 0;
  size_t off_upart = 0;  // partial sums of the upsample kernel's norm (largest member)
  size_t need_bytes = 0;

  // work items (library-allocated, depend on the tuning): d_items in member
  // order (a member's items at [item_begin, item_end), for per-member
  // launches), d_order the same items in the order whole-batch launches
  // process them, d_titems the tiles of two-step passes in processing order
  // (tblock = 2 only); one allocation of 2 * items_cap + titems_cap
  Item* d_items = nullptr;
  Item* d_order = nullptr;
  Item* d_titems = nullptr;
  double* d_partials = nullptr;
  int n_items = 0;
  int items_cap = 0;
  int n_titems = 0;
  int titems_cap = 0;
  bool items_valid = false;

  int cur = 0;  // buffer holding the current state (all members)
  fdtd_tuning tun{};
  bool tuned = false;
  bool table_v_only = false;  // set while the gradient driver recomputes the forward
  int n_cu = 256;  // compute units of the device: work-groups of a persistent launch
  std::string arch = "gfx";  // the device's architecture name (gfx950 ...), for tuning keys
  unsigned spin_limit = 1u << 22;  // polls of a persistent dependency wait

  // pinned host staging for small readbacks
  double* h_pin = nullptr;
  size_t h_pin_doubles = 0;

  std::vector<GraphEntry> graphs;

  // projection scratch: per-work-group partial sums and the coefficients
  double* d_proj = nullptr;

  // device memory of fdtd_energy_grad: bound by the caller, or allocated by
  // the library and kept for later calls
  char* gws = nullptr;
  size_t gws_bytes = 0;
  bool gws_owned = false;

  // counters (fdtd_get_counters)
  long long n_captures = 0;  // HIP graphs captured
  long long n_replays = 0;   // HIP graph launches
  long long n_allocs = 0;    // device and pinned host allocations made for the handle

  MemberDev* d_members() { return reinterpret_cast<MemberDev*>(ws + off_members); }
  MemberState* d_states() { return reinterpret_cast<MemberState*>(ws + off_states); }
  double* d_ring() { return reinterpret_cast<double*>(ws + off_ring); }
  double* d_obs() { return reinterpret_cast<double*>(ws + off_obs); }
  double* d_params() { return reinterpret_cast<double*>(ws + off_params); }
  Control* d_ctrl() { return reinterpret_cast<Control*>(ws + off_ctrl); }
  double* d_upart() { return reinterpret_cast<double*>(ws + off_upart); }
  void* psi(int m, int b) { return ws + mem[m].off_psi[b]; }
  void* V(int m) { return ws + mem[m].off_V; }
};

namespace {

// Every allocation made for a handle goes through these two (counted).
hipError_t dev_malloc(fdtd_ctx* h, void** p, size_t bytes) {
  ++h->n_allocs;
  return hipMalloc(p, bytes);
}

hipError_t host_malloc(fdtd_ctx* h, void** p, size_t bytes) {
  ++h->n_allocs;
  return hipHostMalloc(p, bytes, hipHostMallocDefault);
}

constexpr int kMaxParams = 3 + 5 * 256;

void compute_layout(fdtd_ctx* h) {
  size_t off = 0;
  const size_t es = elem_size(h->dtype), vs = elem_size(h->vdtype);
  for (auto& m : h->mem) {
    m.off_psi[0] = off;
    off = align256(off + es * (size_t)m.n3);
    m.off_psi[1] = off;
    off = align256(off + es * (size_t)m.n3);
    m.off_V = off;
    off = align256(off + vs * (size_t)m.n3);
  }
  h->off_members = off;
  off = align256(off + sizeof(MemberDev) * h->count);
  h->off_states = off;
  off = align256(off + sizeof(MemberState) * h->count);
  h->off_ring = off;
  off = align256(off + sizeof(double) * kRec * (size_t)h->ring_cap * h->count);
  h->off_obs = off;
  off = align256(off + sizeof(double) * kRec * h->count);
  h->off_params = off;
  off = align256(off + sizeof(double) * (kMaxParams + 64));
  h->off_ctrl = off;
  off = align256(off + sizeof(Control));
  long long groups = 1;
  for (auto& m : h->mem) groups = std::max(groups, upsample_groups(m.N));
  h->off_upart = off;
  off = align256(off + sizeof(double) * (size_t)groups);
  h->need_bytes = off;
}

fdtd_status validate_cfg(const fdtd_config& c, const char* who) {
  if (c.n < 2 || c.n > 8192) return fail(FDTD_EINVAL, std::string(who) + ": n must be in [2, 8192]");
  if (!(c.box_len > 0) || !std::isfinite(c.box_len)) return fail(FDTD_EINVAL, std::string(who) + ": box_len must be > 0");
  if (!(c.mass > 0) || !std::isfinite(c.mass)) return fail(FDTD_EINVAL, std::string(who) + ": mass must be > 0");
  if (!(c.dt > 0) || !std::isfinite(c.dt)) return fail(FDTD_EINVAL, std::string(who) + ": dt must be > 0");
  if (!std::isfinite(c.v_inf)) return fail(FDTD_EINVAL, std::string(who) + ": v_inf must be finite");
  if (c.psi_dtype < FDTD_F64 || c.psi_dtype > FDTD_BF16) return fail(FDTD_EINVAL, std::string(who) + ": bad psi_dtype");
  if (c.history < 0) return fail(FDTD_EINVAL, std::string(who) + ": history must be >= 0");
  const double a = c.box_len / c.n;
  if (!(c.dt < c.mass * a * a / 3.0)) {
    char buf[160];
    snprintf(buf, sizeof buf, "%s: dt = %.6g violates the stability bound dt < m a^2 / 3 = %.6g", who,
             c.dt, c.mass * a * a / 3.0);
    return fail(FDTD_EUNSTABLE, buf);
  }
  return FDTD_OK;
}

fdtd_status make_ctx(const fdtd_config* cfgs, int count, fdtd_t* out) {
  if (!cfgs || !out || count < 1) return fail(FDTD_EINVAL, "create: null argument or count < 1");
  *out = nullptr;
  for (int i = 0; i < count; ++i) {
    ST_TRY(validate_cfg(cfgs[i], "create"));
    if (cfgs[i].psi_dtype != cfgs[0].psi_dtype)
      return fail(FDTD_EINVAL, "create_batch: every member must share psi_dtype");
  }
  fdtd_ctx* h = new (std::nothrow) fdtd_ctx();
  if (!h) return fail(FDTD_ENOMEM, "create: host allocation failed");
  h->count = count;
  h->dtype = cfgs[0].psi_dtype;
  h->vdtype = h->dtype == kF64 ? kF64 : kF32;
  h->device = cfgs[0].device;
  h->ring_cap = cfgs[0].history > 0 ? cfgs[0].history : 4096;
  h->stream = static_cast<hipStream_t>(cfgs[0].stream);
  h->mem.resize(count);
  for (int i = 0; i < count; ++i) {
    MemberHost& m = h->mem[i];
    m.N = cfgs[i].n;
    m.L = cfgs[i].box_len;
    m.mass = cfgs[i].mass;
    m.dt = cfgs[i].dt;
    m.v_inf = cfgs[i].v_inf;
    m.a = m.L / m.N;
    m.ha = 0.5 * m.a;
    m.c = m.dt / (2.0 * m.mass * m.a * m.a);
    m.kin_scale = 1.0 / (2.0 * m.mass * m.a * m.a);
    m.a3 = m.a * m.a * m.a;
    m.n3 = (long long)m.N * m.N * m.N;
  }
  compute_layout(h);
  // default launch shape: widest vector the sizes allow
  const int vw = vec_width(h->dtype);
  bool all_div = true;
  for (auto& m : h->mem) all_div = all_div && (m.N % vw == 0);
  h->tun.vz = all_div ? vw : 1;
  // vectors per lane: two (BF16: one), but one on a small single lattice,
  // whose planes then split into twice as many work-item chunks.  Measured
  // per step with the automatic x-chunk, two -> one: FP32 128^3 15.2 -> 13.4
  // us, 160^3 27.4 -> 16.5, 176^3 28.0 -> 19.5 (192^3 22.6 -> 22.9, 256^3
  // 35.2 -> 36.5); FP64 64^3 11.6 -> 9.5, 96^3 12.6 -> 11.9 (128^3 16.2 ->
  // 16.6).  Batches keep two (64 lattices of side 48..160: 245.7 against
  // 267.7 us).
  h->tun.ry = (h->dtype == kBF16 && h->tun.vz > 1) ? 1 : 2;
  if (h->count == 1 && h->tun.vz > 1) {
    const int small = h->dtype == kF32 ? 176 : (h->dtype == kF64 ? 96 : 0);
    if (h->mem[0].N <= small) h->tun.ry = 1;
  }
  h->tun.xchunk = 0;  // automatic: see auto_xchunk
  h->tun.grid = 0;
  h->tun.xcd_remap = 1;
  h->tun.depth = 1;
  // a single lattice whose fields fit in the last-level cache (256 MB MALL)
  // keeps the state written there for the next step: variant 3 (256^3 FP32
  // 51.7 -> 42.5 us, 320^3 101.9 -> 88.5 us per step; neutral to slightly
  // slower from 384^3 FP32 up)
  long long field_bytes = 0;
  for (auto& m : h->mem)
    field_bytes += m.n3 * (long long)(2 * elem_size(h->dtype) + (h->dtype == kF64 ? 8 : 4));
  h->tun.variant = (h->count == 1 && all_div && field_bytes <= (512LL << 20)) ? 3 : 0;
  // batches: one persistent launch per 64 steps lets the next step of a
  // finished lattice fill the end of the current one (measured on 64 lattices
  // of side 48..160: 299 -> 257 us per step); a single lattice keeps one
  // launch per step, whose fixed XCD-local tile order the dynamic tickets lose
  h->tun.persist = h->count > 1 ? 64 : 0;
  h->tun.vfuse = 1;
  // test hook: a small bound makes a persistent launch give up its first
  // unmet dependency wait (and drain), so the error path can be exercised
  if (const char* e = std::getenv("FDTD_PERSIST_SPIN_LIMIT")) h->spin_limit = (unsigned)std::strtoul(e, nullptr, 10);
  *out = h;
  return FDTD_OK;
}

fdtd_status set_device(fdtd_ctx* h) {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) return fail(FDTD_EHIP, "no HIP device available (the library has no CPU fallback)");
  if (h->device < 0 || h->device >= n) return fail(FDTD_EINVAL, "device ordinal out of range");
  HIP_TRY(hipSetDevice(h->device));
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess && cu > 0)
    h->n_cu = cu;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) {
    std::string a(prop.gcnArchName);
    h->arch = a.substr(0, a.find(':'));  // drop the feature suffixes
  }
  return FDTD_OK;
}

MemberDev member_dev(fdtd_ctx* h, int i) {
  const MemberHost& m = h->mem[i];
  MemberDev d;
  memset(&d, 0, sizeof d);
  d.psi[0] = h->psi(i, 0);
  d.psi[1] = h->psi(i, 1);
  d.V = h->V(i);
  d.N = m.N;
  d.item_begin = m.item_begin;
  d.item_end = m.item_end;
  d.tb_begin = m.tb_begin;
  d.tb_end = m.tb_end;
  d.plane = (long long)m.N * m.N;
  d.ha = m.ha;
  d.c = m.c;
  d.dt = m.dt;
  d.kin_scale = m.kin_scale;
  d.a3 = m.a3;
  d.a = m.a;
  d.vkind = m.vkind;
  for (int k = 0; k < 3; ++k) d.vp[k] = m.vp[k];
  return d;
}

fdtd_status upload_members(fdtd_ctx* h) {
  std::vector<MemberDev> md(h->count);
  for (int i = 0; i < h->count; ++i) md[i] = member_dev(h, i);
  HIP_TRY(hipMemcpyAsync(h->d_members(), md.data(), sizeof(MemberDev) * h->count,
                         hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));  // md is a temporary
  return FDTD_OK;
}

// Device memory: bound workspace or a library allocation, made on first use.
fdtd_status ensure_memory(fdtd_ctx* h) {
  ST_TRY(set_device(h));
  if (!h->ws) {
    void* p = nullptr;
    hipError_t e = dev_malloc(h, &p, h->need_bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(FDTD_ENOMEM, "device allocation of the workspace failed");
    }
    h->ws = static_cast<char*>(p);
    h->ws_bytes = h->need_bytes;
    h->ws_owned = true;
    for (int m = 0; m < h->count; ++m) HIP_TRY(launch_set_state(h->d_states(), m, 1.0, 0, 1, h->stream));
    HIP_TRY(launch_persist_reset(h->d_ctrl(), h->d_states(), h->count, h->stream));
  }
  if (!h->h_pin) {
    h->h_pin_doubles = (size_t)kRec * (h->count + 8) + 4096;
    HIP_TRY(host_malloc(h, (void**)&h->h_pin, h->h_pin_doubles * sizeof(double)));
  }
  return FDTD_OK;
}

void xcd_permute(std::vector<int>& pos, int n) {
  // hardware dispatches work-group b to XCD b % 8: give each XCD a contiguous
  // run of work items so tiles that share halos share an L2
  pos.resize(n);
  const int q = n / 8;
  for (int b = 0; b < n; ++b) pos[b] = (b < 8 * q) ? (b % 8) * q + b / 8 : b;
}

// Sites of a plane that one work item covers.
long long chunk_sites(const fdtd_ctx* h, const fdtd_tuning& t) {
  if (t.variant == 1) return (long long)tile_threads(h->dtype) * vec_width(h->dtype);
  return (long long)(t.variant == 2 ? 512 : kBlock) * t.vz * t.ry;
}

// Near-equal split of a member's N planes into ceil(N / xc) x-ranges.
int x_parts(int N, int xc) { return (N + std::max(1, std::min(xc, N)) - 1) / std::max(1, std::min(xc, N)); }
int x_bound(int N, int nx, int b) { return (int)(((long long)b * N) / nx); }

// Two-step tiles of the tuning t: 16 x 128 (tile = 1, F32 / BF16) instead of
// the dtype's default shape.
bool tb_wide(const fdtd_ctx* h, const fdtd_tuning& t) { return t.tile == 1 && h->dtype != kF64; }

// Work items per plane of a lattice of side N: chunks of the flattened plane,
// or (two steps per pass) tiles of the (y, z) plane.
long long plane_items(const fdtd_ctx* h, const fdtd_tuning& t, int N) {
  if (t.tblock == 2) {
    const long long ty = kTbRows(h->dtype, tb_wide(h, t)), tz = kTbCols(h->dtype, tb_wide(h, t));
    return ((N + ty - 1) / ty) * ((N + tz - 1) / tz);
  }
  const long long F = chunk_sites(h, t);
  return ((long long)N * N + F - 1) / F;
}

// Longest x-stream (fewest re-read halo planes, least per-item start-up)
// that still keeps the CUs busy.  Measured (FP32, one step per pass): a
// single lattice wants about one long-streaming work-group per CU, and a few
// CUs idle beat twice as many shorter items (384^3: 216 items of 128 planes
// 132 us, 432 of 64 planes 145 us; 512^3: 256 of 256 planes 274 us, 512 of
// 128 planes 341 us), so it takes the longest stream giving at least 80% of
// the CUs an item.  On a batch, items of uneven length are handed out longest
// first and about two per CU balance best (64 lattices of side 48..160: 530
// items of at most 128 planes 234 us, 374 whole-N items 258 us, 850 of 64
// planes 244 us).  Two-step tiles: one per CU; a CU holds one 512-lane tile
// of an FP32-arithmetic lattice (two waves per SIMD) or one 256-lane FP64
// tile (one wave per SIMD: 433 against 441 us with two).  With 256-lane F32
// tiles two per CU were best (512^3: 512 tiles of 256 planes 206 us per
// step, 256 of 512 planes 297 us).
int auto_xchunk(const fdtd_ctx* h, const fdtd_tuning& t) {
  const long long cu = std::max(1, h->n_cu);
  const long long need = t.tblock == 2 ? (h->dtype == kF64 || kTbThreads(h->dtype) > 256 ? cu : 2 * cu)
                                       : (h->count > 1 ? 2 * cu : (4 * cu + 4) / 5);
  for (int xc : {512, 256, 128, 64, 32, 16}) {
    long long items = 0;
    for (const auto& m : h->mem) items += plane_items(h, t, m.N) * x_parts(m.N, xc);
    if (items >= need) return xc;
  }
  return 8;
}

// Work items of every member for the tuning t: chunks of the flattened plane
// (tiles = false) or tiles of the (y, z) plane (two steps per pass), times
// the x-ranges; phys in member order (slot = index), order in processing
// order: each member's items optionally permuted so that the work-groups one
// XCD runs take neighbouring tiles; on a batch, longest items first (stable,
// so the permutation survives among equal lengths), which keeps the slots
// busy to the end of the launch.
void make_items(fdtd_ctx* h, fdtd_tuning t, bool tiles, std::vector<Item>& phys,
                std::vector<Item>& order, std::vector<int>& begin, std::vector<int>& end) {
  t.tblock = tiles ? 2 : 0;
  if (t.xchunk == 0) t.xchunk = auto_xchunk(h, t);
  const long long F = chunk_sites(h, t);
  const int ty = kTbRows(h->dtype, tb_wide(h, t)), tz = kTbCols(h->dtype, tb_wide(h, t));
  phys.clear();
  order.clear();
  begin.assign(h->count, 0);
  end.assign(h->count, 0);
  for (int i = 0; i < h->count; ++i) {
    const int N = h->mem[i].N;
    const int nchunk = (int)plane_items(h, t, N);
    const int tz_n = (N + tz - 1) / tz;  // tiles row-major over the plane
    const int nx = x_parts(N, t.xchunk);
    begin[i] = (int)phys.size();
    for (int bx = 0; bx < nx; ++bx)
      for (int ch = 0; ch < nchunk; ++ch) {
        Item it;
        it.member = i;
        it.f0 = tiles ? (ch / tz_n) * ty * N + (ch % tz_n) * tz : (int)(ch * F);
        it.xb = x_bound(N, nx, bx);
        it.xe = x_bound(N, nx, bx + 1);
        it.slot = (int)phys.size();
        phys.push_back(it);
      }
    end[i] = (int)phys.size();
  }
  order.reserve(phys.size());
  for (int i = 0; i < h->count; ++i) {
    const int cnt = end[i] - begin[i];
    std::vector<int> p;
    if (t.xcd_remap) xcd_permute(p, cnt);
    else {
      p.resize(cnt);
      for (int b = 0; b < cnt; ++b) p[b] = b;
    }
    for (int b = 0; b < cnt; ++b) order.push_back(phys[begin[i] + p[b]]);
  }
  if (h->count > 1)
    std::stable_sort(order.begin(), order.end(),
                     [](const Item& a, const Item& b) { return a.xe - a.xb > b.xe - b.xb; });
}

void drop_graphs(fdtd_ctx* h);

fdtd_status build_items(fdtd_ctx* h) {
  if (h->items_valid) return FDTD_OK;
  // a captured graph bakes in the item and partial-sum pointers and counts of
  // the shape it was recorded with; the buffers below may be reallocated
  drop_graphs(h);
  std::vector<Item> phys, order, tphys, torder;
  std::vector<int> b, e, tb, te;
  make_items(h, h->tun, false, phys, order, b, e);
  if (h->tun.tblock == 2) make_items(h, h->tun, true, tphys, torder, tb, te);
  for (int i = 0; i < h->count; ++i) {
    h->mem[i].item_begin = b[i];
    h->mem[i].item_end = e[i];
    h->mem[i].tb_begin = tb.empty() ? 0 : tb[i];
    h->mem[i].tb_end = te.empty() ? 0 : te[i];
  }
  const int n = (int)phys.size(), nt = (int)tphys.size();
  if (n > h->items_cap || nt > h->titems_cap) {
    if (h->d_items) (void)hipFree(h->d_items);
    if (h->d_partials) (void)hipFree(h->d_partials);
    h->d_items = nullptr;
    h->d_order = nullptr;
    h->d_titems = nullptr;
    h->d_partials = nullptr;
    h->items_cap = 0;
    h->titems_cap = 0;
    const int cap = n, tcap = nt;
    // chunk items in member and processing order, then the tiles in
    // processing order; partials: one slot per chunk item, two per tile (a
    // two-step pass keeps both steps' sums)
    hipError_t e1 = dev_malloc(h, (void**)&h->d_items, sizeof(Item) * (2 * (size_t)cap + (size_t)tcap));
    hipError_t e2 = dev_malloc(h, (void**)&h->d_partials,
                              sizeof(double) * kRec * std::max((size_t)cap, 2 * (size_t)tcap));
    if (e1 != hipSuccess || e2 != hipSuccess) {
      (void)hipGetLastError();
      return fail(FDTD_ENOMEM, "device allocation of work items failed");
    }
    h->items_cap = cap;
    h->titems_cap = tcap;
  }
  h->d_order = h->d_items + h->items_cap;
  h->d_titems = h->d_order + h->items_cap;
  HIP_TRY(hipMemcpyAsync(h->d_items, phys.data(), sizeof(Item) * n, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(h->d_order, order.data(), sizeof(Item) * n, hipMemcpyHostToDevice, h->stream));
  if (nt)
    HIP_TRY(hipMemcpyAsync(h->d_titems, torder.data(), sizeof(Item) * nt, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->n_items = n;
  h->n_titems = nt;
  ST_TRY(upload_members(h));
  h->items_valid = true;
  return FDTD_OK;
}

int launch_grid(const fdtd_ctx* h, int n_items) {
  if (h->tun.grid > 0) return std::min(h->tun.grid, n_items);
  return n_items;
}

int max_n(const fdtd_ctx* h) {
  int n = 0;
  for (const auto& m : h->mem) n = std::max(n, m.N);
  return n;
}

// Launch the fused step (update) or the reduction-only pass with the
// handle's launch shape.
// The step evaluates the potential itself: FP32 / BF16 lattices, variant 0
// or 2, every member's potential one of the analytic kinds 0..4, tun.vfuse set.
bool use_fv(const fdtd_ctx* h) {
  if (!h->tun.vfuse || h->dtype == kF64 || h->tun.variant == 1 || h->table_v_only) return false;
  for (const auto& m : h->mem)
    if (m.vkind < 0) return false;
  return true;
}

hipError_t launch_kernel(const fdtd_ctx* h, bool update, int grid, const StepArgs& a,
                         hipStream_t s) {
  if (h->tun.variant == 1)
    return launch_step_tile(h->dtype, update ? std::min(h->tun.depth, 3) : 1, update, grid, max_n(h), a, s);
  // one-step launches prefetch at most 3 planes (depths 4 and 5 are the
  // two-step pass's; the odd last step of a two-step evolve takes 3)
  return launch_step(h->dtype, h->tun.vz, h->tun.ry, update ? std::min(h->tun.depth, 3) : 1, update, grid,
                     h->tun.variant == 2 ? 512 : 256, use_fv(h), h->tun.variant == 3, a, s);
}

StepArgs base_args(fdtd_ctx* h) {
  StepArgs a;
  memset(&a, 0, sizeof a);
  a.members = h->d_members();
  a.states = h->d_states();
  a.items = h->d_order;
  a.n_items = h->n_items;
  a.item_offset = 0;
  a.src = h->cur;
  a.partials = h->d_partials;
  a.ring = h->d_ring();
  a.ring_cap = h->ring_cap;
  a.obs_out = h->d_obs();
  return a;
}

// Reduction-only pass over member m (-1: all); optionally sets the scale of
// the next step to 1/sqrt(a^3 S0).  Results land in d_obs.
fdtd_status observe(fdtd_ctx* h, int member, bool set_scale) {
  ST_TRY(build_items(h));
  StepArgs a = base_args(h);
  a.set_scale = set_scale ? 1 : 0;
  if (member >= 0) {
    a.items = h->d_items;
    a.item_offset = h->mem[member].item_begin;
    a.n_items = h->mem[member].item_end - h->mem[member].item_begin;
  }
  HIP_TRY(launch_kernel(h, false, launch_grid(h, a.n_items), a, h->stream));
  return FDTD_OK;
}

// n steps: one launch per step, or with tun.persist > 0 persistent launches
// of up to tun.persist steps each (a reset kernel before each).
fdtd_status launch_steps(fdtd_ctx* h, int n, int renorm_every, hipStream_t s) {
  if (h->tun.persist > 0 && h->tun.tblock == 2 && !h->table_v_only) {
    // persistent two-step passes; an odd last step runs as a one-step launch
    int done = 0;
    while (n - done >= 2) {
      const int k = std::min({h->tun.persist, (n - done) / 2,
                              std::max(1, (1 << 30) / std::max(1, h->n_titems))});
      StepArgs a = base_args(h);
      a.renorm_every = renorm_every;
      a.items = h->d_titems;
      a.n_items = h->n_titems;
      a.slot_stride = h->n_titems;
      a.steps = k;
      a.spin_limit = h->spin_limit;
      a.ctrl = h->d_ctrl();
      const int grid = h->tun.grid > 0 ? h->tun.grid : h->n_cu;
      HIP_TRY(launch_persist_reset(a.ctrl, a.states, h->count, s));
      HIP_TRY(launch_step2(h->dtype, h->tun.depth, use_fv(h), tb_wide(h, h->tun), grid, true, a, s));
      if (k & 1) h->cur ^= 1;
      done += 2 * k;
    }
    for (; done < n; ++done) {
      StepArgs a = base_args(h);
      a.renorm_every = renorm_every;
      HIP_TRY(launch_kernel(h, true, launch_grid(h, a.n_items), a, s));
      h->cur ^= 1;
    }
    return FDTD_OK;
  }
  if (h->tun.persist > 0 && h->tun.tblock != 2) {
    for (int done = 0; done < n;) {
      // tickets (steps x items) stay below 2^30
      const int k = std::min({h->tun.persist, n - done, std::max(1, (1 << 30) / std::max(1, h->n_items))});
      StepArgs a = base_args(h);
      a.renorm_every = renorm_every;
      a.steps = k;
      a.spin_limit = h->spin_limit;
      a.ctrl = h->d_ctrl();
      const int grid = h->tun.grid > 0 ? h->tun.grid : h->n_cu;
      HIP_TRY(launch_persist_reset(a.ctrl, a.states, h->count, s));
      HIP_TRY(launch_step_persist(h->dtype, h->tun.vz, h->tun.ry, std::min(h->tun.depth, 3), grid, use_fv(h), a, s));
      if (k & 1) h->cur ^= 1;
      done += k;
    }
    return FDTD_OK;
  }
  int k = 0;
  if (h->tun.tblock == 2 && !h->table_v_only) {
    // two steps per pass; a rescale due after a pass's first step is
    // deferred to its second
    for (; k + 2 <= n; k += 2) {
      StepArgs a = base_args(h);
      a.renorm_every = renorm_every;
      a.items = h->d_titems;
      a.n_items = h->n_titems;
      a.slot_stride = h->n_titems;
      HIP_TRY(launch_step2(h->dtype, h->tun.depth, use_fv(h), tb_wide(h, h->tun), launch_grid(h, a.n_items),
                           false, a, s));
      h->cur ^= 1;  // psi_{t+2} is in the other buffer
    }
  }
  for (; k < n; ++k) {
    StepArgs a = base_args(h);
    a.renorm_every = renorm_every;
    HIP_TRY(launch_kernel(h, true, launch_grid(h, a.n_items), a, s));
    h->cur ^= 1;
  }
  return FDTD_OK;
}

bool same_tuning(const fdtd_tuning& a, const fdtd_tuning& b) {
  return a.vz == b.vz && a.ry == b.ry && a.xchunk == b.xchunk && a.grid == b.grid &&
         a.xcd_remap == b.xcd_remap && a.depth == b.depth && a.variant == b.variant &&
         a.persist == b.persist && a.vfuse == b.vfuse && a.tblock == b.tblock && a.tile == b.tile;
}

void drop_graphs(fdtd_ctx* h) {
  for (auto& g : h->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  h->graphs.clear();
}

// Run K steps through a cached, replayed HIP graph.
fdtd_status graph_steps(fdtd_ctx* h, int K, int renorm_every) {
  GraphEntry* ge = nullptr;
  for (auto& g : h->graphs)
    if (g.K == K && g.renorm == renorm_every && g.src == h->cur && same_tuning(g.tun, h->tun)) ge = &g;
  if (!ge) {
    if (!h->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    const int cur0 = h->cur;
    HIP_TRY(hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal));
    fdtd_status st = launch_steps(h, K, renorm_every, h->capture_stream);
    hipError_t e = hipStreamEndCapture(h->capture_stream, &graph);
    const int cur1 = h->cur;
    h->cur = cur0;
    if (st != FDTD_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    ++h->n_captures;
    if (h->graphs.size() >= 8) drop_graphs(h);
    GraphEntry g;
    g.exec = exec;
    g.K = K;
    g.renorm = renorm_every;
    g.src = cur0;
    g.dst = cur1;
    g.tun = h->tun;
    h->graphs.push_back(g);
    ge = &h->graphs.back();
  }
  HIP_TRY(hipGraphLaunch(ge->exec, h->stream));
  ++h->n_replays;
  h->cur = ge->dst;
  return FDTD_OK;
}

fdtd_status require_ready(fdtd_ctx* h) {
  for (int i = 0; i < h->count; ++i) {
    if (!h->mem[i].pot_set) return fail(FDTD_ENOTREADY, "potential not set for member " + std::to_string(i));
    if (!h->mem[i].init_set) return fail(FDTD_ENOTREADY, "initial state not set for member " + std::to_string(i));
  }
  return FDTD_OK;
}

// Copy member states (device) to the host; fails if a persistent launch
// gave up a dependency wait (its results are then invalid).
fdtd_status read_states(fdtd_ctx* h, std::vector<MemberState>& out) {
  out.resize(h->count);
  Control c;
  HIP_TRY(hipMemcpyAsync(out.data(), h->d_states(), sizeof(MemberState) * h->count,
                         hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipMemcpyAsync(&c, h->d_ctrl(), sizeof c, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (c.abort)
    return fail(FDTD_EHIP, "persistent step: a dependency wait exceeded its bound; the state is invalid");
  return FDTD_OK;
}

fdtd_status check_bad(fdtd_ctx* h, const std::vector<MemberState>& st) {
  for (int i = 0; i < h->count; ++i)
    if (st[i].bad) {
      char buf[128];
      snprintf(buf, sizeof buf, "non-finite reduction in member %d at step %lld", i,
               (long long)st[i].bad_step);
      return fail(FDTD_ENONFINITE, buf);
    }
  return FDTD_OK;
}

fdtd_obs to_obs(const MemberHost& m, const double* r, long long step) {
  fdtd_obs o;
  const double s0 = r[kS0];
  o.norm2 = m.a3 * s0;
  o.kinetic = r[kKin] / s0;
  o.potential = r[kPot] / s0;
  o.energy = (r[kKin] + r[kPot]) / s0;
  o.r_rms = std::sqrt(r[kR2] / s0);
  o.binding = o.energy - m.v_inf;
  o.step = step;
  o.tau = (double)step * m.dt;
  return o;
}

fdtd_status copy_in_field(fdtd_ctx* h, const void* src, int sdtype, int on_device, int ddtype,
                          void* dst, long long n) {
  if (sdtype < FDTD_F64 || sdtype > FDTD_BF16) return fail(FDTD_EINVAL, "bad source dtype");
  const size_t bytes = elem_size(sdtype) * (size_t)n;
  const void* dsrc = src;
  void* tmp = nullptr;
  if (!on_device) {
    hipError_t e = dev_malloc(h, &tmp, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(FDTD_ENOMEM, "staging allocation failed");
    }
    e = hipMemcpyAsync(tmp, src, bytes, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) {
      (void)hipFree(tmp);
      return hip_fail(e, "hipMemcpyAsync H2D");
    }
    dsrc = tmp;
  }
  hipError_t e = launch_convert(sdtype, dsrc, ddtype, dst, n, 1.0, h->stream);
  if (tmp) {
    hipError_t e2 = hipStreamSynchronize(h->stream);
    (void)hipFree(tmp);
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamSynchronize");
  }
  if (e != hipSuccess) return hip_fail(e, "convert kernel");
  return FDTD_OK;
}

constexpr int kMaxProj = 16;

// Project member m's current state against its kept states (Sec. III), one
// after the other, then reset the pending scale from the new norm.  coef
// (optional, host) receives the nproj coefficients.
fdtd_status project_member(fdtd_ctx* h, int m, double* coef) {
  MemberHost& mh = h->mem[m];
  if (mh.nproj == 0) return FDTD_OK;
  if (!h->d_proj) {
    hipError_t e = dev_malloc(h, (void**)&h->d_proj, sizeof(double) * (project_partials_doubles() + kMaxProj));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(FDTD_ENOMEM, "projection scratch allocation failed");
    }
  }
  double* coef_dev = h->d_proj + project_partials_doubles();
  const size_t cs = h->dtype == kF64 ? 8 : 4;
  for (int k = 0; k < mh.nproj; ++k)
    HIP_TRY(launch_project(h->dtype, h->psi(m, h->cur), static_cast<char*>(mh.proj) + cs * (size_t)mh.n3 * k,
                           mh.n3, h->d_proj, coef_dev + k, h->stream));
  ST_TRY(observe(h, m, true));
  if (coef) {
    HIP_TRY(hipMemcpyAsync(coef, coef_dev, sizeof(double) * mh.nproj, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
  }
  return FDTD_OK;
}

fdtd_status check_member(fdtd_ctx* h, int member, bool allow_all) {
  if (member == -1 && allow_all) return FDTD_OK;
  if (member < 0 || member >= h->count) return fail(FDTD_EINVAL, "member index out of range");
  return FDTD_OK;
}

// after a new initial state: zero step, clear flags, scale = 1/norm
fdtd_status start_state(fdtd_ctx* h, int m) {
  HIP_TRY(launch_set_state(h->d_states(), m, 1.0, 0, 1, h->stream));
  ST_TRY(observe(h, m, true));
  h->mem[m].init_set = true;
  h->mem[m].hist_from = 0;
  return FDTD_OK;
}

std::mutex g_tune_mu;
std::map<std::string, fdtd_tuning> g_tune_cache;

// Cache key of a launch shape: the device's architecture and CU count, the
// dtype and every member's side (no spaces: one token of the cache file).
// Autotuner cache key: device (architecture, CU count), dtype, the members'
// sides and, with ":fv", a step that evaluates V itself (the fastest shapes
// differ: with the V table the 512^3 F32 two-step pass wants 16 x 128 tiles,
// with the in-kernel potential 32 x 64).
std::string tune_key(const fdtd_ctx* h) {
  std::string k = h->arch + "/" + std::to_string(h->n_cu) + "cu:" + std::to_string(h->dtype);
  for (auto& m : h->mem) k += ":" + std::to_string(m.N);
  if (use_fv(h)) k += ":fv";
  return k;
}

fdtd_status validate_tuning(const fdtd_ctx* h, const fdtd_tuning& t) {
  if (t.vz != 1 && t.vz != vec_width(h->dtype)) return fail(FDTD_EINVAL, "tuning: vz must be 1 or the dtype's vector width");
  for (auto& m : h->mem)
    if (m.N % t.vz != 0) return fail(FDTD_EINVAL, "tuning: vz must divide every N");
  if (t.ry != 1 && t.ry != 2 && t.ry != 4) return fail(FDTD_EINVAL, "tuning: ry must be 1, 2 or 4");
  if (t.vz * t.ry > (h->dtype == kF64 ? 4 : 8))
    return fail(FDTD_EINVAL, "tuning: vz * ry must be <= 8 (<= 4 for F64)");
  if (t.xchunk < 0) return fail(FDTD_EINVAL, "tuning: xchunk must be >= 0 (0: automatic)");
  if (t.grid < 0) return fail(FDTD_EINVAL, "tuning: grid must be >= 0");
  if (t.depth < 1 || t.depth > 5) return fail(FDTD_EINVAL, "tuning: depth must be in 1..5");
  if (t.depth >= 4 && (t.tblock != 2 || h->dtype == kF64))
    return fail(FDTD_EINVAL, "tuning: depth 4 or 5 needs tblock = 2 and an F32 or BF16 state");
  if (t.vz == 1 && t.depth != 1) return fail(FDTD_EINVAL, "tuning: depth must be 1 when vz = 1");
  if (t.variant < 0 || t.variant > 3) return fail(FDTD_EINVAL, "tuning: variant must be 0, 1, 2 or 3");
  if (t.variant == 3 && (t.vz != vec_width(h->dtype) || t.ry > 2))
    return fail(FDTD_EINVAL, "tuning: variant 3 needs vz = the dtype's vector width and ry <= 2");
  if (t.persist < 0 || t.persist > 65536) return fail(FDTD_EINVAL, "tuning: persist must be in [0, 65536]");
  if (t.persist > 0 && t.variant != 0) return fail(FDTD_EINVAL, "tuning: persistent launches need variant 0");
  if (t.persist > 0 && t.tblock == 2 && t.persist > 32768)
    return fail(FDTD_EINVAL, "tuning: persistent two-step launches take at most 32768 passes");
  if (t.vfuse != 0 && t.vfuse != 1) return fail(FDTD_EINVAL, "tuning: vfuse must be 0 or 1");
  if (t.tblock != 0 && t.tblock != 2) return fail(FDTD_EINVAL, "tuning: tblock must be 0 or 2");
  if (t.tile != 0 && t.tile != 1) return fail(FDTD_EINVAL, "tuning: tile must be 0 or 1");
  if (t.tile == 1 && (t.tblock != 2 || h->dtype == kF64))
    return fail(FDTD_EINVAL, "tuning: tile 1 (16 x 128 tiles) needs tblock = 2 and an F32 or BF16 state");
  if (t.tblock == 2) {
    if (t.variant != 0) return fail(FDTD_EINVAL, "tuning: tblock = 2 needs variant 0");
    if (t.ry != 1 || t.vz != vec_width(h->dtype)) return fail(FDTD_EINVAL, "tuning: tblock = 2 needs ry = 1 and vz = the dtype's vector width");
    for (auto& m : h->mem)
      if (m.N % kTbVec(h->dtype) != 0) return fail(FDTD_EINVAL, "tuning: tblock = 2 needs every N to be a multiple of its lane vector");
  }
  if (t.variant == 2) {
    if (t.ry != 1) return fail(FDTD_EINVAL, "tuning: variant 2 needs ry = 1");
    if (h->dtype == kBF16 && t.vz > 1) return fail(FDTD_EINVAL, "tuning: variant 2 needs vz = 1 for BF16");
    if (h->dtype == kF64 && t.depth > 1) return fail(FDTD_EINVAL, "tuning: variant 2 needs depth = 1 for F64");
  }
  if (t.variant == 1) {
    const int vw = vec_width(h->dtype);
    if (t.vz != vw) return fail(FDTD_EINVAL, "tuning: the LDS-tile variant needs vz = the dtype's vector width");
    const long long tb = tile_threads(h->dtype), cs = h->dtype == kF64 ? 8 : 4;
    for (auto& m : h->mem) {
      if (2LL * m.N / vw > tb) return fail(FDTD_EINVAL, "tuning: the LDS-tile variant needs 2N / vz <= its work-group size");
      if (2LL * (tb * vw + 2LL * m.N) * cs > 65536) return fail(FDTD_EINVAL, "tuning: the LDS tile would exceed 64 KiB");
    }
  }
  return FDTD_OK;
}

}  // namespace

// =============================================================== C ABI =====
extern "C" {

fdtd_status fdtd_create(const fdtd_config* cfg, fdtd_t* out) { return make_ctx(cfg, 1, out); }

fdtd_status fdtd_create_batch(const fdtd_config* cfgs, int32_t count, fdtd_t* out) {
  return make_ctx(cfgs, count, out);
}

fdtd_status fdtd_workspace_size(fdtd_t h, size_t* bytes) {
  if (!h || !bytes) return fail(FDTD_EINVAL, "workspace_size: null argument");
  *bytes = h->need_bytes;
  return FDTD_OK;
}

fdtd_status fdtd_bind_workspace(fdtd_t h, void* dev_ptr, size_t bytes) {
  if (!h || !dev_ptr) return fail(FDTD_EINVAL, "bind_workspace: null argument");
  if (h->ws) return fail(FDTD_EINVAL, "bind_workspace: the handle already has device memory");
  if (bytes < h->need_bytes) return fail(FDTD_ENOMEM, "bind_workspace: workspace smaller than fdtd_workspace_size");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % 256 != 0) return fail(FDTD_EINVAL, "bind_workspace: pointer must be 256-byte aligned");
  ST_TRY(set_device(h));
  h->ws = static_cast<char*>(dev_ptr);
  h->ws_bytes = bytes;
  h->ws_owned = false;
  for (int m = 0; m < h->count; ++m) HIP_TRY(launch_set_state(h->d_states(), m, 1.0, 0, 1, h->stream));
  HIP_TRY(launch_persist_reset(h->d_ctrl(), h->d_states(), h->count, h->stream));
  return FDTD_OK;
}

fdtd_status fdtd_destroy(fdtd_t h) {
  if (!h) return FDTD_OK;
  if (h->ws || h->h_pin || h->d_items) {
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
  }
  drop_graphs(h);
  if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
  if (h->d_items) (void)hipFree(h->d_items);
  if (h->d_partials) (void)hipFree(h->d_partials);
  if (h->d_proj) (void)hipFree(h->d_proj);
  if (h->gws && h->gws_owned) (void)hipFree(h->gws);
  for (auto& m : h->mem)
    if (m.proj) (void)hipFree(m.proj);
  if (h->ws && h->ws_owned) (void)hipFree(h->ws);
  if (h->h_pin) (void)hipHostFree(h->h_pin);
  delete h;
  return FDTD_OK;
}

fdtd_status fdtd_set_potential(fdtd_t h, int32_t member, const void* v, int32_t dtype,
                               int32_t on_device) {
  if (!h || !v) return fail(FDTD_EINVAL, "set_potential: null argument");
  ST_TRY(check_member(h, member, false));
  if (dtype != FDTD_F64 && dtype != FDTD_F32) return fail(FDTD_EINVAL, "set_potential: dtype must be F64 or F32");
  ST_TRY(ensure_memory(h));
  ST_TRY(copy_in_field(h, v, dtype, on_device, h->vdtype, h->V(member), h->mem[member].n3));
  h->mem[member].pot_set = true;
  h->mem[member].vkind = -1;
  h->mem[member].pkind = -1;
  h->mem[member].params.clear();
  h->items_valid = false;  // re-upload the member table
  drop_graphs(h);
  return FDTD_OK;
}

fdtd_status fdtd_set_potential_analytic(fdtd_t h, int32_t member, int32_t kind, const double* p,
                                        int32_t np) {
  if (!h) return fail(FDTD_EINVAL, "set_potential_analytic: null handle");
  ST_TRY(check_member(h, member, true));
  if (kind < FDTD_POT_CONST || kind > FDTD_POT_DODECA) return fail(FDTD_EINVAL, "set_potential_analytic: unknown kind");
  const int need = (kind == FDTD_POT_HO || kind == FDTD_POT_CORNELL) ? 3 : (kind == FDTD_POT_WELLS ? 3 : 1);
  if (np < need || (np > 0 && !p)) return fail(FDTD_EINVAL, "set_potential_analytic: too few parameters");
  if (kind == FDTD_POT_WELLS && (np - 3) % 5 != 0) return fail(FDTD_EINVAL, "set_potential_analytic: wells need 3 + 5k parameters");
  if (np > kMaxParams) return fail(FDTD_EINVAL, "set_potential_analytic: too many parameters");
  for (int i = 0; i < np; ++i)
    if (!std::isfinite(p[i])) return fail(FDTD_EINVAL, "set_potential_analytic: non-finite parameter");
  ST_TRY(ensure_memory(h));
  HIP_TRY(hipMemcpyAsync(h->d_params(), p, sizeof(double) * np, hipMemcpyHostToDevice, h->stream));
  const int m0 = member < 0 ? 0 : member, m1 = member < 0 ? h->count : member + 1;
  for (int m = m0; m < m1; ++m) {
    const MemberHost& mh = h->mem[m];
    HIP_TRY(launch_potential(h->vdtype, h->V(m), mh.N, mh.ha, mh.a, kind, h->d_params(), np, h->stream));
    h->mem[m].pot_set = true;
    // the table is always filled; kinds 0..4 may also be evaluated in the step
    h->mem[m].vkind = kind <= FDTD_POT_CORNELL ? kind : -1;
    for (int k = 0; k < 3; ++k) h->mem[m].vp[k] = k < np ? p[k] : 0.0;
    h->mem[m].pkind = kind;
    h->mem[m].params.assign(p, p + np);
  }
  HIP_TRY(hipStreamSynchronize(h->stream));  // p is the caller's host memory
  h->items_valid = false;  // re-upload the member table
  drop_graphs(h);
  return FDTD_OK;
}

fdtd_status fdtd_set_initial(fdtd_t h, int32_t member, int32_t kind, uint64_t seed, uint32_t parity,
                             const void* user, int32_t dtype, int32_t on_device) {
  if (!h) return fail(FDTD_EINVAL, "set_initial: null handle");
  ST_TRY(check_member(h, member, true));
  if (kind < FDTD_INIT_UNIFORM || kind > FDTD_INIT_USER) return fail(FDTD_EINVAL, "set_initial: unknown kind");
  if (parity >> 6) return fail(FDTD_EINVAL, "set_initial: parity uses bits 0-5 only");
  for (int ax = 0; ax < 3; ++ax)
    if (((parity >> (2 * ax)) & 3u) == 3u) return fail(FDTD_EINVAL, "set_initial: parity code 3 is invalid");
  if (kind == FDTD_INIT_USER && (!user || member < 0)) return fail(FDTD_EINVAL, "set_initial: USER needs a buffer and one member");
  if (kind == FDTD_INIT_USER && (dtype < FDTD_F64 || dtype > FDTD_BF16)) return fail(FDTD_EINVAL, "set_initial: bad user dtype");
  ST_TRY(ensure_memory(h));
  const int m0 = member < 0 ? 0 : member, m1 = member < 0 ? h->count : member + 1;
  for (int m = m0; m < m1; ++m) {
    const MemberHost& mh = h->mem[m];
    if (kind == FDTD_INIT_USER) {
      ST_TRY(copy_in_field(h, user, dtype, on_device, h->dtype, h->psi(m, h->cur), mh.n3));
    } else {
      HIP_TRY(launch_initial(h->dtype, h->psi(m, h->cur), mh.N, seed, (uint32_t)m, kind, parity, h->stream));
    }
    h->mem[m].parity = parity;
  }
  for (int m = m0; m < m1; ++m) {
    ST_TRY(start_state(h, m));
    HIP_TRY(hipMemcpyAsync(h->h_pin, h->d_obs() + (size_t)m * kRec, sizeof(double) * kRec,
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    const double s0 = h->h_pin[kS0];
    if (!(s0 > 0) || !std::isfinite(s0)) {
      h->mem[m].init_set = false;
      return fail(FDTD_ENONFINITE, "set_initial: the initial state has a zero or non-finite norm");
    }
  }
  return FDTD_OK;
}

fdtd_status fdtd_set_projection_states(fdtd_t h, int32_t member, const void* states, int32_t n,
                                       int32_t dtype, int32_t on_device) {
  if (!h) return fail(FDTD_EINVAL, "set_projection_states: null handle");
  ST_TRY(check_member(h, member, false));
  if (n < 0 || n > kMaxProj) return fail(FDTD_EINVAL, "set_projection_states: n must be in [0, 16]");
  if (n > 0 && !states) return fail(FDTD_EINVAL, "set_projection_states: null states");
  if (n > 0 && (dtype < FDTD_F64 || dtype > FDTD_BF16)) return fail(FDTD_EINVAL, "set_projection_states: bad dtype");
  ST_TRY(ensure_memory(h));
  MemberHost& mh = h->mem[member];
  HIP_TRY(hipStreamSynchronize(h->stream));  // the old states may still be read
  if (mh.proj) (void)hipFree(mh.proj);
  mh.proj = nullptr;
  mh.nproj = 0;
  if (n == 0) return FDTD_OK;
  const int cdt = h->dtype == kF64 ? FDTD_F64 : FDTD_F32;  // kept in the arithmetic type
  const size_t cs = elem_size(cdt);
  hipError_t e = dev_malloc(h, &mh.proj, cs * (size_t)mh.n3 * n);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    mh.proj = nullptr;
    return fail(FDTD_ENOMEM, "set_projection_states: allocation failed");
  }
  const size_t sb = elem_size(dtype) * (size_t)mh.n3;
  for (int k = 0; k < n; ++k) {
    fdtd_status st = copy_in_field(h, static_cast<const char*>(states) + sb * k, dtype, on_device,
                                   cdt, static_cast<char*>(mh.proj) + cs * (size_t)mh.n3 * k, mh.n3);
    if (st != FDTD_OK) {
      (void)hipFree(mh.proj);
      mh.proj = nullptr;
      return st;
    }
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  mh.nproj = n;
  return FDTD_OK;
}

fdtd_status fdtd_project(fdtd_t h, int32_t member, double* coef) {
  if (!h) return fail(FDTD_EINVAL, "project: null handle");
  ST_TRY(check_member(h, member, false));
  ST_TRY(require_ready(h));
  if (h->mem[member].nproj == 0) return fail(FDTD_EINVAL, "project: no projection states set");
  ST_TRY(ensure_memory(h));
  ST_TRY(build_items(h));
  return project_member(h, member, coef);
}

fdtd_status fdtd_evolve(fdtd_t h, const fdtd_evolve_opts* o, int64_t* steps_done, int32_t* converged) {
  if (!h || !o) return fail(FDTD_EINVAL, "evolve: null argument");
  if (o->max_steps < 0 || o->renorm_every < 0 || o->check_every < 0 ||
      o->reimpose_parity_every < 0 || o->project_every < 0)
    return fail(FDTD_EINVAL, "evolve: negative option");
  if (o->check_every > 0 && !(o->rel_tol >= 0)) return fail(FDTD_EINVAL, "evolve: rel_tol must be >= 0");
  if (o->flags & ~FDTD_EVOLVE_ASYNC) return fail(FDTD_EINVAL, "evolve: unknown flag");
  const bool async = (o->flags & FDTD_EVOLVE_ASYNC) != 0;
  if (async && o->check_every > 0)
    return fail(FDTD_EINVAL, "evolve: FDTD_EVOLVE_ASYNC cannot be combined with a convergence check");
  if (steps_done) *steps_done = 0;
  if (converged) *converged = 0;
  ST_TRY(require_ready(h));
  ST_TRY(ensure_memory(h));
  ST_TRY(build_items(h));
  std::vector<MemberState> st;
  long long step0 = 0;
  if (!async) {
    ST_TRY(read_states(h, st));
    ST_TRY(check_bad(h, st));
    step0 = st[0].step;
  }
  const int K = o->check_every > 0 ? o->check_every : 64;
  const int P = o->reimpose_parity_every;
  const int PE = o->project_every;
  std::vector<double> e_prev(h->count, NAN);
  long long done = 0;
  bool conv = false;
  while (done < o->max_steps) {
    // chunks end at every check, parity and projection boundary
    long long n = std::min<long long>(K - (done % K), o->max_steps - done);
    if (P > 0) n = std::min<long long>(n, P - (done % P));
    if (PE > 0) n = std::min<long long>(n, PE - (done % PE));
    if (o->use_graph && n >= 8) ST_TRY(graph_steps(h, (int)n, o->renorm_every));
    else ST_TRY(launch_steps(h, (int)n, o->renorm_every, h->stream));
    done += n;
    if (P > 0 && done % P == 0)
      for (int m = 0; m < h->count; ++m)
        if (h->mem[m].parity) HIP_TRY(launch_reimpose(h->dtype, h->psi(m, h->cur), h->mem[m].N, h->mem[m].parity, h->stream));
    if (PE > 0 && done % PE == 0)
      for (int m = 0; m < h->count; ++m) ST_TRY(project_member(h, m, nullptr));
    const bool check = o->check_every > 0 && done % K == 0;
    if (check) {
      const long long t = step0 + done - 1;  // the step whose input is checked
      double* pin = h->h_pin;
      for (int m = 0; m < h->count; ++m)
        HIP_TRY(hipMemcpyAsync(pin + (size_t)m * kRec,
                               h->d_ring() + ((size_t)m * h->ring_cap + (size_t)(t % h->ring_cap)) * kRec,
                               sizeof(double) * kRec, hipMemcpyDeviceToHost, h->stream));
      ST_TRY(read_states(h, st));
      ST_TRY(check_bad(h, st));
      bool all = true;
      for (int m = 0; m < h->count; ++m) {
        const double* r = pin + (size_t)m * kRec;
        const double e = (r[kKin] + r[kPot]) / r[kS0];
        const bool c = !std::isnan(e_prev[m]) &&
                       std::fabs(e - e_prev[m]) <= o->rel_tol * std::fabs(e - h->mem[m].v_inf);
        all = all && c;
        e_prev[m] = e;
      }
      if (all) {
        conv = true;
        break;
      }
    }
  }
  if (steps_done) *steps_done = done;
  if (async) return FDTD_OK;  // a non-finite step shows up at the next synchronous call
  ST_TRY(read_states(h, st));
  if (converged) *converged = conv ? 1 : 0;
  ST_TRY(check_bad(h, st));
  return FDTD_OK;
}

fdtd_status fdtd_observables(fdtd_t h, fdtd_obs* out) {
  if (!h || !out) return fail(FDTD_EINVAL, "observables: null argument");
  ST_TRY(require_ready(h));
  ST_TRY(ensure_memory(h));
  ST_TRY(observe(h, -1, false));
  double* pin = h->h_pin;
  HIP_TRY(hipMemcpyAsync(pin, h->d_obs(), sizeof(double) * kRec * h->count, hipMemcpyDeviceToHost, h->stream));
  std::vector<MemberState> st;
  ST_TRY(read_states(h, st));
  for (int m = 0; m < h->count; ++m) out[m] = to_obs(h->mem[m], pin + (size_t)m * kRec, st[m].step);
  return FDTD_OK;
}

fdtd_status fdtd_history(fdtd_t h, int32_t member, fdtd_obs* out, int64_t max, int64_t* count) {
  if (!h || !out || !count || max < 0) return fail(FDTD_EINVAL, "history: bad argument");
  ST_TRY(check_member(h, member, false));
  *count = 0;
  if (!h->ws) return FDTD_OK;
  std::vector<MemberState> st;
  ST_TRY(read_states(h, st));
  const long long steps = st[member].step;
  const long long n = std::min<long long>({(long long)max, steps - h->mem[member].hist_from,
                                           (long long)h->ring_cap});
  std::vector<double> buf((size_t)h->ring_cap * kRec);
  HIP_TRY(hipMemcpyAsync(buf.data(), h->d_ring() + (size_t)member * h->ring_cap * kRec,
                         sizeof(double) * kRec * h->ring_cap, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (long long k = 0; k < n; ++k) {
    const long long t = steps - n + k;
    const double* r = buf.data() + (size_t)(t % h->ring_cap) * kRec;
    out[k] = to_obs(h->mem[member], r, t);
  }
  *count = n;
  return FDTD_OK;
}

fdtd_status fdtd_get_psi(fdtd_t h, int32_t member, void* dst, int32_t dtype, int32_t on_device) {
  if (!h || !dst) return fail(FDTD_EINVAL, "get_psi: null argument");
  ST_TRY(check_member(h, member, false));
  if (dtype < FDTD_F64 || dtype > FDTD_BF16) return fail(FDTD_EINVAL, "get_psi: bad dtype");
  if (!h->mem[member].init_set) return fail(FDTD_ENOTREADY, "get_psi: no state set");
  ST_TRY(ensure_memory(h));
  ST_TRY(build_items(h));
  // norm of the stored state from a reduction pass
  {
    StepArgs a = base_args(h);
    a.items = h->d_items;
    a.item_offset = h->mem[member].item_begin;
    a.n_items = h->mem[member].item_end - h->mem[member].item_begin;
    // the reduction needs V only for the energy sums; it is harmless if unset
    HIP_TRY(launch_kernel(h, false, launch_grid(h, a.n_items), a, h->stream));
  }
  HIP_TRY(hipMemcpyAsync(h->h_pin, h->d_obs() + (size_t)member * kRec, sizeof(double) * kRec,
                         hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  const MemberHost& m = h->mem[member];
  const double s0 = h->h_pin[kS0];
  if (!(s0 > 0) || !std::isfinite(s0)) return fail(FDTD_ENONFINITE, "get_psi: state has zero or non-finite norm");
  const double scale = 1.0 / std::sqrt(m.a3 * s0);
  const size_t bytes = elem_size(dtype) * (size_t)m.n3;
  if (on_device) {
    HIP_TRY(launch_convert(h->dtype, h->psi(member, h->cur), dtype, dst, m.n3, scale, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
  } else {
    void* tmp = nullptr;
    hipError_t e = dev_malloc(h, &tmp, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(FDTD_ENOMEM, "get_psi: staging allocation failed");
    }
    e = launch_convert(h->dtype, h->psi(member, h->cur), dtype, tmp, m.n3, scale, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dst, tmp, bytes, hipMemcpyDeviceToHost, h->stream);
    hipError_t e2 = hipStreamSynchronize(h->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "get_psi copy");
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamSynchronize");
  }
  return FDTD_OK;
}

fdtd_status fdtd_get_state(fdtd_t h, int32_t member, void* dst, int32_t on_device, int64_t* step) {
  if (!h || !dst) return fail(FDTD_EINVAL, "get_state: null argument");
  ST_TRY(check_member(h, member, false));
  if (!h->mem[member].init_set) return fail(FDTD_ENOTREADY, "get_state: no state set");
  ST_TRY(ensure_memory(h));
  const size_t bytes = elem_size(h->dtype) * (size_t)h->mem[member].n3;
  HIP_TRY(hipMemcpyAsync(dst, h->psi(member, h->cur), bytes,
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
  std::vector<MemberState> st;
  ST_TRY(read_states(h, st));
  if (step) *step = st[member].step;
  return FDTD_OK;
}

// The fine member's state <- trilinear interpolation of the coarse member's
// (Sec. VI), renormalised by the kernel itself: `partials` holds
// upsample_groups(N_fine) doubles.  The step counter restarts at 0.
static fdtd_status upsample_into(fdtd_ctx* coarse, int cm, fdtd_ctx* fine, int fm, double* partials) {
  const MemberHost& c = coarse->mem[cm];
  MemberHost& f = fine->mem[fm];
  HIP_TRY(hipSetDevice(fine->device));
  // order the fine stream after the coarse work
  if (coarse->stream != fine->stream) HIP_TRY(hipStreamSynchronize(coarse->stream));
  HIP_TRY(launch_set_state(fine->d_states(), fm, 1.0, 0, 1, fine->stream));  // counter 0, step 0
  UpNorm u;
  u.partials = partials;
  u.st = fine->d_states() + fm;
  u.obs = fine->d_obs() + (size_t)fm * kRec;
  u.a3 = f.a3;
  HIP_TRY(launch_upsample(coarse->dtype, coarse->psi(cm, coarse->cur), c.N, c.ha, c.a, fine->dtype,
                          fine->psi(fm, fine->cur), f.N, f.ha, u, fine->stream));
  HIP_TRY(hipMemcpyAsync(fine->h_pin, u.obs + kS0, sizeof(double), hipMemcpyDeviceToHost, fine->stream));
  HIP_TRY(hipStreamSynchronize(fine->stream));
  const double s0 = fine->h_pin[0];
  f.parity = c.parity;
  f.hist_from = 0;
  if (!(s0 > 0) || !std::isfinite(s0)) {
    f.init_set = false;
    return fail(FDTD_ENONFINITE, "upsample: the interpolated state has a zero or non-finite norm");
  }
  f.init_set = true;
  return FDTD_OK;
}

// Checkpoint record: this header, then the stored state as held.
struct CkptHeader {
  uint64_t magic;     // kCkptMagic
  int32_t version;    // 1
  int32_t dtype;      // storage dtype of the state
  int64_t n;          // lattice side
  int64_t step;       // steps taken
  double scale;       // pending scale of the next update
  uint32_t parity;    // parity word of the member
  uint32_t pad;
  double L, dt;       // box and time step (checked on load)
  uint64_t reserved[2];
};
static_assert(sizeof(CkptHeader) == 80, "checkpoint header layout");
constexpr uint64_t kCkptMagic = 0x314b435044544446ull;  // "FDTDPCK1"

fdtd_status fdtd_checkpoint_size(fdtd_t h, int32_t member, size_t* bytes) {
  if (!h || !bytes) return fail(FDTD_EINVAL, "checkpoint_size: null argument");
  ST_TRY(check_member(h, member, false));
  *bytes = sizeof(CkptHeader) + elem_size(h->dtype) * (size_t)h->mem[member].n3;
  return FDTD_OK;
}

fdtd_status fdtd_checkpoint_save(fdtd_t h, int32_t member, void* dst, int32_t on_device) {
  if (!h || !dst) return fail(FDTD_EINVAL, "checkpoint_save: null argument");
  ST_TRY(check_member(h, member, false));
  if (!h->mem[member].init_set) return fail(FDTD_ENOTREADY, "checkpoint_save: no state set");
  ST_TRY(ensure_memory(h));
  const MemberHost& m = h->mem[member];
  std::vector<MemberState> st;
  ST_TRY(read_states(h, st));
  ST_TRY(check_bad(h, st));
  CkptHeader hd;
  memset(&hd, 0, sizeof hd);
  hd.magic = kCkptMagic;
  hd.version = 1;
  hd.dtype = h->dtype;
  hd.n = m.N;
  hd.step = st[member].step;
  hd.scale = st[member].scale;
  hd.parity = m.parity;
  hd.L = m.L;
  hd.dt = m.dt;
  char* d = static_cast<char*>(dst);
  const size_t bytes = elem_size(h->dtype) * (size_t)m.n3;
  if (on_device) {
    HIP_TRY(hipMemcpyAsync(d, &hd, sizeof hd, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(d + sizeof hd, h->psi(member, h->cur), bytes, hipMemcpyDeviceToDevice, h->stream));
  } else {
    memcpy(d, &hd, sizeof hd);
    HIP_TRY(hipMemcpyAsync(d + sizeof hd, h->psi(member, h->cur), bytes, hipMemcpyDeviceToHost, h->stream));
  }
  HIP_TRY(hipStreamSynchronize(h->stream));  // hd is a temporary
  return FDTD_OK;
}

fdtd_status fdtd_checkpoint_load(fdtd_t h, int32_t member, const void* src, int32_t on_device) {
  if (!h || !src) return fail(FDTD_EINVAL, "checkpoint_load: null argument");
  ST_TRY(check_member(h, member, false));
  CkptHeader hd;
  if (on_device) {
    ST_TRY(ensure_memory(h));
    HIP_TRY(hipMemcpy(&hd, src, sizeof hd, hipMemcpyDeviceToHost));
  } else {
    memcpy(&hd, src, sizeof hd);
  }
  const MemberHost& m = h->mem[member];
  if (hd.magic != kCkptMagic || hd.version != 1) return fail(FDTD_EINVAL, "checkpoint_load: not a checkpoint record");
  if (hd.dtype != h->dtype || hd.n != m.N)
    return fail(FDTD_EINVAL, "checkpoint_load: the record's lattice side or dtype differs from the member's");
  if (hd.L != m.L || hd.dt != m.dt)
    return fail(FDTD_EINVAL, "checkpoint_load: the record's box length or time step differs from the member's");
  if (hd.step < 0 || !(hd.scale > 0) || !std::isfinite(hd.scale) || (hd.parity >> 6))
    return fail(FDTD_EINVAL, "checkpoint_load: corrupt header");
  ST_TRY(ensure_memory(h));
  const size_t bytes = elem_size(h->dtype) * (size_t)m.n3;
  const char* s = static_cast<const char*>(src) + sizeof hd;
  HIP_TRY(hipMemcpyAsync(h->psi(member, h->cur), s, bytes,
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->stream));
  HIP_TRY(launch_set_state(h->d_states(), member, hd.scale, hd.step, 1, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));  // src may be the caller's pageable memory
  h->mem[member].parity = hd.parity;
  h->mem[member].init_set = true;
  h->mem[member].hist_from = hd.step;
  return FDTD_OK;
}

fdtd_status fdtd_upsample(fdtd_t coarse, int32_t cm, fdtd_t fine, int32_t fm) {
  if (!coarse || !fine) return fail(FDTD_EINVAL, "upsample: null handle");
  ST_TRY(check_member(coarse, cm, false));
  ST_TRY(check_member(fine, fm, false));
  if (coarse->device != fine->device) return fail(FDTD_EINVAL, "upsample: handles on different devices");
  const MemberHost& c = coarse->mem[cm];
  MemberHost& f = fine->mem[fm];
  if (std::fabs(c.L - f.L) > 1e-12 * std::max(c.L, f.L)) return fail(FDTD_EINVAL, "upsample: box lengths differ");
  if (!c.init_set) return fail(FDTD_ENOTREADY, "upsample: coarse state not set");
  if (!f.pot_set) return fail(FDTD_ENOTREADY, "upsample: fine potential not set");
  ST_TRY(ensure_memory(coarse));
  ST_TRY(ensure_memory(fine));
  return upsample_into(coarse, cm, fine, fm, fine->d_upart());
}

// ---- the upsample for callers that cannot allocate ----------------------
// Partial sums of the upsample kernel's norm in a fixed device array instead
// of the fine handle's workspace.  Each GPU holds its own copy of the array;
// host code reaches it only through the address hipGetSymbolAddress gives on
// that device (the array's name is a host-side stand-in), taken once per
// device on the first call there.
constexpr size_t kNoAllocScratchDoubles = 131072;  // 1 MiB: fine sides up to 1620
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];
constexpr int kMaxDevices = 64;

static fdtd_status scratch_on_device(int device, double** out) {
  static std::mutex mu;
  static double* ptr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return fail(FDTD_EINVAL, "upsample_noalloc: device ordinal out of range");
  std::lock_guard<std::mutex> lk(mu);
  if (!ptr[device]) {
    HIP_TRY(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    ptr[device] = static_cast<double*>(p);
  }
  *out = ptr[device];
  return FDTD_OK;
}

fdtd_status fdtd_upsample_noalloc(fdtd_t coarse, int32_t cm, fdtd_t fine, int32_t fm) {
  if (!coarse || !fine) return fail(FDTD_EINVAL, "upsample_noalloc: null handle");
  ST_TRY(check_member(coarse, cm, false));
  ST_TRY(check_member(fine, fm, false));
  const MemberHost& c = coarse->mem[cm];
  const MemberHost& f = fine->mem[fm];
  if ((size_t)upsample_groups(f.N) > kNoAllocScratchDoubles)
    return fail(FDTD_EINVAL, "upsample_noalloc: the fine side " + std::to_string(f.N) +
                                 " needs more partial sums than the static scratch holds (fine sides up to 1620)");
  if (coarse->device != fine->device) return fail(FDTD_EINVAL, "upsample_noalloc: handles on different devices");
  if (std::fabs(c.L - f.L) > 1e-12 * std::max(c.L, f.L)) return fail(FDTD_EINVAL, "upsample_noalloc: box lengths differ");
  if (!c.init_set) return fail(FDTD_ENOTREADY, "upsample_noalloc: coarse state not set");
  if (!f.pot_set) return fail(FDTD_ENOTREADY, "upsample_noalloc: fine potential not set");
  if (!coarse->ws || !fine->ws || !fine->h_pin)
    return fail(FDTD_ENOTREADY, "upsample_noalloc: the handles' device memory is not set up");
  double* p = nullptr;
  ST_TRY(scratch_on_device(fine->device, &p));
  return upsample_into(coarse, cm, fine, fm, p);
}

fdtd_status fdtd_get_tuning(fdtd_t h, fdtd_tuning* out) {
  if (!h || !out) return fail(FDTD_EINVAL, "get_tuning: null argument");
  *out = h->tun;
  return FDTD_OK;
}

fdtd_status fdtd_set_tuning(fdtd_t h, const fdtd_tuning* t) {
  if (!h || !t) return fail(FDTD_EINVAL, "set_tuning: null argument");
  ST_TRY(validate_tuning(h, *t));
  if (!same_tuning(*t, h->tun)) {
    h->tun = *t;
    h->items_valid = false;
  }
  return FDTD_OK;
}

fdtd_status fdtd_synchronize(fdtd_t h) {
  if (!h) return fail(FDTD_EINVAL, "synchronize: null handle");
  if (!h->ws) return FDTD_OK;
  HIP_TRY(hipSetDevice(h->device));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return FDTD_OK;
}

fdtd_status fdtd_get_counters(fdtd_t h, fdtd_counters* out) {
  if (!h || !out) return fail(FDTD_EINVAL, "get_counters: null argument");
  out->graph_captures = h->n_captures;
  out->graph_replays = h->n_replays;
  out->allocations = h->n_allocs;
  out->reserved = 0;
  return FDTD_OK;
}

fdtd_status fdtd_info(fdtd_t h, int32_t* count, void** stream) {
  if (!h) return fail(FDTD_EINVAL, "info: null handle");
  if (count) *count = h->count;
  if (stream) *stream = h->stream;
  return FDTD_OK;
}

const char* fdtd_status_string(fdtd_status s) {
  switch (s) {
    case FDTD_OK: return "FDTD_OK";
    case FDTD_EINVAL: return "FDTD_EINVAL: invalid argument";
    case FDTD_ENOMEM: return "FDTD_ENOMEM: out of memory";
    case FDTD_EHIP: return "FDTD_EHIP: HIP runtime error";
    case FDTD_EUNSTABLE: return "FDTD_EUNSTABLE: dt >= m a^2 / 3";
    case FDTD_ENOTREADY: return "FDTD_ENOTREADY: potential or initial state not set";
    case FDTD_ENONFINITE: return "FDTD_ENONFINITE: non-finite reduction";
  }
  return "unknown fdtd_status";
}

const char* fdtd_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------- autotune --
extern "C" fdtd_status fdtd_autotune(fdtd_t h, int32_t steps_per_trial, fdtd_tuning* chosen,
                                     double* best_ms) {
  if (!h) return fail(FDTD_EINVAL, "autotune: null handle");
  if (steps_per_trial < 2) return fail(FDTD_EINVAL, "autotune: steps_per_trial must be >= 2");
  ST_TRY(require_ready(h));
  ST_TRY(ensure_memory(h));
  const std::string key = tune_key(h);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      if (fdtd_set_tuning(h, &it->second) == FDTD_OK) {
        if (chosen) *chosen = it->second;
        if (best_ms) *best_ms = -1.0;
        return FDTD_OK;
      }
      g_tune_cache.erase(it);  // a loaded entry this handle rejects: tune anew
    }
  }
  // save what the trial steps overwrite: the current field of every member,
  // the member states and the history ring
  size_t field_bytes = 0;
  for (auto& m : h->mem) field_bytes += elem_size(h->dtype) * (size_t)m.n3;
  const size_t ring_bytes = sizeof(double) * kRec * (size_t)h->ring_cap * h->count;
  char* save = nullptr;
  hipError_t e = dev_malloc(h, (void**)&save, field_bytes + sizeof(MemberState) * h->count + ring_bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(FDTD_ENOMEM, "autotune: no memory to save the state");
  }
  const int cur0 = h->cur;
  size_t off = 0;
  for (int m = 0; m < h->count; ++m) {
    const size_t b = elem_size(h->dtype) * (size_t)h->mem[m].n3;
    (void)hipMemcpyAsync(save + off, h->psi(m, cur0), b, hipMemcpyDeviceToDevice, h->stream);
    off += b;
  }
  (void)hipMemcpyAsync(save + off, h->d_states(), sizeof(MemberState) * h->count, hipMemcpyDeviceToDevice, h->stream);
  (void)hipMemcpyAsync(save + off + sizeof(MemberState) * h->count, h->d_ring(), ring_bytes,
                       hipMemcpyDeviceToDevice, h->stream);

  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const fdtd_tuning orig = h->tun;
  fdtd_tuning best = orig;
  double best_t = 1e30;
  fdtd_status st = FDTD_OK;
  const int vw = vec_width(h->dtype);
  int maxN = 0;
  for (auto& m : h->mem) maxN = std::max(maxN, m.N);
  std::vector<int> vzs = {1};
  bool all_div = true;
  for (auto& m : h->mem) all_div = all_div && (m.N % vw == 0);
  if (all_div) vzs.push_back(vw);
  {
    // time one candidate; false stops the search (st holds the error)
    auto trial = [&](fdtd_tuning t) -> bool {
      t.vfuse = orig.vfuse;
      if (validate_tuning(h, t) != FDTD_OK) return true;
      h->tun = t;
      h->items_valid = false;
      if ((st = build_items(h)) != FDTD_OK) return false;
      if ((st = launch_steps(h, 1, 1, h->stream)) != FDTD_OK) return false;  // warm-up
      (void)hipEventRecord(e0, h->stream);
      if ((st = launch_steps(h, steps_per_trial, 1, h->stream)) != FDTD_OK) return false;
      (void)hipEventRecord(e1, h->stream);
      if ((e = hipEventSynchronize(e1)) != hipSuccess) {
        st = hip_fail(e, "autotune timing");
        return false;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double per = ms / steps_per_trial;
      if (per < best_t) {
        best_t = per;
        best = t;
      }
      return true;
    };
    bool go = true;
    std::vector<int> persists = {0};
    if (h->count > 1) persists.push_back(64);
    for (int vz : vzs)
      for (int ry : {1, 2, 4})
        for (int xc : {0, 32, 64, 128, 256})
          for (int depth : {1, 2, 3})
            for (int variant : {0, 2, 3})
              for (int persist : persists) {
                if (!go || xc > maxN || (vz == 1 && depth > 1) || (persist && variant)) continue;
                go = trial(fdtd_tuning{vz, ry, xc, 0, 1, depth, variant, persist});
              }
    // LDS-tile variant
    for (int xc : {0, 64, 128, 256})
      for (int depth : {1, 2, 3}) {
        if (!go || xc > maxN || !all_div) continue;
        go = trial(fdtd_tuning{vw, 1, xc, 0, 1, depth, 1});
      }
    // two steps per pass (validation drops the shapes it does not cover),
    // one launch per pass or (batches) persistent passes, on both tile shapes
    // of F32 / BF16 states; the x-chunks between 64 and 128 matter on batches
    // (64 lattices of side 48..160, depth 4: x-chunk 64 151.1 us per step, 80
    // 140.7, 96 147.4)
    for (int tile : {0, 1})
      for (int xc : {0, 32, 64, 80, 96, 128, 256})
        for (int depth : {1, 2, 3, 4, 5})
          for (int persist : persists) {
            if (!go || xc > maxN || !all_div || (h->dtype == kF64 && (depth >= 4 || tile))) continue;
            go = trial(fdtd_tuning{vw, 1, xc, 0, 1, depth, 0, persist / 2, 0, 2, tile});
          }
  }
  // restore
  h->cur = cur0;
  off = 0;
  for (int m = 0; m < h->count; ++m) {
    const size_t b = elem_size(h->dtype) * (size_t)h->mem[m].n3;
    (void)hipMemcpyAsync(h->psi(m, cur0), save + off, b, hipMemcpyDeviceToDevice, h->stream);
    off += b;
  }
  (void)hipMemcpyAsync(h->d_states(), save + off, sizeof(MemberState) * h->count, hipMemcpyDeviceToDevice, h->stream);
  (void)hipMemcpyAsync(h->d_ring(), save + off + sizeof(MemberState) * h->count, ring_bytes,
                       hipMemcpyDeviceToDevice, h->stream);
  (void)hipStreamSynchronize(h->stream);
  (void)hipFree(save);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->tun = (st == FDTD_OK) ? best : orig;
  h->items_valid = false;
  drop_graphs(h);
  if (st != FDTD_OK) return st;
  ST_TRY(build_items(h));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
  }
  if (chosen) *chosen = best;
  if (best_ms) *best_ms = best_t;
  return FDTD_OK;
}

// ------------------------------------------------------ launch-shape cache --
namespace {
constexpr const char* kTuneHeader =
    "# fdtd launch shapes: key vz ry xchunk grid xcd_remap depth variant persist vfuse tblock tile";
}

extern "C" fdtd_status fdtd_tune_cache_save(const char* path) {
  if (!path) return fail(FDTD_EINVAL, "tune_cache_save: null path");
  std::map<std::string, fdtd_tuning> copy;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    copy = g_tune_cache;
  }
  std::ofstream f(path, std::ios::trunc);
  if (!f) return fail(FDTD_EINVAL, std::string("tune_cache_save: cannot open ") + path);
  f << kTuneHeader << "\n";
  for (const auto& kv : copy) {
    const fdtd_tuning& t = kv.second;
    f << kv.first << ' ' << t.vz << ' ' << t.ry << ' ' << t.xchunk << ' ' << t.grid << ' '
      << t.xcd_remap << ' ' << t.depth << ' ' << t.variant << ' ' << t.persist << ' ' << t.vfuse
      << ' ' << t.tblock << ' ' << t.tile << "\n";
  }
  f.flush();
  if (!f) return fail(FDTD_EINVAL, std::string("tune_cache_save: write failed on ") + path);
  return FDTD_OK;
}

extern "C" fdtd_status fdtd_tune_cache_load(const char* path) {
  if (!path) return fail(FDTD_EINVAL, "tune_cache_load: null path");
  std::ifstream f(path);
  if (!f) return fail(FDTD_EINVAL, std::string("tune_cache_load: cannot open ") + path);
  std::map<std::string, fdtd_tuning> got;
  std::string line;
  int no = 0;
  while (std::getline(f, line)) {
    ++no;
    const size_t b = line.find_first_not_of(" \t\r");
    if (b == std::string::npos || line[b] == '#') continue;
    std::istringstream in(line);
    std::string key, extra;
    fdtd_tuning t{};
    if (!(in >> key >> t.vz >> t.ry >> t.xchunk >> t.grid >> t.xcd_remap >> t.depth >> t.variant >>
          t.persist >> t.vfuse >> t.tblock >> t.tile) ||
        (in >> extra))
      return fail(FDTD_EINVAL, "tune_cache_load: " + std::string(path) + " line " +
                                   std::to_string(no) + ": expected a key and 11 integers");
    got[key] = t;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache.swap(got);
  return FDTD_OK;
}

// ---------------------------------------------------------------- gradient --
namespace {
// Layout of the gradient driver's device memory for T steps with checkpoints
// every k: the checkpoints, one segment of recomputed states, two adjoint
// fields, the FP64 dE/dV sum and (F32 states) its FP32 segment accumulator,
// the recompute's member descriptors and states, and a small scratch area.
struct GradLayout {
  size_t ck, sg, lam0, lam1, G, G32, descs, cks, scratch, bytes;
};

GradLayout grad_layout(const fdtd_ctx* h, int T, int k) {
  const MemberHost& m = h->mem[0];
  const size_t fb = align256(elem_size(h->dtype) * (size_t)m.n3);
  const int nck = (T + k - 1) / k;
  const int seg = std::min(k, T);
  GradLayout L;
  size_t off = 0;
  L.ck = off; off += fb * (size_t)nck;
  L.sg = off; off += fb * (size_t)(seg + 1);
  L.lam0 = off; off += fb;
  L.lam1 = off; off += fb;
  L.G = off; off += align256(sizeof(double) * (size_t)m.n3);
  L.G32 = off; off += h->dtype == kF32 ? align256(sizeof(float) * (size_t)m.n3) : 0;
  L.descs = off; off += align256(sizeof(MemberDev) * seg);
  L.cks = off; off += align256(sizeof(MemberState) * (size_t)(nck + 1));
  L.scratch = off; off += 65536 * sizeof(double);
  L.bytes = off;
  return L;
}
}  // namespace

extern "C" fdtd_status fdtd_grad_workspace_size(fdtd_t h, int32_t steps, int32_t checkpoint_every,
                                                size_t* bytes) {
  if (!h || !bytes) return fail(FDTD_EINVAL, "grad_workspace_size: null argument");
  if (steps < 1 || checkpoint_every < 1) return fail(FDTD_EINVAL, "grad_workspace_size: steps and checkpoint_every must be >= 1");
  if (h->count != 1) return fail(FDTD_EINVAL, "grad_workspace_size: single-lattice handles only");
  *bytes = grad_layout(h, steps, checkpoint_every).bytes;
  return FDTD_OK;
}

extern "C" fdtd_status fdtd_bind_grad_workspace(fdtd_t h, void* dev_ptr, size_t bytes) {
  if (!h) return fail(FDTD_EINVAL, "bind_grad_workspace: null handle");
  if (dev_ptr && reinterpret_cast<uintptr_t>(dev_ptr) % 256 != 0)
    return fail(FDTD_EINVAL, "bind_grad_workspace: pointer must be 256-byte aligned");
  if (h->gws && h->gws_owned) {
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(h->gws);
  }
  h->gws = static_cast<char*>(dev_ptr);
  h->gws_bytes = dev_ptr ? bytes : 0;
  h->gws_owned = false;
  return FDTD_OK;
}

extern "C" fdtd_status fdtd_energy_grad(fdtd_t h, int32_t steps, int32_t checkpoint_every,
                                        const double* theta, int32_t ntheta, const int32_t* wrt,
                                        int32_t nwrt, void* dE_dV, double* dE_dtheta,
                                        double* energy) {
  if (!h) return fail(FDTD_EINVAL, "energy_grad: null handle");
  if (h->count != 1) return fail(FDTD_EINVAL, "energy_grad: single-lattice handles only");
  if (h->dtype == kBF16) return fail(FDTD_EINVAL, "energy_grad: psi dtype must be F64 or F32");
  if (steps < 1 || checkpoint_every < 1) return fail(FDTD_EINVAL, "energy_grad: steps and checkpoint_every must be >= 1");
  if (nwrt > 0) {
    if (!theta || !wrt || !dE_dtheta || nwrt > 64) return fail(FDTD_EINVAL, "energy_grad: theta, wrt and dE_dtheta needed (nwrt <= 64)");
    const MemberHost& m0 = h->mem[0];
    if (m0.pkind < 0) return fail(FDTD_EINVAL, "energy_grad: dE_dtheta needs a potential set by fdtd_set_potential_analytic");
    if (ntheta != (int)m0.params.size() || !std::equal(theta, theta + ntheta, m0.params.begin()))
      return fail(FDTD_EINVAL, "energy_grad: theta must be the parameters the potential was set from");
    // parameters each kind has (the rest of theta, if any, does not enter V)
    const int nparam = (m0.pkind == FDTD_POT_HO || m0.pkind == FDTD_POT_CORNELL) ? 3
                       : m0.pkind == FDTD_POT_WELLS ? ntheta : 1;
    for (int k = 0; k < nwrt; ++k)
      if (wrt[k] < 0 || wrt[k] >= nparam)
        return fail(FDTD_EINVAL, "energy_grad: a wrt entry is not a parameter of the potential's kind");
  }
  ST_TRY(require_ready(h));
  ST_TRY(ensure_memory(h));
  ST_TRY(build_items(h));
  // the adjoint reads the V table: the forward and its recompute read it too,
  // so all three see the same potential to the last bit
  struct TableV {
    fdtd_ctx* h;
    ~TableV() { h->table_v_only = false; }
  } table_v{h};
  h->table_v_only = true;
  const MemberHost& m = h->mem[0];
  const size_t es = elem_size(h->dtype);
  const size_t fb = align256(es * (size_t)m.n3);
  const int T = steps, k = checkpoint_every;
  const int nck = (T + k - 1) / k;
  const int seg = std::min(k, T);
  const GradLayout GL = grad_layout(h, T, k);
  if (h->gws && h->gws_bytes < GL.bytes) {
    if (!h->gws_owned)
      return fail(FDTD_ENOMEM, "energy_grad: the bound gradient workspace is smaller than fdtd_grad_workspace_size");
    HIP_TRY(hipStreamSynchronize(h->stream));
    (void)hipFree(h->gws);
    h->gws = nullptr;
    h->gws_bytes = 0;
  }
  if (!h->gws) {
    hipError_t e = dev_malloc(h, (void**)&h->gws, GL.bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      h->gws = nullptr;
      return fail(FDTD_ENOMEM, "energy_grad: cannot allocate checkpoint memory");
    }
    h->gws_bytes = GL.bytes;
    h->gws_owned = true;
  }
  char* buf = h->gws;
  char* ck = buf + GL.ck;
  char* sg = buf + GL.sg;
  char* lam[2] = {buf + GL.lam0, buf + GL.lam1};
  double* G = reinterpret_cast<double*>(buf + GL.G);
  float* G32 = h->dtype == kF32 ? reinterpret_cast<float*>(buf + GL.G32) : nullptr;
  MemberDev* descs = reinterpret_cast<MemberDev*>(buf + GL.descs);
  MemberState* cks = reinterpret_cast<MemberState*>(buf + GL.cks);
  double* scratch = reinterpret_cast<double*>(buf + GL.scratch);

  std::vector<double> scales((size_t)T, 1.0);
  std::vector<double> rec((size_t)seg * kRec);
  // ---- forward, checkpointing every k steps
  std::vector<MemberState> st;
  ST_TRY(read_states(h, st));
  ST_TRY(check_bad(h, st));
  for (int j = 0; j < nck; ++j) {
    const int len = std::min(k, T - j * k);
    HIP_TRY(hipMemcpyAsync(ck + fb * j, h->psi(0, h->cur), es * (size_t)m.n3, hipMemcpyDeviceToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(cks + j, h->d_states(), sizeof(MemberState), hipMemcpyDeviceToDevice, h->stream));
    ST_TRY(read_states(h, st));
    const long long t0 = st[0].step;
    // scales folded into each step, from the history ring: read back after
    // at most ring_cap steps, before the ring wraps over them
    for (int i0 = 0; i0 < len; i0 += h->ring_cap) {
      const int n = std::min(len - i0, h->ring_cap);
      ST_TRY(launch_steps(h, n, 1, h->stream));
      // the n records, in at most two contiguous runs of the ring
      const long long s0 = (t0 + i0) % h->ring_cap;
      const int n1 = (int)std::min<long long>(n, h->ring_cap - s0);
      HIP_TRY(hipMemcpyAsync(rec.data() + (size_t)i0 * kRec, h->d_ring() + (size_t)s0 * kRec,
                             sizeof(double) * kRec * n1, hipMemcpyDeviceToHost, h->stream));
      if (n1 < n)
        HIP_TRY(hipMemcpyAsync(rec.data() + (size_t)(i0 + n1) * kRec, h->d_ring(),
                               sizeof(double) * kRec * (n - n1), hipMemcpyDeviceToHost, h->stream));
      HIP_TRY(hipStreamSynchronize(h->stream));
    }
    for (int i = 0; i < len; ++i) scales[(size_t)j * k + i] = rec[(size_t)i * kRec + kScale];
  }
  ST_TRY(read_states(h, st));
  ST_TRY(check_bad(h, st));
  // ---- energy of psi_T
  ST_TRY(observe(h, 0, false));
  HIP_TRY(hipMemcpyAsync(h->h_pin, h->d_obs(), sizeof(double) * kRec, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  const double S0 = h->h_pin[kS0];
  const double E = (h->h_pin[kKin] + h->h_pin[kPot]) / S0;
  if (!std::isfinite(E) || !(S0 > 0)) return fail(FDTD_ENONFINITE, "energy_grad: non-finite final energy");
  // ---- adjoint start: lambda_T = 2 (H psi_T - E psi_T) / S0, G = psi_T^2 / S0
  {
    AdjInitArgs a;
    memset(&a, 0, sizeof a);
    a.V = h->V(0);
    a.psi = h->psi(0, h->cur);
    a.lam = lam[0];
    a.G = G;
    a.G32 = G32;
    a.N = m.N;
    a.kin_scale = m.kin_scale;
    a.E = E;
    a.S0 = S0;
    HIP_TRY(launch_adjoint_init(h->dtype, a, h->stream));
  }
  int lc = 0;
  // descriptors: descs[i] maps buffer 0 -> sg[i], buffer 1 -> sg[i+1]
  {
    std::vector<MemberDev> md(seg);
    const MemberDev base = member_dev(h, 0);
    for (int i = 0; i < seg; ++i) {
      md[i] = base;
      md[i].psi[0] = sg + fb * i;
      md[i].psi[1] = sg + fb * (i + 1);
    }
    HIP_TRY(hipMemcpyAsync(descs, md.data(), sizeof(MemberDev) * seg, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
  }
  // recompute uses a private state slot so the handle's state is untouched
  MemberState* rst = cks + nck;
  for (int j = nck - 1; j >= 0; --j) {
    const int len = std::min(k, T - j * k);
    HIP_TRY(hipMemcpyAsync(sg, ck + fb * j, es * (size_t)m.n3, hipMemcpyDeviceToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(rst, cks + j, sizeof(MemberState), hipMemcpyDeviceToDevice, h->stream));
    for (int i = 0; i < len; ++i) {
      StepArgs a = base_args(h);
      a.members = descs + i;
      a.states = rst;
      a.src = 0;
      a.renorm_every = 1;
      a.ring = scratch;  // recompute records are not kept
      a.ring_cap = 1;
      HIP_TRY(launch_kernel(h, true, launch_grid(h, a.n_items), a, h->stream));
    }
    for (int i = len - 1; i >= 0; --i) {
      AdjArgs a;
      memset(&a, 0, sizeof a);
      a.V = h->V(0);
      a.lam_in = lam[lc];
      a.lam_out = lam[lc ^ 1];
      a.psi_t = sg + fb * i;
      a.psi_t1 = sg + fb * (i + 1);
      a.G = G32 ? static_cast<void*>(G32) : static_cast<void*>(G);
      a.N = m.N;
      a.c = m.c;
      a.dt = m.dt;
      a.s_t = scales[(size_t)j * k + i];
      HIP_TRY(launch_adjoint_step(h->dtype, a, h->stream));
      lc ^= 1;
    }
    if (G32) HIP_TRY(launch_fold_grad(G, G32, m.n3, h->stream));
  }
  if (dE_dV) HIP_TRY(hipMemcpyAsync(dE_dV, G, sizeof(double) * (size_t)m.n3, hipMemcpyDeviceToDevice, h->stream));
  if (nwrt > 0) {
    double* p_dev = scratch + 1024;
    int* wrt_dev = reinterpret_cast<int*>(scratch + 1024 + kMaxParams + 8);
    double* part = scratch + 8192;
    double* out_dev = scratch + 512;
    HIP_TRY(hipMemcpyAsync(p_dev, theta, sizeof(double) * ntheta, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(wrt_dev, wrt, sizeof(int) * nwrt, hipMemcpyHostToDevice, h->stream));
    const int nb = 512;
    HIP_TRY(launch_param_contract(G, m.N, m.ha, m.a, m.pkind, p_dev, ntheta, wrt_dev, nwrt, part, nb,
                                  out_dev, h->stream));
    HIP_TRY(hipMemcpyAsync(h->h_pin, out_dev, sizeof(double) * nwrt, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (int i = 0; i < nwrt; ++i) dE_dtheta[i] = h->h_pin[i];
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (energy) *energy = E;
  return FDTD_OK;
}
