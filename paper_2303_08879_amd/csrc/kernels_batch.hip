// Batched forward: prep and permutation kernels of a batch and the host-side
// schedule (work items, per-circuit descriptors), cached per plan set and
// pointer set.  The persistent sweep kernel itself is in batch_sweep.h.
//
// Launch sequence per batch: prep (+ undetected block fill), one workgroup
// per circuit; the persistent sweep; the F0 -> rho permutation of every
// circuit in one launch.
#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>

#include "batch_sweep.h"

namespace fd {

// Prep of every circuit (one workgroup each), then step 1 of Algorithm 2 by
// the first wavefront when the circuit has undetected modes.  Workgroup 0
// also clears the sweep's control words (queue heads, barrier count).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_batch_prep(const BatchCirc<R>* __restrict__ circs, unsigned* ctl,
                                                         int nctl) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const BatchCirc<R>* __restrict__ C = circs + blockIdx.x;
  cx<R>* Ai = load_global(&C->Ai);
  cx<R>* f0 = load_global(&C->f0);
  const int npos = C->P.npos;
  prep_body<R>(load_global(&C->A), load_global(&C->b), load_global(&C->c), Ai, Ai + npos * npos,
               Ai + npos * npos + npos, f0, C->pa, load_global(&C->status));
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < nctl; i += blockDim.x) ctl[i] = 0u;
  if (C->P.B == 1) return;
  __syncthreads();
  if (threadIdx.x < 64) {
    if (C->P.nq == 2)
      ufill_body<R, 2>(C->P, Ai, Ai + npos * npos, f0, load_global(&C->elist), load_global(&C->woff), C->wmax,
                       reinterpret_cast<cx<R>*>(smem_raw));
    else
      ufill_body<R, 4>(C->P, Ai, Ai + npos * npos, f0, load_global(&C->elist), load_global(&C->woff), C->wmax,
                       reinterpret_cast<cx<R>*>(smem_raw));
  }
}

// F0 -> rho of every circuit; block b belongs to the circuit c with
// boff[c] <= b < boff[c + 1] and is one LDS tile of it (undetected modes) or
// kThreads x kOutIter consecutive outputs (every mode detected).
template <typename R>
__global__ __launch_bounds__(kThreads) void k_batch_out(const BatchCirc<R>* __restrict__ circs,
                                                        const int64_t* __restrict__ boff, int n, int pn_bytes,
                                                        int slv_bytes) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t blk = blockIdx.x;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (boff[mid] <= blk)
      lo = mid;
    else
      hi = mid - 1;
  }
  const BatchCirc<R>* __restrict__ C = circs + lo;
  int* spn = reinterpret_cast<int*>(smem_raw);
  int64_t* slv = reinterpret_cast<int64_t*>(smem_raw + pn_bytes);
  const int npn = (C->P.MD + 1) * C->P.pnw;
  const int* pn = load_global(&C->P.pn);
  const int64_t* lvl = load_global(&C->P.lvl);
  for (int i = threadIdx.x; i < npn; i += blockDim.x) spn[i] = pn[i];
  for (int i = threadIdx.x; i <= C->P.smax; i += blockDim.x) slv[i] = C->P.MD > 0 ? lvl[i] : 0;
  __syncthreads();
  const cx<R>* f0 = load_global(&C->f0);
  cx<R>* rho = load_global(&C->rho);
  if (C->P.B > 1) {
    cx<R>* tl = reinterpret_cast<cx<R>*>(smem_raw + pn_bytes + slv_bytes);
    if (out_perm_tile<R>(C->P, spn, slv, f0, rho, C->N, blk - boff[lo], tl)) atomicOr(load_global(&C->status), 1);
    return;
  }
  const int64_t base = (blk - boff[lo]) * (int64_t)kThreads * kOutIter;
  int bad = 0;
#pragma unroll
  for (int k = 0; k < kOutIter; ++k) {
    const int64_t idx = base + (int64_t)k * kThreads + threadIdx.x;
    if (idx < C->out_elems) {
      const cx<R> v = out_perm_elem<R>(C->P, spn, slv, f0, C->N, idx);
      if (!isfinite(v.x) || !isfinite(v.y)) bad = 1;
      st(rho + idx, v);
    }
  }
  if (bad) atomicOr(load_global(&C->status), 1);
}

// ---------------------------------------------------------------------------
// host side: schedule construction (cached per plan set and pointer set)
// ---------------------------------------------------------------------------
namespace {

struct BatchSched {
  int device = -1;
  std::vector<uint64_t> key;
  std::vector<uint64_t> uids;
  void* d_circs = nullptr;
  void* d_items = nullptr;
  void* d_boff = nullptr;
  void* d_steps = nullptr;             // step offsets into the item table
  void* d_ctl = nullptr;               // queue heads of every step, then the barrier count
  int nitems = 0, nsteps = 0;
  int64_t out_blocks = 0;
  BatchLds lds{};
  size_t shm_prep = 0, shm_sweep = 0, shm_out = 0;
  int out_pn_bytes = 0, out_slv_bytes = 0;
  int grid = 0;
  int mdmax = 8;
  uint64_t last_use = 0;
  std::vector<unsigned char> h_circs;   // host images kept alive for the asynchronous uploads
  std::vector<BatchItem> h_items;
  std::vector<int64_t> h_boff;
  std::vector<int> h_steps;
};

std::mutex g_mu;
std::vector<BatchSched> g_cache;
fd_batch_tuning g_tuning = {2, 64, 4, 2048, 0};

fd_batch_tuning batch_tuning() { return g_tuning; }
uint64_t g_clock = 0;
constexpr size_t kBatchCache = 8;

void free_sched(BatchSched& s) {
  if (unloading()) return;   // the HIP runtime may be gone
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(s.device);
  (void)hipFree(s.d_circs);
  (void)hipFree(s.d_items);
  (void)hipFree(s.d_boff);
  (void)hipFree(s.d_steps);
  (void)hipFree(s.d_ctl);
  (void)hipSetDevice(cur);
  s.d_circs = s.d_items = s.d_boff = s.d_steps = s.d_ctl = nullptr;
}

size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

template <typename R>
fd_status build_sched(int n, Plan* const* plans, const bool* odd, const void* const* A, const void* const* b,
                 const void* const* c, void* const* rho, void* const* ws, hipStream_t st, BatchSched* S,
                 std::string* err) {
  const size_t eb = sizeof(cx<R>);
  std::vector<BatchCirc<R>> hc(n);
  BatchLds lds{16, 0, 0, 4};
  int out_pn = 16;
  int64_t out_slv = 8;
  size_t ufill_lds = 0;
  std::vector<double> work(n, 0.0);
  for (int i = 0; i < n; ++i) {
    const Plan& Pl = *plans[i];
    BatchCirc<R>& C = hc[i];
    std::memset(&C, 0, sizeof(C));
    C.P = make_devplan(Pl, odd[i]);
    C.kind = Pl.B > 1 ? 1 : 0;
    if (Pl.nq > 4) {
      *err = "the batched sweep runs at most two undetected modes";
      return FD_ERR_UNSUPPORTED;
    }
    if (C.kind) {
      C.G = chunk_geo(Pl);
      C.Gh = chunk_geo(Pl, kBT / 2);
    }
    for (int p = 0; p < Pl.npos; ++p) C.pa.pos2blk[p] = Pl.pos2blk[p];
    C.pa.npos = Pl.npos;
    C.pa.M2 = 2 * Pl.M;
    C.pa.check_b_zero = Pl.flags == FD_B_ZERO ? 1 : 0;
    C.steps = Pl.MD > 0 ? Pl.smax + 1 : 0;
    C.wmax = Pl.wmax;
    const FwdLayout Lw = fwd_layout(Pl, odd[i], false, 0);
    char* w = static_cast<char*>(ws[i]);
    for (int f = 1; f < Pl.nfam; ++f) {
      if (Lw.fam[f] == 0) continue;
      C.fam[f] = reinterpret_cast<cx<R>*>(w + Lw.fam[f]);
      C.fstride[f] = Pl.maxN[Pl.fam_group[f]] * (int64_t)Pl.B;
    }
    C.f0 = reinterpret_cast<cx<R>*>(w + Lw.f0);
    C.Ai = reinterpret_cast<cx<R>*>(w + Lw.prep);
    C.A = static_cast<const cx<R>*>(A[i]);
    C.b = static_cast<const cx<R>*>(b[i]);
    C.c = static_cast<const cx<R>*>(c[i]);
    C.rho = static_cast<cx<R>*>(rho[i]);
    C.elist = Pl.d_elist;
    C.woff = Pl.d_woff;
    C.status = Pl.d_status;
    C.out_elems = Pl.out_elems;
    C.N = Pl.nodes_total;
    const int pnb = (int)align16((size_t)(Pl.MD + 1) * (Pl.smax + 3) * sizeof(int));
    lds.pn_bytes = std::max(lds.pn_bytes, pnb);
    out_pn = std::max(out_pn, pnb);
    out_slv = std::max<int64_t>(out_slv, (int64_t)(Pl.smax + 2) * 8);
    if (C.kind) {
      lds.sa_bytes = std::max(lds.sa_bytes, (int)align16((size_t)Pl.npos * (Pl.npos + 1) * eb));
      ufill_lds = std::max(ufill_lds, ufill_lds_bytes(Pl, false));
    }
    for (int s = 0; s < C.steps; ++s) work[i] += (double)Pl.ncnt[s] * Pl.B;
  }
  // per-wave bytes: PN, A/b, then the block unit rows (largest circuit): a
  // unit of chunk geometry G touches F0 rows [k0-2, k1) and MD bridge pivot
  // blocks of rows [k0-1, k1) (fwd_block_unit), for either of the circuit's
  // two geometries (full- and half-height chunks)
  size_t rows = 0;
  auto unit_rows = [&](const ChunkGeo& G, int MD) {
    return ((size_t)(G.RC + 2) + (size_t)MD * (G.RC + 1)) * G.R0 * eb;
  };
  for (int i = 0; i < n; ++i)
    if (hc[i].kind) rows = std::max({rows, unit_rows(hc[i].G, hc[i].P.MD), unit_rows(hc[i].Gh, hc[i].P.MD)});
  lds.wave_bytes = (int)align16((size_t)lds.pn_bytes + lds.sa_bytes + rows);
  lds.waves = 4;
  while (lds.waves > 1 && kTabBytes + (size_t)lds.waves * lds.wave_bytes > kMaxLds) --lds.waves;
  if (kTabBytes + (size_t)lds.wave_bytes > kMaxLds || ufill_lds > kMaxLds) {
    *err = "a circuit's undetected block is too large for the batched sweep's LDS staging";
    return FD_ERR_UNSUPPORTED;
  }
  S->lds = lds;
  S->shm_sweep = kTabBytes + (size_t)lds.waves * lds.wave_bytes;
  S->shm_prep = ufill_lds;
  S->out_pn_bytes = out_pn;
  S->out_slv_bytes = (int)align16((size_t)out_slv);
  S->shm_out = (size_t)out_pn + S->out_slv_bytes + (size_t)kOutTN * (kOutTK + 1) * eb;

  // persistent grid: every workgroup that fits at once
  bool small = true;   // within the (6, 5, 2) build
  for (int i = 0; i < n; ++i)
    small = small && (hc[i].kind ? (hc[i].P.MD <= 5 && hc[i].P.nq <= 2) : hc[i].P.MD <= 6);
  S->mdmax = small ? 6 : 8;
  if (S->shm_prep > 65536 &&
      hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_prep<R>), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)S->shm_prep) != hipSuccess) {
    *err = "hipFuncSetAttribute failed";
    return FD_ERR_HIP;
  }
  int per_cu = 0, cus = 0, dev = 0;
  (void)hipGetDevice(&dev);
  BatchSweepArgs qa{};
  qa.lds = lds;
  qa.shm = S->shm_sweep;
  const bool c64 = sizeof(R) == 4;
  const hipError_t qe = S->mdmax == 6 ? batch_sweep_md6(c64, &qa, &per_cu, nullptr)
                                      : batch_sweep_md8(c64, &qa, &per_cu, nullptr);
  if (qe == hipSuccess && per_cu == -1) {
    *err = "the batched sweep kernel was built with scratch memory; refusing its cooperative launch";
    return FD_ERR_UNSUPPORTED;
  }
  if (qe != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      per_cu < 1) {
    *err = "occupancy query for the batched sweep failed (" + std::string(hipGetErrorString(qe)) +
           ", workgroups per CU " + std::to_string(per_cu) + ", LDS bytes " + std::to_string(S->shm_sweep) +
           ", wavefronts per workgroup " + std::to_string(lds.waves) + ")";
    return FD_ERR_HIP;
  }
  int coop = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) {
    *err = "the device does not support cooperative launches";
    return FD_ERR_UNSUPPORTED;
  }
  S->grid = per_cu * cus;
  const int64_t waves = (int64_t)S->grid * lds.waves;

  // work items, step-major; within a step larger circuits first, each step
  // of a circuit cut into items of units / (items_per_wave x wavefronts)
  // units, at least min_block_units / min_point_units
  const fd_batch_tuning T = batch_tuning();
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
  int max_steps = 0;
  for (int i = 0; i < n; ++i) max_steps = std::max(max_steps, hc[i].steps);
  const int64_t div = std::max<int64_t>(1, (int64_t)T.items_per_wave * waves);
  S->h_items.clear();
  S->h_steps.assign(1, 0);
  for (int s = 0; s < max_steps; ++s) {
    for (int i : order) {
      if (s >= hc[i].steps) continue;
      const int64_t pts = plans[i]->ncnt[s];
      if (pts <= 0) continue;
      const bool half = hc[i].kind && pts * hc[i].G.nchunks < kSmallLevelUnits;
      const int64_t units = hc[i].kind ? pts * (half ? hc[i].Gh.nchunks : hc[i].G.nchunks) : pts;
      int64_t per = std::max<int64_t>(hc[i].kind ? T.min_block_units : T.min_point_units, (units + div - 1) / div);
      if (!hc[i].kind) per = (per + 63) / 64 * 64;   // whole wavefronts of lattice points
      if (units > 0x7fffffff) {
        *err = "a step of circuit " + std::to_string(i) + " has too many units for one work item table";
        return FD_ERR_UNSUPPORTED;
      }
      for (int64_t u0 = 0; u0 < units; u0 += per) {
        BatchItem I;
        std::memset(&I, 0, sizeof(I));
        I.circ = i;
        I.step = s;
        I.u0 = (int)u0;
        I.u1 = (int)std::min(units, u0 + per);
        I.half = half ? 1 : 0;
        // an item covers whole units of its own geometry: (lattice point, chunk)
        // pairs below pts x nchunks, or lattice points below pts
        if (I.u0 < 0 || I.u1 <= I.u0 || I.u1 > units) {
          *err = "internal error: batch work item outside its step's units";
          return FD_ERR_HIP;
        }
        S->h_items.push_back(I);
      }
    }
    S->h_steps.push_back((int)S->h_items.size());
  }
  S->nsteps = max_steps;
  S->nitems = (int)S->h_items.size();
  // permutation blocks
  S->h_boff.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    const int64_t per_blk = (int64_t)kThreads * kOutIter;
    const int64_t blocks = hc[i].P.B > 1 ? ((hc[i].N + kOutTN - 1) / kOutTN) * ((hc[i].P.B + kOutTK - 1) / kOutTK)
                                         : (hc[i].out_elems + per_blk - 1) / per_blk;
    S->h_boff[i + 1] = S->h_boff[i] + blocks;
  }
  S->out_blocks = S->h_boff[n];
  if (S->out_blocks > 0x7fffffff) {
    *err = "batch output too large for one permutation launch";
    return FD_ERR_UNSUPPORTED;
  }
  // upload
  S->h_circs.resize(sizeof(BatchCirc<R>) * n);
  std::memcpy(S->h_circs.data(), hc.data(), S->h_circs.size());
  S->device = dev;
  if (hipMalloc(&S->d_circs, S->h_circs.size()) != hipSuccess ||
      hipMalloc(&S->d_items, std::max<size_t>(1, S->h_items.size()) * sizeof(BatchItem)) != hipSuccess ||
      hipMalloc(&S->d_boff, S->h_boff.size() * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&S->d_steps, S->h_steps.size() * sizeof(int)) != hipSuccess ||
      hipMalloc(&S->d_ctl, ((size_t)S->nsteps + 1) * sizeof(unsigned)) != hipSuccess) {
    free_sched(*S);
    *err = "device allocation of the batch schedule failed";
    return FD_ERR_OOM;
  }
  if (hipMemcpyAsync(S->d_circs, S->h_circs.data(), S->h_circs.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
      (S->nitems > 0 && hipMemcpyAsync(S->d_items, S->h_items.data(), S->h_items.size() * sizeof(BatchItem),
                                       hipMemcpyHostToDevice, st) != hipSuccess) ||
      hipMemcpyAsync(S->d_boff, S->h_boff.data(), S->h_boff.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                     st) != hipSuccess ||
      hipMemcpyAsync(S->d_steps, S->h_steps.data(), S->h_steps.size() * sizeof(int), hipMemcpyHostToDevice, st) !=
          hipSuccess) {
    free_sched(*S);
    *err = "upload of the batch schedule failed";
    return FD_ERR_HIP;
  }
  return FD_OK;
}

template <typename R>
hipError_t launch_batch(const BatchSched& S, int n, const Plan& P0, hipStream_t st) {
  const BatchCirc<R>* circs = static_cast<const BatchCirc<R>*>(S.d_circs);
  unsigned* ctl = static_cast<unsigned*>(S.d_ctl);
  {
    KTimer kt(P0, KK_BATCH_PREP, st);
    hipLaunchKernelGGL((k_batch_prep<R>), dim3(n), dim3(kThreads), S.shm_prep, st, circs, ctl, S.nsteps + 1);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (S.nitems > 0) {
    KTimer kt(P0, KK_BATCH_SWEEP, st);
    BatchSweepArgs a{};
    a.circs = circs;
    a.items = S.d_items;
    a.step_off = static_cast<const int*>(S.d_steps);
    a.nsteps = S.nsteps;
    a.ctl = ctl;
    a.status = P0.d_status;
    a.lds = S.lds;
    a.grid = S.grid;
    a.shm = S.shm_sweep;
    const bool c64 = sizeof(R) == 4;
    e = S.mdmax == 6 ? batch_sweep_md6(c64, &a, nullptr, st) : batch_sweep_md8(c64, &a, nullptr, st);
    if (e != hipSuccess) return e;
  }
  {
    KTimer kt(P0, KK_BATCH_OUT, st);
    hipLaunchKernelGGL((k_batch_out<R>), dim3((unsigned)S.out_blocks), dim3(kThreads), S.shm_out, st, circs,
                       static_cast<const int64_t*>(S.d_boff), n, S.out_pn_bytes, S.out_slv_bytes);
  }
  return hipGetLastError();
}

}  // namespace

// A circuit fills the device on its own when its levels average at least
// `fill_waves` wavefront-sized units (about what the device holds at once,
// 2048 by default): such circuits run their own level launches, interleaving
// them with other large circuits only multiplies the working set the L2s and
// the MALL hold.
static bool fills_device(const Plan& Pl, double fill_waves) {
  if (Pl.MD == 0) return false;
  double units = 0.0;
  const ChunkGeo G = Pl.B > 1 ? chunk_geo(Pl) : ChunkGeo{1, 1, 1, 1};
  for (int s = 0; s <= Pl.smax; ++s)
    units += Pl.B > 1 ? (double)Pl.ncnt[s] * G.nchunks : (double)Pl.ncnt[s] / 64.0;
  return units / (Pl.smax + 1) >= fill_waves;
}

// The persistent sweep runs blocks of at most four coordinates (two
// undetected modes) whose unit rows and fill fit its LDS staging; other
// circuits take their own level launches.
// Per-wave LDS parts of a circuit in the sweep (as build_sched lays them
// out): its PN table, A and b, its block unit rows.
struct WaveParts {
  size_t pn = 0, sa = 0, rows = 0;
};
static WaveParts wave_parts(const Plan& Pl) {
  const size_t eb = elem_bytes(Pl.dt);
  WaveParts w;
  w.pn = align16((size_t)(Pl.MD + 1) * (Pl.smax + 3) * sizeof(int));
  if (Pl.B > 1) {
    w.sa = align16((size_t)Pl.npos * (Pl.npos + 1) * eb);
    for (const ChunkGeo& G : {chunk_geo(Pl), chunk_geo(Pl, kBT / 2)})
      w.rows = std::max(w.rows, ((size_t)(G.RC + 2) + (size_t)Pl.MD * (G.RC + 1)) * G.R0 * eb);
  }
  return w;
}
static bool sweep_takes(const Plan& Pl) {
  if (Pl.B == 1) return true;
  if (Pl.nq > 4) return false;
  const WaveParts w = wave_parts(Pl);
  return kTabBytes + align16(w.pn + w.sa + w.rows) <= kMaxLds && ufill_lds_bytes(Pl, false) <= kMaxLds;
}

namespace {

// Cache key of a batched call: device, plans, schedules, pointers, knobs.
std::vector<uint64_t> batch_key(int n, Plan* const* plans, const bool* odd, const void* const* A,
                                const void* const* b, const void* const* c, void* const* rho, void* const* ws,
                                const fd_batch_tuning& T) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::vector<uint64_t> key;
  key.reserve(7 + 7 * (size_t)n);
  key.push_back((uint64_t)dev);
  key.push_back((uint64_t)n);
  for (int i = 0; i < n; ++i) {
    key.push_back(plans[i]->uid);
    key.push_back(odd[i] ? 1 : 0);
    for (const void* p : {A[i], b[i], c[i], (const void*)rho[i], (const void*)ws[i]})
      key.push_back((uint64_t)reinterpret_cast<uintptr_t>(p));
  }
  key.push_back((uint64_t)T.min_block_units);
  key.push_back((uint64_t)T.min_point_units);
  key.push_back((uint64_t)T.items_per_wave);
  key.push_back((uint64_t)T.fill_waves);
  return key;
}

// The schedule of the persistent sweep over these circuits, built and
// uploaded on `st` on first use.  Caller holds g_mu.
fd_status sweep_sched(int n, Plan* const* plans, const bool* odd, const void* const* A, const void* const* b,
                      const void* const* c, void* const* rho, void* const* ws, const fd_batch_tuning& T,
                      hipStream_t st, BatchSched** out, std::string* err) {
  std::vector<uint64_t> key = batch_key(n, plans, odd, A, b, c, rho, ws, T);
  for (BatchSched& s : g_cache)
    if (s.key == key) {
      s.last_use = ++g_clock;
      *out = &s;
      return FD_OK;
    }
  BatchSched ns;
  ns.key = std::move(key);
  for (int i = 0; i < n; ++i) ns.uids.push_back(plans[i]->uid);
  const fd_status bs = plans[0]->dt == FD_C64 ? build_sched<float>(n, plans, odd, A, b, c, rho, ws, st, &ns, err)
                                              : build_sched<double>(n, plans, odd, A, b, c, rho, ws, st, &ns, err);
  if (bs != FD_OK) return bs;
  if (g_cache.size() >= kBatchCache) {
    auto it = std::min_element(g_cache.begin(), g_cache.end(),
                               [](const BatchSched& x, const BatchSched& y) { return x.last_use < y.last_use; });
    free_sched(*it);
    g_cache.erase(it);
  }
  g_cache.push_back(std::move(ns));
  *out = &g_cache.back();
  (*out)->last_use = ++g_clock;
  return FD_OK;
}

// A batched call captured into a graph: the level launches of the circuits
// that fill the device, then the persistent sweep's three launches.
struct BatchGraph {
  int device = -1;
  std::vector<uint64_t> key, uids;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t last_use = 0;
};
std::vector<BatchGraph> g_graphs;
hipStream_t g_capture[64] = {};   // private capture stream per device
bool g_graph_failed = false;      // a capture was refused: batched calls run eagerly

void free_graph(BatchGraph& g) {
  if (unloading()) return;
  (void)hipGraphExecDestroy(g.exec);
  (void)hipGraphDestroy(g.graph);
  g.exec = nullptr;
  g.graph = nullptr;
}

struct Split {
  std::vector<int> big, small;
};

Split split_batch(int n, Plan* const* plans, const fd_batch_tuning& T) {
  Split sp;
  for (int i = 0; i < n; ++i)
    (fills_device(*plans[i], (double)T.fill_waves) || !sweep_takes(*plans[i]) ? sp.big : sp.small).push_back(i);
  // one wave's LDS holds the largest PN table, A/b and unit rows of all
  // members together: while they do not fit, the member with the most unit
  // rows leaves the sweep
  for (;;) {
    WaveParts mx;
    int worst = -1;
    size_t worst_rows = 0;
    for (size_t k = 0; k < sp.small.size(); ++k) {
      const WaveParts w = wave_parts(*plans[sp.small[k]]);
      mx.pn = std::max(mx.pn, w.pn);
      mx.sa = std::max(mx.sa, w.sa);
      mx.rows = std::max(mx.rows, w.rows);
      if (worst < 0 || w.rows + w.sa > worst_rows) {
        worst = (int)k;
        worst_rows = w.rows + w.sa;
      }
    }
    if (worst < 0 || kTabBytes + align16(mx.pn + mx.sa + mx.rows) <= kMaxLds) break;
    sp.big.push_back(sp.small[worst]);
    sp.small.erase(sp.small.begin() + worst);
  }
  return sp;
}

// Enqueues the whole batched call on `st`: the circuits that fill the device
// (or that the sweep cannot stage) with their own level launches, then the
// sweep over the others (its schedule `S`, built beforehand).
hipError_t enqueue_batch(const Split& sp, Plan* const* plans, const bool* odd, const void* const* A,
                         const void* const* b, const void* const* c, void* const* rho, void* const* ws,
                         const BatchSched* S, hipStream_t st) {
  for (int i : sp.big) {
    const hipError_t e = run_forward(*plans[i], odd[i], A[i], b[i], c[i], rho[i], ws[i], nullptr, st);
    if (e != hipSuccess) return e;
  }
  if (!S) return hipSuccess;
  const Plan& P0 = *plans[sp.small[0]];
  return P0.dt == FD_C64 ? launch_batch<float>(*S, (int)sp.small.size(), P0, st)
                         : launch_batch<double>(*S, (int)sp.small.size(), P0, st);
}

}  // namespace

fd_status run_forward_batch(int n, Plan* const* plans, const bool* odd, const void* const* A,
                            const void* const* b, const void* const* c, void* const* rho, void* const* ws,
                            hipStream_t st, std::string* err) {
  if (n == 0) return FD_OK;
  std::lock_guard<std::mutex> lock(g_mu);
  const fd_batch_tuning T = g_tuning;
  const Split sp = split_batch(n, plans, T);
  // the sweep's members, as arrays of their own
  const size_t m = sp.small.size();
  std::vector<Plan*> p2(m);
  std::unique_ptr<bool[]> o2(new bool[m > 0 ? m : 1]);
  std::vector<const void*> A2(m), b2(m), c2(m);
  std::vector<void*> r2(m), w2(m);
  for (size_t k = 0; k < m; ++k) {
    const int i = sp.small[k];
    p2[k] = plans[i];
    o2[k] = odd[i];
    A2[k] = A[i];
    b2[k] = b[i];
    c2[k] = c[i];
    r2[k] = rho[i];
    w2[k] = ws[i];
  }
  BatchSched* S = nullptr;
  if (m > 0) {
    const fd_status s = sweep_sched((int)m, p2.data(), o2.get(), A2.data(), b2.data(), c2.data(), r2.data(),
                                    w2.data(), T, st, &S, err);
    if (s != FD_OK) return s;
  }
  bool timing = false;
  for (int i = 0; i < n; ++i) timing = timing || plans[i]->timing.mask != 0;
  auto fail_hip = [&](hipError_t e) {
    *err = std::string("kernel launch failed: ") + hipGetErrorString(e);
    return FD_ERR_HIP;
  };
  if (T.use_graph <= 0 || g_graph_failed || timing) {
    const hipError_t e = enqueue_batch(sp, plans, odd, A, b, c, rho, ws, S, st);
    return e == hipSuccess ? FD_OK : fail_hip(e);
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::vector<uint64_t> key = batch_key(n, plans, odd, A, b, c, rho, ws, T);
  for (BatchGraph& g : g_graphs)
    if (g.key == key) {
      g.last_use = ++g_clock;
      const hipError_t e = hipGraphLaunch(g.exec, st);
      return e == hipSuccess ? FD_OK : fail_hip(e);
    }
  hipError_t e;
  if (dev < 0 || dev >= 64) return fail_hip(hipErrorInvalidDevice);
  if (!g_capture[dev] && (e = hipStreamCreateWithFlags(&g_capture[dev], hipStreamNonBlocking)) != hipSuccess)
    return fail_hip(e);
  hipStream_t cs = g_capture[dev];
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool captured = false;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    const hipError_t eb = enqueue_batch(sp, plans, odd, A, b, c, rho, ws, S, cs);
    const hipError_t ee = hipStreamEndCapture(cs, &graph);
    captured = eb == hipSuccess && ee == hipSuccess && graph &&
               hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
  }
  (void)hipGetLastError();
  if (!captured) {
    // the runtime would not capture (cooperative launches, for one): run
    // this and later calls eagerly
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    g_graph_failed = true;
    e = enqueue_batch(sp, plans, odd, A, b, c, rho, ws, S, st);
    return e == hipSuccess ? FD_OK : fail_hip(e);
  }
  if (g_graphs.size() >= kBatchCache) {
    auto it = std::min_element(g_graphs.begin(), g_graphs.end(),
                               [](const BatchGraph& x, const BatchGraph& y) { return x.last_use < y.last_use; });
    free_graph(*it);
    g_graphs.erase(it);
  }
  BatchGraph g;
  g.device = dev;
  g.key = std::move(key);
  for (int i = 0; i < n; ++i) g.uids.push_back(plans[i]->uid);
  g.graph = graph;
  g.exec = exec;
  g.last_use = ++g_clock;
  g_graphs.push_back(std::move(g));
  e = hipGraphLaunch(exec, st);
  return e == hipSuccess ? FD_OK : fail_hip(e);
}

fd_status batch_set_tuning(const fd_batch_tuning& T) {
  if (T.min_block_units < 1 || T.min_point_units < 1 || T.items_per_wave < 1 || T.fill_waves < 1 ||
      T.use_graph < 0 || T.use_graph > 1)
    return FD_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_mu);
  g_tuning = T;
  return FD_OK;
}

fd_batch_tuning batch_get_tuning() {
  std::lock_guard<std::mutex> lock(g_mu);
  fd_batch_tuning t = g_tuning;
  if (t.use_graph > 0 && g_graph_failed) t.use_graph = -1;
  return t;
}

void batch_forget(uint64_t uid) {
  std::lock_guard<std::mutex> lock(g_mu);
  for (size_t i = 0; i < g_graphs.size();) {
    if (std::find(g_graphs[i].uids.begin(), g_graphs[i].uids.end(), uid) != g_graphs[i].uids.end()) {
      free_graph(g_graphs[i]);
      g_graphs.erase(g_graphs.begin() + i);
    } else {
      ++i;
    }
  }
  for (size_t i = 0; i < g_cache.size();) {
    if (std::find(g_cache[i].uids.begin(), g_cache[i].uids.end(), uid) != g_cache[i].uids.end()) {
      free_sched(g_cache[i]);
      g_cache.erase(g_cache.begin() + i);
    } else {
      ++i;
    }
  }
}

}  // namespace fd
