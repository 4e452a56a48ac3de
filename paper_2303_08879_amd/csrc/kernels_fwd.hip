// Forward level kernels of the selective Fock-amplitude sweep (gfx950): one
// launch per sweep step S (all targets of one step are independent, Sec. 2.2).
// The per-point and per-(node, chunk) work lives in fwd_units.h.
#include <algorithm>
#include <cstring>

#include "fwd_units.h"

namespace fd {

template <typename R>
__global__ void k_prep(const cx<R>* __restrict__ A, const cx<R>* __restrict__ b, const cx<R>* __restrict__ c,
                       cx<R>* __restrict__ Ai, cx<R>* __restrict__ bi, cx<R>* __restrict__ ci,
                       cx<R>* __restrict__ f0node0, PrepArgs a, int* status) {
  prep_body<R>(A, b, c, Ai, bi, ci, f0node0, a, status);
}

// Step 1 of Algorithm 2: one wavefront, the undetected block in LDS.
template <typename R, int NQ>
__global__ __launch_bounds__(64) void k_ufill(DevPlan P, const cx<R>* __restrict__ Ai,
                                              const cx<R>* __restrict__ bi, cx<R>* G,
                                              const int* __restrict__ elist, const int* __restrict__ woff,
                                              int wmax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  ufill_body<R, NQ>(P, Ai, bi, G, elist, woff, wmax, reinterpret_cast<cx<R>*>(smem_raw));
}

// Algorithm 1 (every mode detected): one thread per lattice point of level S.
template <int MD, bool ODD, typename R>
__global__ __launch_bounds__(kThreads) void k_fwd_point(DevPlan P, LevelPtrs<R> L, const cx<R>* __restrict__ Ai,
                                                        const cx<R>* __restrict__ bi, int S, int nwork) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* sq = reinterpret_cast<R*>(smem_raw);
  R* isq = sq + (kMaxCut + 4);
  int* spn = reinterpret_cast<int*>(isq + (kMaxCut + 4));
  load_tables(P, spn, sq, isq);
  __syncthreads();
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nwork) return;
  fwd_point_unit<MD, ODD, R>(P, L, Ai, bi, spn, sq, isq, S, r);
}

// Algorithm 2: one wavefront per (lattice point, chunk of undetected rows).
template <int MD, int NQ, typename R>
__global__ __launch_bounds__(kBT) void k_fwd_block(DevPlan P, LevelPtrs<R> L, const cx<R>* __restrict__ Ai,
                                                   const cx<R>* __restrict__ bi, int S, int nwork, ChunkGeo G) {
  constexpr int NPOS = NQ + 2 * MD;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int R0 = G.R0;
  cx<R>* lf0 = reinterpret_cast<cx<R>*>(smem_raw);             // (RC + 2) rows
  cx<R>* lpk = lf0 + (size_t)(G.RC + 2) * R0;                  // MD x (RC + 1) rows
  cx<R>* sA = lpk + (size_t)MD * (G.RC + 1) * R0;              // A (NPOS x NPOS) then b (NPOS)
  const cx<R>* sb = sA + NPOS * NPOS;
  R* sq = reinterpret_cast<R*>(sA + NPOS * NPOS + NPOS);
  R* isq = sq + (kMaxCut + 4);
  for (int v = threadIdx.x; v < kMaxCut + 4; v += blockDim.x) {
    sq[v] = sqrt(R(v));
    isq[v] = v ? R(1) / sqrt(R(v)) : R(0);
  }
  for (int i = threadIdx.x; i < NPOS * NPOS + NPOS; i += blockDim.x) sA[i] = ld(Ai + i);
  // one wavefront per workgroup: the unit's first wave_sync orders these
  // LDS writes before their reads
  for (int w = blockIdx.x; w < nwork * G.nchunks; w += gridDim.x) {
    const int r = w / G.nchunks, c = w - r * G.nchunks;
    fwd_block_unit<MD, NQ, R>(P, L, sA, sb, sq, isq, S, r, c, G, lf0, lpk);
  }
}

// F0 (level-major nodes of B entries) -> rho, C order [kappa][n_D].
template <typename R>
__global__ __launch_bounds__(kThreads) void k_out_perm(DevPlan P, const cx<R>* __restrict__ f0,
                                                       cx<R>* __restrict__ rho, int64_t N, int64_t total,
                                                       int* status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int* spn = reinterpret_cast<int*>(smem_raw);
  int64_t* slv = reinterpret_cast<int64_t*>(smem_raw + 16 * ((((P.MD + 1) * P.pnw) * 4 + 15) / 16));
  const int npn = (P.MD + 1) * P.pnw;
  for (int i = threadIdx.x; i < npn; i += blockDim.x) spn[i] = P.pn[i];
  for (int i = threadIdx.x; i <= P.smax; i += blockDim.x) slv[i] = P.MD > 0 ? P.lvl[i] : 0;
  __syncthreads();
  int bad = 0;
  if (P.B > 1) {
    cx<R>* tl = reinterpret_cast<cx<R>*>(reinterpret_cast<unsigned char*>(slv) + 16 * (((P.smax + 2) * 8 + 15) / 16));
    const int64_t tiles = ((N + kOutTN - 1) / kOutTN) * ((P.B + kOutTK - 1) / kOutTK);
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) bad |= out_perm_tile<R>(P, spn, slv, f0, rho, N, t, tl);
  } else {
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
      const cx<R> v = out_perm_elem<R>(P, spn, slv, f0, N, idx);
      if (!isfinite(v.x) || !isfinite(v.y)) bad = 1;
      st(rho + idx, v);
    }
  }
  if (bad) atomicOr(status, 1);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
// Rows of the first undetected coordinate per chunk: about `target` own
// entries (default one wavefront), spread evenly over the rows.
ChunkGeo chunk_geo(const Plan& Pl, int target) {
  ChunkGeo G;
  G.C0 = Pl.udims[0];
  G.R0 = Pl.B / G.C0;
  int rc = std::max(1, (target + G.R0 / 2) / G.R0);
  rc = std::min(rc, G.C0);
  G.nchunks = (G.C0 + rc - 1) / rc;
  G.RC = (G.C0 + G.nchunks - 1) / G.nchunks;
  return G;
}

template <typename R>
static hipError_t launch_fwd_level_t(const Plan& Pl, const DevPlan& P, bool odd, int S, const LevelPtrs<R>& L,
                                     const void* Ai, const void* bi, hipStream_t st) {
  const int MD = Pl.MD;
  if (MD == 0) return hipSuccess;
  const int nwork = (int)Pl.ncnt[S];   // lattice points of level S
  if (nwork <= 0) return hipSuccess;
  const cx<R>* A = reinterpret_cast<const cx<R>*>(Ai);
  const cx<R>* b = reinterpret_cast<const cx<R>*>(bi);
  const size_t tab = 2 * (kMaxCut + 4) * sizeof(R) + (size_t)(MD + 1) * (Pl.smax + 3) * sizeof(int);
  if (Pl.B == 1) {
    const int grid = (nwork + kThreads - 1) / kThreads;
#define FD_LAUNCH_POINT(MDV)                                                                              \
  case MDV:                                                                                               \
    if (odd)                                                                                              \
      hipLaunchKernelGGL((k_fwd_point<MDV, true, R>), dim3(grid), dim3(kThreads), tab, st, P, L, A, b, S, \
                         nwork);                                                                          \
    else                                                                                                  \
      hipLaunchKernelGGL((k_fwd_point<MDV, false, R>), dim3(grid), dim3(kThreads), tab, st, P, L, A, b, \
                         S, nwork);                                                                       \
    break;
    switch (MD) {
      FD_LAUNCH_POINT(1)
      FD_LAUNCH_POINT(2)
      FD_LAUNCH_POINT(3)
      FD_LAUNCH_POINT(4)
      FD_LAUNCH_POINT(5)
      FD_LAUNCH_POINT(6)
      FD_LAUNCH_POINT(7)
      FD_LAUNCH_POINT(8)
      default:
        return hipErrorInvalidValue;
    }
#undef FD_LAUNCH_POINT
  } else {
    // a level with few units is latency-bound: halve the chunks to put more
    // wavefronts in flight (config-2-sized levels: -7 %); a large level keeps
    // whole-wavefront chunks (halving them costs 30-40 % there)
    ChunkGeo G = chunk_geo(Pl);
    if ((int64_t)nwork * G.nchunks < kSmallLevelUnits) G = chunk_geo(Pl, kBT / 2);
    const size_t shm = (((size_t)(G.RC + 2) + (size_t)MD * (G.RC + 1)) * G.R0 + (size_t)Pl.npos * (Pl.npos + 1)) *
                           sizeof(cx<R>) + 2 * (kMaxCut + 4) * sizeof(R);
    const int grid = nwork * G.nchunks;
#define FD_LAUNCH_BLOCK(MDV)                                                                               \
  case MDV:                                                                                                \
    if (Pl.nq == 2) {                                                                                      \
      if (shm > 65536)                                                                                     \
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fwd_block<MDV, 2, R>),                 \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);                   \
      hipLaunchKernelGGL((k_fwd_block<MDV, 2, R>), dim3(grid), dim3(kBT), shm, st, P, L, A, b, S,         \
                         nwork, G);                                                                        \
    } else {                                                                                               \
      if (shm > 65536)                                                                                     \
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fwd_block<MDV, 4, R>),                 \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);                   \
      hipLaunchKernelGGL((k_fwd_block<MDV, 4, R>), dim3(grid), dim3(kBT), shm, st, P, L, A, b, S,         \
                         nwork, G);                                                                        \
    }                                                                                                      \
    break;
    switch (MD) {
      FD_LAUNCH_BLOCK(1)
      FD_LAUNCH_BLOCK(2)
      FD_LAUNCH_BLOCK(3)
      FD_LAUNCH_BLOCK(4)
      FD_LAUNCH_BLOCK(5)
      FD_LAUNCH_BLOCK(6)
      FD_LAUNCH_BLOCK(7)
      FD_LAUNCH_BLOCK(8)
      default:
        return hipErrorInvalidValue;
    }
#undef FD_LAUNCH_BLOCK
  }
  return hipGetLastError();
}

// Node-0 pointer of family f of group g at level S.
template <typename R>
static cx<R>* fam_level_ptr(const Plan& Pl, char* base, size_t off, int g, int S, bool ring) {
  if (S < 0) return nullptr;
  const size_t eb = sizeof(cx<R>);
  size_t node = ring ? (size_t)(S & 1) * Pl.maxN[g] : (size_t)Pl.lvl[(size_t)g * (Pl.smax + 2) + S];
  return reinterpret_cast<cx<R>*>(base + off + node * Pl.B * eb);
}

hipError_t launch_prep(const Plan& Pl, const void* A, const void* b, const void* c, void* Ai, void* f0node0,
                       hipStream_t st) {
  PrepArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  for (int p = 0; p < Pl.npos; ++p) pa.pos2blk[p] = Pl.pos2blk[p];
  pa.npos = Pl.npos;
  pa.M2 = 2 * Pl.M;
  pa.check_b_zero = (Pl.flags == FD_B_ZERO) ? 1 : 0;
  const size_t n2 = (size_t)Pl.npos * Pl.npos;
  if (Pl.dt == FD_C64) {
    cx<float>* a = reinterpret_cast<cx<float>*>(Ai);
    hipLaunchKernelGGL((k_prep<float>), dim3(1), dim3(kThreads), 0, st, reinterpret_cast<const cx<float>*>(A),
                       reinterpret_cast<const cx<float>*>(b), reinterpret_cast<const cx<float>*>(c), a, a + n2,
                       a + n2 + Pl.npos, reinterpret_cast<cx<float>*>(f0node0), pa, Pl.d_status);
  } else {
    cx<double>* a = reinterpret_cast<cx<double>*>(Ai);
    hipLaunchKernelGGL((k_prep<double>), dim3(1), dim3(kThreads), 0, st, reinterpret_cast<const cx<double>*>(A),
                       reinterpret_cast<const cx<double>*>(b), reinterpret_cast<const cx<double>*>(c), a, a + n2,
                       a + n2 + Pl.npos, reinterpret_cast<cx<double>*>(f0node0), pa, Pl.d_status);
  }
  return hipGetLastError();
}

// Plans with a total photon cutoff return F0 in level order: a copy with the
// non-finite check.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_copy_levels(const cx<R>* __restrict__ f0, cx<R>* __restrict__ rho,
                                                          int64_t n, int* status) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const cx<R> v = ld(f0 + i);
    if (!isfinite(v.x) || !isfinite(v.y)) bad = 1;
    st(rho + i, v);
  }
  if (bad) atomicOr(status, 1);
}

// Partial masses of level S = S0 + blockIdx.y (the sum of Re F0, i.e. of the
// detection probabilities of the level): part blockIdx.x of kMassParts
// contiguous chunks, strided per-thread sums, then a fixed-order tree;
// mass[S * kMassParts + part].
template <typename R>
__global__ __launch_bounds__(kThreads) void k_level_mass(const cx<R>* __restrict__ f0, const int64_t* __restrict__ lvl,
                                                         int S0, double* mass) {
  __shared__ double red[kThreads];
  const int S = S0 + blockIdx.y;
  const int64_t n = lvl[S + 1] - lvl[S];
  const int64_t chunk = (n + kMassParts - 1) / kMassParts;
  const int64_t i0 = lvl[S] + (int64_t)blockIdx.x * chunk;
  const int64_t i1 = min(lvl[S + 1], i0 + chunk);
  double acc = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) acc += (double)ld(f0 + i).x;
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) mass[(size_t)S * kMassParts + blockIdx.x] = red[0];
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_clear(cx<R>* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    st(p + i, czero<R>());
}

// F0 in node order -> rho (C order), with the non-finite check.
template <typename R>
static hipError_t launch_out_perm_t(const Plan& Pl, const DevPlan& P, const cx<R>* f0, void* rho, hipStream_t st) {
  if (Pl.level_cap >= 0) {
    const int64_t n = Pl.nodes_total;
    KTimer kt(Pl, KK_OUT_PERM, st);
    hipLaunchKernelGGL((k_copy_levels<R>), dim3((unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 65536)),
                       dim3(kThreads), 0, st, f0, reinterpret_cast<cx<R>*>(rho), n, Pl.d_status);
    return hipGetLastError();
  }
  const int64_t total = Pl.out_elems;
  const int64_t tiles = ((Pl.nodes_total + kOutTN - 1) / kOutTN) * ((Pl.B + kOutTK - 1) / kOutTK);
  const int64_t grid = std::min<int64_t>(Pl.B > 1 ? tiles : (total + kThreads - 1) / kThreads, 65536);
  const size_t shm = 16 * ((((size_t)(Pl.MD + 1) * (Pl.smax + 3)) * 4 + 15) / 16) +
                     16 * (((size_t)(Pl.smax + 2) * 8 + 15) / 16) + (size_t)kOutTN * (kOutTK + 1) * sizeof(cx<R>);
  KTimer kt(Pl, KK_OUT_PERM, st);
  hipLaunchKernelGGL((k_out_perm<R>), dim3(grid), dim3(kThreads), shm, st, P, f0, reinterpret_cast<cx<R>*>(rho),
                     (int64_t)Pl.nodes_total, total, Pl.d_status);
  return hipGetLastError();
}

template <typename R>
static hipError_t run_forward_t(const Plan& Pl, bool odd, const void* A, const void* b, const void* c, void* rho,
                                char* ws, char* saved, hipStream_t st, StopRule* stop) {
  const bool store_all = saved != nullptr;
  // prep lives in the workspace; intermediates in `saved` (store-all) or the workspace (ring)
  FwdLayout Lw = fwd_layout(Pl, odd, false, 0);
  FwdLayout Ls = fwd_layout(Pl, true, true, 0);
  char* fb = store_all ? saved : ws;
  const FwdLayout& LF = store_all ? Ls : Lw;
  cx<R>* Ai = reinterpret_cast<cx<R>*>(ws + Lw.prep);
  cx<R>* bi = Ai + (size_t)Pl.npos * Pl.npos;
  cx<R>* ci = bi + Pl.npos;
  cx<R>* f0 = reinterpret_cast<cx<R>*>(fb + LF.f0);
  DevPlan P = make_devplan(Pl, odd);
  (void)ci;
  hipError_t e;
  if (stop) {
    stop->levels_done = Pl.smax + 1;
    stop->mass = 0.0;
  }
  {
    KTimer kt(Pl, KK_PREP, st);
    e = launch_prep(Pl, A, b, c, Ai, f0, st);
  }
  if (e != hipSuccess) return e;
  if (Pl.B > 1) {
    KTimer kt(Pl, KK_UFILL, st);
    const size_t shm = ufill_lds_bytes(Pl, false);
    auto* kfn = Pl.nq == 2 ? &k_ufill<R, 2> : &k_ufill<R, 4>;
    if (shm > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kfn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shm);
    hipLaunchKernelGGL(kfn, dim3(1), dim3(64), shm, st, P, Ai, bi, f0, Pl.d_elist, Pl.d_woff, Pl.wmax);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  for (int S = 0; S <= Pl.smax && Pl.MD > 0; ++S) {
    LevelPtrs<R> L;
    std::memset(&L, 0, sizeof(L));
    for (int f = 1; f < Pl.nfam; ++f) {
      if (LF.fam[f] == 0) continue;
      const int g = Pl.fam_group[f];
      L.rd[f] = fam_level_ptr<R>(Pl, fb, LF.fam[f], g, S - 1, !store_all);
      L.wr[f] = fam_level_ptr<R>(Pl, fb, LF.fam[f], g, S, !store_all);
    }
    L.f0cur = fam_level_ptr<R>(Pl, fb, LF.f0, 0, S, false);
    L.node = Pl.d_node ? Pl.d_node + (size_t)Pl.lvl[S] * kNodeStride : nullptr;
    L.f0nxt = S < Pl.smax ? fam_level_ptr<R>(Pl, fb, LF.f0, 0, S + 1, false) : nullptr;
    {
      KTimer kt(Pl, KK_FWD_LEVEL, st);
      e = launch_fwd_level_t<R>(Pl, P, odd, S, L, Ai, bi, st);
    }
    if (e != hipSuccess) return e;
    if (stop && ((S + 1) % kStopBlock == 0 || S == Pl.smax)) {
      // levels S0..S are final (F0 of a level is written by the launch below it)
      const int S0 = S - S % kStopBlock;
      hipLaunchKernelGGL((k_level_mass<R>), dim3(kMassParts, S - S0 + 1), dim3(kThreads), 0, st, f0, Pl.d_lvl, S0,
                         Pl.d_mass);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      double hm[kStopBlock * kMassParts];
      if ((e = hipMemcpyAsync(hm, Pl.d_mass + (size_t)S0 * kMassParts, (size_t)(S - S0 + 1) * kMassParts * sizeof(double),
                              hipMemcpyDeviceToHost, st)) != hipSuccess ||
          (e = hipStreamSynchronize(st)) != hipSuccess)
        return e;
      int hit = -1;
      for (int k = 0; k <= S - S0 && hit < 0; ++k) {
        double m = 0.0;
        for (int q = 0; q < kMassParts; ++q) m += hm[k * kMassParts + q];
        stop->mass += m;
        if (stop->mass >= 1.0 - stop->eps) hit = S0 + k;
      }
      if (hit >= 0) {
        stop->levels_done = hit + 1;
        const int64_t from = Pl.lvl[hit + 1], to = Pl.lvl[Pl.smax + 1];   // F0 above level hit
        if (to > from) {
          hipLaunchKernelGGL((k_clear<R>), dim3((unsigned)std::min<int64_t>((to - from + kThreads - 1) / kThreads, 65536)),
                             dim3(kThreads), 0, st, f0 + from, to - from);
          if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        break;
      }
    }
  }
  if (!rho) return hipSuccess;   // recompute for the reverse sweep: no output needed
  return launch_out_perm_t<R>(Pl, P, f0, rho, st);
}

hipError_t launch_out_perm(const Plan& Pl, const void* f0, void* rho, hipStream_t st) {
  const DevPlan P = make_devplan(Pl, false);
  if (Pl.dt == FD_C64) return launch_out_perm_t<float>(Pl, P, static_cast<const cx<float>*>(f0), rho, st);
  return launch_out_perm_t<double>(Pl, P, static_cast<const cx<double>*>(f0), rho, st);
}

hipError_t run_forward(const Plan& Pl, bool odd, const void* A, const void* b, const void* c, void* rho, void* ws,
                       void* saved, hipStream_t st, StopRule* stop) {
  if (Pl.dt == FD_C64)
    return run_forward_t<float>(Pl, odd, A, b, c, rho, (char*)ws, (char*)saved, st, stop);
  return run_forward_t<double>(Pl, odd, A, b, c, rho, (char*)ws, (char*)saved, st, stop);
}

}  // namespace fd
