// Forward level kernels of the selective Fock-amplitude sweep (gfx950): one
// launch per sweep step S (all targets of one step are independent, Sec. 2.2).
// The per-point and per-(node, chunk) work lives in fwd_units.h.
#include <algorithm>
#include <cstring>
#include <type_traits>

#include "fwd_units.h"

namespace fd {

template <typename R>
__global__ void k_prep(const cx<R>* __restrict__ A, const cx<R>* __restrict__ b, const cx<R>* __restrict__ c,
                       cx<R>* __restrict__ Ai, cx<R>* __restrict__ bi, cx<R>* __restrict__ ci,
                       cx<R>* __restrict__ f0node0, PrepArgs a, int* status) {
  prep_body<R>(A, b, c, Ai, bi, ci, f0node0, a, status);
}

// Step 1 of Algorithm 2: one wavefront, the undetected block in LDS (with
// E = dual<R>: values and tangents, the tangents dT bytes after the values).
template <typename R, int NQ, typename E = cx<R>, bool ST = false>
__global__ __launch_bounds__(64) void k_ufill(DevPlan P, const cx<R>* __restrict__ Ai,
                                              const cx<R>* __restrict__ bi, cx<R>* G,
                                              const int* __restrict__ elist, const int* __restrict__ woff,
                                              int wmax, int64_t dT) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  ufill_body<R, NQ, E, ST>(P, Ai, bi, G, elist, woff, wmax, reinterpret_cast<E*>(smem_raw), dT);
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

// Algorithm 2: one workgroup of WV wavefronts per (lattice point, chunk of
// undetected rows).  Chunks of about 112 entries per wavefront over four
// wavefronts leave fewer rows to the halo than one-wavefront chunks (the
// 5-mode conditional forward sweep 2.29 -> 1.78 ms, the 4-mode one 0.45 ->
// 0.40 ms, the 6-mode gradient circuit 4.61 -> 3.75 ms).
// E = dual<R> carries every amplitude's tangent along (forward mode), dT
// bytes after the value.  ST: the rows stream from HBM (blocks whose rows do
// not fit the LDS); the bridge pivot blocks then go to the workgroup's slot
// of `slots` (slot_len entries each).
template <int MD, int NQ, typename R, typename E, bool ST, int WV>
__global__ __launch_bounds__(kBT * WV) void k_fwd_block(DevPlan P, LevelPtrs<R> L, const cx<R>* __restrict__ Ai,
                                                   const cx<R>* __restrict__ bi, int S, int nwork, ChunkGeo G,
                                                   int64_t dT, cx<R>* slots, int64_t slot_len) {
  static_assert(!ST || std::is_same<E, cx<R>>::value, "streamed rows carry values only");
  constexpr int NPOS = NQ + 2 * MD;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int R0 = G.R0;
  E* lf0 = reinterpret_cast<E*>(smem_raw);                                  // (RC + 2) rows
  E* lpk = ST ? reinterpret_cast<E*>(slots + (size_t)blockIdx.x * slot_len)  // MD x (RC + 1) rows
              : lf0 + (size_t)(G.RC + 2) * R0;
  E* sA = ST ? lf0 : lpk + (size_t)MD * (G.RC + 1) * R0;                   // A (NPOS x NPOS) then b (NPOS)
  const E* sb = sA + NPOS * NPOS;
  R* sq = reinterpret_cast<R*>(sA + NPOS * NPOS + NPOS);
  R* isq = sq + (kMaxCut + 4);
  for (int v = threadIdx.x; v < kMaxCut + 4; v += blockDim.x) {
    sq[v] = sqrt(R(v));
    isq[v] = v ? R(1) / sqrt(R(v)) : R(0);
  }
  for (int i = threadIdx.x; i < NPOS * NPOS + NPOS; i += blockDim.x) sA[i] = ET<E>::load(Ai + i, dT);
  // the unit's first unit_sync orders these LDS writes before their reads
  for (int w = blockIdx.x; w < nwork * G.nchunks; w += gridDim.x) {
    const int r = w / G.nchunks, c = w - r * G.nchunks;
    fwd_block_unit<MD, NQ, R, LevelPtrs<R>, E, ST, WV>(P, L, sA, sb, sq, isq, S, r, c, G, lf0, lpk, dT);
    if constexpr (WV > 1) __syncthreads();   // the next unit overwrites the rows
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
template <int MD, int NQ, typename R, typename E, bool ST, int WV>
static void launch_fwd_block_w(size_t shm, int grid, hipStream_t st, const DevPlan& P, const LevelPtrs<R>& L,
                               const cx<R>* A, const cx<R>* b, int S, int nwork, const ChunkGeo& G, int64_t dT,
                               cx<R>* slots, int64_t slot_len) {
  if (shm > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fwd_block<MD, NQ, R, E, ST, WV>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipLaunchKernelGGL((k_fwd_block<MD, NQ, R, E, ST, WV>), dim3(grid), dim3(kBT * WV), shm, st, P, L, A, b, S, nwork,
                     G, dT, slots, slot_len);
}
template <int MD, int NQ, typename R, typename E = cx<R>, bool ST = false>
static void launch_fwd_block_k(size_t shm, int grid, hipStream_t st, const DevPlan& P, const LevelPtrs<R>& L,
                               const cx<R>* A, const cx<R>* b, int S, int nwork, const ChunkGeo& G,
                               int64_t dT = 0, cx<R>* slots = nullptr, int64_t slot_len = 0) {
  // values with rows in LDS: kFwdWaves wavefronts per unit; the streamed
  // rows and the forward mode: one
  if constexpr (std::is_same<E, cx<R>>::value && !ST)
    launch_fwd_block_w<MD, NQ, R, E, ST, kFwdWaves>(shm, grid, st, P, L, A, b, S, nwork, G, dT, slots, slot_len);
  else
    launch_fwd_block_w<MD, NQ, R, E, ST, 1>(shm, grid, st, P, L, A, b, S, nwork, G, dT, slots, slot_len);
}

// The undetected-block fill for the plan's number of block coordinates.
template <typename R>
static hipError_t launch_ufill(const Plan& Pl, const DevPlan& P, const cx<R>* Ai, const cx<R>* bi, cx<R>* f0,
                               hipStream_t st) {
  const size_t shm = ufill_launch_lds_bytes(Pl, false);
  if (shm > kMaxLds) return hipErrorInvalidConfiguration;
  auto* kfn = Pl.st_ufill ? (Pl.nq == 2   ? &k_ufill<R, 2, cx<R>, true>
                             : Pl.nq == 4 ? &k_ufill<R, 4, cx<R>, true>
                                          : &k_ufill<R, 6, cx<R>, true>)
                          : (Pl.nq == 2   ? &k_ufill<R, 2>
                             : Pl.nq == 4 ? &k_ufill<R, 4>
                                          : &k_ufill<R, 6>);
  if (shm > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kfn), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)shm);
  hipLaunchKernelGGL(kfn, dim3(1), dim3(64), shm, st, P, Ai, bi, f0, Pl.d_elist, Pl.d_woff, Pl.wmax, (int64_t)0);
  return hipGetLastError();
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
    // wavefronts in flight; a large level keeps the full height
    const bool stm = Pl.st_fwd;
    ChunkGeo G = stm ? chunk_geo(Pl) : fwd_geo(Pl, nwork);
    if (stm && (int64_t)nwork * G.nchunks < kSmallLevelUnits) G = chunk_geo(Pl, kBT / 2);
    const size_t shm = stm ? fwd_stream_lds_bytes(Pl) : fwd_lds_bytes_for(Pl, G);
    if (shm > kMaxLds) return hipErrorInvalidConfiguration;
    // streamed rows: at most kStreamSlots workgroups, each with its slot after
    // the prep block
    const int grid = stm ? (int)std::min<int64_t>((int64_t)nwork * G.nchunks, kStreamSlots) : nwork * G.nchunks;
    cx<R>* slots = stm ? reinterpret_cast<cx<R>*>(reinterpret_cast<char*>(const_cast<cx<R>*>(A)) + prep_core_bytes(Pl))
                       : nullptr;
    const int64_t slen = (int64_t)fwd_stream_entries(Pl);
#define FD_LAUNCH_BLOCK_NQ(MDV, NQV)                                                                     \
  if (stm)                                                                                               \
    launch_fwd_block_k<MDV, NQV, R, cx<R>, true>(shm, grid, st, P, L, A, b, S, nwork, G, 0, slots, slen); \
  else                                                                                                   \
    launch_fwd_block_k<MDV, NQV, R>(shm, grid, st, P, L, A, b, S, nwork, G);
#define FD_LAUNCH_BLOCK(MDV)        \
  case MDV:                         \
    if (Pl.nq == 2) {               \
      FD_LAUNCH_BLOCK_NQ(MDV, 2)    \
    } else if (Pl.nq == 4) {        \
      FD_LAUNCH_BLOCK_NQ(MDV, 4)    \
    } else {                        \
      FD_LAUNCH_BLOCK_NQ(MDV, 6)    \
    }                               \
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
#undef FD_LAUNCH_BLOCK_NQ
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

hipError_t launch_fwd_level(const Plan& Pl, bool odd, int S, const void* const* rd, void* const* wr,
                            const void* f0cur, void* f0nxt, const void* Ai, const void* bi, hipStream_t st) {
  if (!f0cur || !Ai || !bi) return hipErrorInvalidValue;   // read by every unit
  const DevPlan P = make_devplan(Pl, odd);
  if (Pl.dt == FD_C64) {
    LevelPtrs<float> L;
    std::memset(&L, 0, sizeof(L));
    for (int f = 1; f < Pl.nfam; ++f) {
      L.rd[f] = static_cast<const cx<float>*>(rd[f]);
      L.wr[f] = static_cast<cx<float>*>(wr[f]);
    }
    L.f0cur = static_cast<const cx<float>*>(f0cur);
    L.f0nxt = static_cast<cx<float>*>(f0nxt);
    L.node = Pl.d_node ? Pl.d_node + (size_t)Pl.lvl[S] * kNodeStride : nullptr;
    return launch_fwd_level_t<float>(Pl, P, odd, S, L, Ai, bi, st);
  }
  LevelPtrs<double> L;
  std::memset(&L, 0, sizeof(L));
  for (int f = 1; f < Pl.nfam; ++f) {
    L.rd[f] = static_cast<const cx<double>*>(rd[f]);
    L.wr[f] = static_cast<cx<double>*>(wr[f]);
  }
  L.f0cur = static_cast<const cx<double>*>(f0cur);
  L.f0nxt = static_cast<cx<double>*>(f0nxt);
  L.node = Pl.d_node ? Pl.d_node + (size_t)Pl.lvl[S] * kNodeStride : nullptr;
  return launch_fwd_level_t<double>(Pl, P, odd, S, L, Ai, bi, st);
}

// Copy of one level of every family (checkpoints of a checkpointed sweep):
// family blockIdx.y, n[f] 16-byte (complex128) or 8-byte entries.
struct CopyFams {
  const void* src[kMaxFam];
  void* dst[kMaxFam];
  int64_t n[kMaxFam];
};

template <typename R>
__global__ __launch_bounds__(kThreads) void k_copy_fams(CopyFams a) {
  const int f = blockIdx.y;
  const cx<R>* src = static_cast<const cx<R>*>(a.src[f]);
  cx<R>* dst = static_cast<cx<R>*>(a.dst[f]);
  if (!src) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n[f]; i += (int64_t)gridDim.x * blockDim.x)
    st(dst + i, ld(src + i));
}

hipError_t launch_copy_fams(const Plan& Pl, const void* const* src, void* const* dst, const int64_t* n,
                            hipStream_t st) {
  CopyFams a;
  std::memset(&a, 0, sizeof(a));
  int64_t nmax = 0;
  for (int f = 0; f < Pl.nfam; ++f) {
    a.src[f] = src[f];
    a.dst[f] = dst[f];
    a.n[f] = src[f] ? n[f] : 0;
    nmax = std::max(nmax, a.n[f]);
  }
  if (nmax == 0) return hipSuccess;
  const unsigned gx = (unsigned)std::min<int64_t>((nmax + kThreads - 1) / kThreads, 1024);
  if (Pl.dt == FD_C64)
    hipLaunchKernelGGL((k_copy_fams<float>), dim3(gx, Pl.nfam), dim3(kThreads), 0, st, a);
  else
    hipLaunchKernelGGL((k_copy_fams<double>), dim3(gx, Pl.nfam), dim3(kThreads), 0, st, a);
  return hipGetLastError();
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

// Forward sweep for a checkpointed reverse sweep: F0 at every level goes to
// the saved buffer, the other families run in a two-level ring (the first
// two slots of the segment buffer), and the level just below each segment is
// copied into its checkpoint.
template <typename R>
static hipError_t run_forward_ckpt_t(const Plan& Pl, bool odd, const void* A, const void* b, const void* c,
                                     void* rho, char* ws, char* saved, hipStream_t st) {
  const CkptLayout Lc = ckpt_layout(Pl);
  const SegLayout Sg = seg_layout(Pl);
  const size_t eb = sizeof(cx<R>);
  cx<R>* Ai = reinterpret_cast<cx<R>*>(ws);   // prep block at the start of the workspace
  cx<R>* bi = Ai + (size_t)Pl.npos * Pl.npos;
  cx<R>* f0 = reinterpret_cast<cx<R>*>(saved + Lc.f0);
  const DevPlan P = make_devplan(Pl, odd);
  hipError_t e;
  {
    KTimer kt(Pl, KK_PREP, st);
    e = launch_prep(Pl, A, b, c, Ai, f0, st);
  }
  if (e != hipSuccess) return e;
  if (Pl.B > 1) {
    KTimer kt(Pl, KK_UFILL, st);
    if ((e = launch_ufill<R>(Pl, P, Ai, bi, f0, st)) != hipSuccess) return e;
  }
  const int s = Pl.ckpt, MD = Pl.MD;
  auto used = [&](int f) { return ckpt_keeps_family(Pl, f) && (odd || f >= 1 + 2 * MD); };
  auto slot = [&](int f, int k) {   // ring slot k of family f
    return ws + Sg.fam[f] + (size_t)k * Pl.maxN[Pl.fam_group[f]] * Pl.B * eb;
  };
  for (int S = 0; S <= Pl.smax && MD > 0; ++S) {
    const void* rd[kMaxFam] = {};
    void* wr[kMaxFam] = {};
    for (int f = 1; f < Pl.nfam; ++f) {
      if (!used(f)) continue;
      rd[f] = S > 0 ? slot(f, (S - 1) & 1) : nullptr;
      wr[f] = slot(f, S & 1);
    }
    const cx<R>* f0cur = f0 + (size_t)Pl.lvl[S] * Pl.B;
    cx<R>* f0nxt = S < Pl.smax ? f0 + (size_t)Pl.lvl[S + 1] * Pl.B : nullptr;
    {
      KTimer kt(Pl, KK_FWD_LEVEL, st);
      e = launch_fwd_level(Pl, odd, S, rd, wr, f0cur, f0nxt, Ai, bi, st);
    }
    if (e != hipSuccess) return e;
    if ((S + 1) % s == 0 && S < Pl.smax) {
      // level S is the one below segment (S + 1) / s: keep it
      const int ck = (S + 1) / s - 1;
      const void* src[kMaxFam] = {};
      void* dst[kMaxFam] = {};
      int64_t n[kMaxFam] = {};
      for (int f = 1; f < Pl.nfam; ++f) {
        if (!used(f)) continue;
        src[f] = wr[f];
        dst[f] = saved + Lc.ck[(size_t)ck * Pl.nfam + f];
        n[f] = Pl.ncnt[(size_t)Pl.fam_group[f] * (Pl.smax + 1) + S] * Pl.B;
      }
      if ((e = launch_copy_fams(Pl, src, dst, n, st)) != hipSuccess) return e;
    }
  }
  if (!rho) return hipSuccess;
  return launch_out_perm_t<R>(Pl, P, f0, rho, st);
}

template <typename R>
static hipError_t run_forward_t(const Plan& Pl, bool odd, const void* A, const void* b, const void* c, void* rho,
                                char* ws, char* saved, hipStream_t st, StopRule* stop) {
  if (saved && Pl.ckpt > 0) return run_forward_ckpt_t<R>(Pl, odd, A, b, c, rho, ws, saved, st);
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
  if (store_all && Pl.wcnt) {   // debug write counters over the saved buffer
    P.wcnt = Pl.wcnt;
    P.wbase = saved;
    P.wcnt_n = (int64_t)Pl.wcnt_n;
  }
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
    if ((e = launch_ufill<R>(Pl, P, Ai, bi, f0, st)) != hipSuccess) return e;
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


// ---------------------------------------------------------------------------
// Forward mode of Algorithm 1 (the tangent recurrences of Sec. 2.5, summed
// along one direction (dA, db, dc)): differentiating Eq. recrel gives, for a
// pivot p and write direction i,
//   sqrt(p_i + 1) dG_{p+1_i} = db_i G_p + b_i dG_p
//                              + sum_l sqrt(p_l) (dA_il G_{p-1_l} + A_il dG_{p-1_l}),
// with dG_0 = dc.  The tangents need exactly the reads and writes of the
// values, so every kept amplitude gets its tangent in a second workspace of
// the same layout, dT bytes further on, and one thread carries both.
// ---------------------------------------------------------------------------

template <int MD, typename R>
__global__ __launch_bounds__(kThreads) void k_fwd_point_jvp(DevPlan P, LevelPtrs<R> L, int64_t dT,
                                                            const cx<R>* __restrict__ Ai, const cx<R>* __restrict__ bi,
                                                            const cx<R>* __restrict__ dAi,
                                                            const cx<R>* __restrict__ dbi, int S, int nwork) {
  constexpr int NP = 2 * MD;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* sq = reinterpret_cast<R*>(smem_raw);
  R* isq = sq + (kMaxCut + 4);
  int* spn = reinterpret_cast<int*>(isq + (kMaxCut + 4));
  load_tables(P, spn, sq, isq);
  __syncthreads();
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nwork) return;
  int m[MD], s[MD + 1], rdn[MD], rup[MD];
  unrank<MD>(spn, P.pnw, P.CD, S, r, m, s);
  neighbour_ranks<MD>(spn, P.pnw, s, rdn, rup);
  // value and tangent of a family entry
  auto rd2 = [&](int f, int idx, R w, cx<R>& v, cx<R>& t) {
    v = cscale(ld(at32(L.rd[f], (uint32_t)idx)), w);
    t = cscale(ld(at32(tangent_of(L.rd[f], dT), (uint32_t)idx)), w);
  };
  auto wr2 = [&](cx<R>* dst, const cx<R>& v, const cx<R>& t) {
    st(dst, v);
    st(tangent_of(dst, dT), t);
  };
  const cx<R> g0 = ld(at32(L.f0cur, (uint32_t)r));
  const cx<R> t0 = ld(at32(tangent_of(L.f0cur, dT), (uint32_t)r));
  cx<R> yk[MD], tyk[MD];
#pragma unroll
  for (int K = 0; K < MD; ++K) yk[K] = tyk[K] = czero<R>();

  if (m[0] <= P.CD[0] - 2) {
    // diagonal pivot d(m): reads d(m) - 1_l (type-1 families one level down)
    cx<R> x[NP], tx[NP];
#pragma unroll
    for (int j = 0; j < MD; ++j) {
      if (m[j] > 0) {
        rd2(fam_f1b(MD, j), rdn[j], sq[m[j]], x[2 * j], tx[2 * j]);
        rd2(fam_f1k(j), rdn[j], sq[m[j]], x[2 * j + 1], tx[2 * j + 1]);
      } else {
        x[2 * j] = x[2 * j + 1] = tx[2 * j] = tx[2 * j + 1] = czero<R>();
      }
    }
#pragma unroll
    for (int j = 0; j < MD; ++j) {
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int i = 2 * j + side;
        const cx<R> bv = ld(bi + i), dbv = ld(dbi + i);
        cx<R> acc = czero<R>(), tacc = czero<R>();
        cfma(acc, bv, g0);
        cfma(tacc, dbv, g0);
        cfma(tacc, bv, t0);
#pragma unroll
        for (int l = 0; l < NP; ++l) {
          const cx<R> a = ld(Ai + i * NP + l), da = ld(dAi + i * NP + l);
          cfma(acc, a, x[l]);
          cfma(tacc, da, x[l]);
          cfma(tacc, a, tx[l]);
        }
        acc = cscale(acc, isq[m[j] + 1]);
        tacc = cscale(tacc, isq[m[j] + 1]);
        if (side == 0) {
          yk[j] = acc;
          tyk[j] = tacc;
          if (j == 0 || m[j] <= P.CD[j] - 2) wr2(at32(L.wr[fam_f1k(j)], (uint32_t)r), acc, tacc);
        } else {
          const bool ok = (j == 0) ? (m[0] <= P.CD[0] - 3) : (m[j] <= P.CD[j] - 2);
          if (ok) wr2(at32(L.wr[fam_f1b(MD, j)], (uint32_t)r), acc, tacc);
        }
      }
    }
  }

  int K0 = MD;
#pragma unroll
  for (int d = MD - 1; d >= 0; --d)
    if (m[d] > 0) K0 = d;
#pragma unroll
  for (int K = 0; K < MD; ++K) {
    if (K > K0) break;
    if (m[K] > P.CD[K] - 2) continue;
    // pivot d(m) + 1_ket(K): reads p - 1_l for l >= ket(K)
    cx<R> x[NP], tx[NP];
    x[2 * K] = cscale(g0, sq[m[K] + 1]);
    tx[2 * K] = cscale(t0, sq[m[K] + 1]);
    if (m[K] > 0)
      rd2(fam_f2(MD, K), rdn[K], sq[m[K]], x[2 * K + 1], tx[2 * K + 1]);
    else
      x[2 * K + 1] = tx[2 * K + 1] = czero<R>();
#pragma unroll
    for (int j = K + 1; j < MD; ++j) {
      if (m[j] > 0) {
        rd2(fam_1001(MD, K, j), rdn[j], sq[m[j]], x[2 * j], tx[2 * j]);
        rd2(fam_1010(MD, K, j), rdn[j], sq[m[j]], x[2 * j + 1], tx[2 * j + 1]);
      } else {
        x[2 * j] = x[2 * j + 1] = tx[2 * j] = tx[2 * j + 1] = czero<R>();
      }
    }
#pragma unroll
    for (int i = 2 * K; i < NP; ++i) {
      const int j = i >> 1;
      bool ok;
      R scale;
      cx<R>* dst;
      if (i == 2 * K + 1) {                 // d(m + 1_K): the next level's F0
        ok = L.f0nxt != nullptr;
        scale = isq[m[K] + 1];
        dst = ok ? at32(L.f0nxt, (uint32_t)rup[K]) : nullptr;
      } else if (i == 2 * K) {              // F2(K)(m)
        ok = (m[K] <= P.CD[K] - 3);
        scale = isq[m[K] + 2];
        dst = at32(L.wr[fam_f2(MD, K)], (uint32_t)r);
      } else {                              // F1010(K,j)(m) / F1001(K,j)(m)
        ok = (m[j] <= P.CD[j] - 2);
        scale = isq[m[j] + 1];
        dst = at32(L.wr[(i & 1) ? fam_1001(MD, K, j) : fam_1010(MD, K, j)], (uint32_t)r);
      }
      if (!ok) continue;
      const cx<R> bv = ld(bi + i), dbv = ld(dbi + i);
      cx<R> acc = czero<R>(), tacc = czero<R>();
      cfma(acc, bv, yk[K]);
      cfma(tacc, dbv, yk[K]);
      cfma(tacc, bv, tyk[K]);
#pragma unroll
      for (int l = 2 * K; l < NP; ++l) {
        const cx<R> a = ld(Ai + i * NP + l), da = ld(dAi + i * NP + l);
        cfma(acc, a, x[l]);
        cfma(tacc, da, x[l]);
        cfma(tacc, a, tx[l]);
      }
      wr2(dst, cscale(acc, scale), cscale(tacc, scale));
    }
  }
}

template <typename R>
static hipError_t run_jvp_t(const Plan& Pl, const void* A, const void* b, const void* c, const void* dA,
                            const void* db, const void* dc, void* rho, void* drho, char* ws, int64_t half,
                            hipStream_t st) {
  const FwdLayout Lw = fwd_layout(Pl, true, false, 0);
  char* wt = ws + half;
  cx<R>* Ai = reinterpret_cast<cx<R>*>(ws + Lw.prep);
  cx<R>* bi = Ai + (size_t)Pl.npos * Pl.npos;
  cx<R>* dAi = reinterpret_cast<cx<R>*>(wt + Lw.prep);
  cx<R>* dbi = dAi + (size_t)Pl.npos * Pl.npos;
  cx<R>* f0 = reinterpret_cast<cx<R>*>(ws + Lw.f0);
  cx<R>* tf0 = reinterpret_cast<cx<R>*>(wt + Lw.f0);
  const DevPlan P = make_devplan(Pl, true);
  hipError_t e;
  {
    KTimer kt(Pl, KK_PREP, st);
    if ((e = launch_prep(Pl, A, b, c, Ai, f0, st)) != hipSuccess) return e;
    if ((e = launch_prep(Pl, dA, db, dc, dAi, tf0, st)) != hipSuccess) return e;
  }
  if (Pl.B > 1) {
    // step 1 of Algorithm 2 with tangents
    KTimer kt(Pl, KK_UFILL, st);
    const size_t shm = ufill_jvp_lds_bytes(Pl);
    if (shm > kMaxLds) return hipErrorInvalidConfiguration;   // rejected before the sweep
    auto* kfn = Pl.nq == 2 ? &k_ufill<R, 2, dual<R>> : Pl.nq == 4 ? &k_ufill<R, 4, dual<R>> : &k_ufill<R, 6, dual<R>>;
    if (shm > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kfn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shm);
    hipLaunchKernelGGL(kfn, dim3(1), dim3(64), shm, st, P, Ai, bi, f0, Pl.d_elist, Pl.d_woff, Pl.wmax, half);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const size_t tab = 2 * (kMaxCut + 4) * sizeof(R) + (size_t)(Pl.MD + 1) * (Pl.smax + 3) * sizeof(int);
  for (int S = 0; S <= Pl.smax && Pl.MD > 0; ++S) {
    const int nwork = (int)Pl.ncnt[S];
    if (nwork <= 0) continue;
    LevelPtrs<R> L;
    std::memset(&L, 0, sizeof(L));
    for (int f = 1; f < Pl.nfam; ++f) {
      if (Lw.fam[f] == 0) continue;
      const int g = Pl.fam_group[f];
      L.rd[f] = fam_level_ptr<R>(Pl, ws, Lw.fam[f], g, S - 1, true);
      L.wr[f] = fam_level_ptr<R>(Pl, ws, Lw.fam[f], g, S, true);
    }
    L.f0cur = fam_level_ptr<R>(Pl, ws, Lw.f0, 0, S, false);
    L.f0nxt = S < Pl.smax ? fam_level_ptr<R>(Pl, ws, Lw.f0, 0, S + 1, false) : nullptr;
    KTimer kt(Pl, KK_FWD_LEVEL, st);
    if (Pl.B > 1) {
      L.node = Pl.d_node + (size_t)Pl.lvl[S] * kNodeStride;
      ChunkGeo G = chunk_geo(Pl);
      if ((int64_t)nwork * G.nchunks < kSmallLevelUnits) G = chunk_geo(Pl, kBT / 2);
      const size_t shm = fwd_lds_bytes_for(Pl, G, true);
      if (shm > kMaxLds) return hipErrorInvalidConfiguration;   // rejected before the sweep
      const int grid = nwork * G.nchunks;
#define FD_LAUNCH_BLOCK_JVP(MDV)                                                                          \
  case MDV:                                                                                              \
    if (Pl.nq == 2)                                                                                      \
      launch_fwd_block_k<MDV, 2, R, dual<R>>(shm, grid, st, P, L, Ai, bi, S, nwork, G, half);            \
    else if (Pl.nq == 4)                                                                                 \
      launch_fwd_block_k<MDV, 4, R, dual<R>>(shm, grid, st, P, L, Ai, bi, S, nwork, G, half);            \
    else                                                                                                 \
      launch_fwd_block_k<MDV, 6, R, dual<R>>(shm, grid, st, P, L, Ai, bi, S, nwork, G, half);            \
    break;
      switch (Pl.MD) {
        FD_LAUNCH_BLOCK_JVP(1)
        FD_LAUNCH_BLOCK_JVP(2)
        FD_LAUNCH_BLOCK_JVP(3)
        FD_LAUNCH_BLOCK_JVP(4)
        FD_LAUNCH_BLOCK_JVP(5)
        FD_LAUNCH_BLOCK_JVP(6)
        FD_LAUNCH_BLOCK_JVP(7)
        FD_LAUNCH_BLOCK_JVP(8)
        default:
          return hipErrorInvalidValue;
      }
#undef FD_LAUNCH_BLOCK_JVP
      if ((e = hipGetLastError()) != hipSuccess) return e;
      continue;
    }
    const int grid = (nwork + kThreads - 1) / kThreads;
#define FD_LAUNCH_JVP(MDV)                                                                                        \
  case MDV:                                                                                                       \
    hipLaunchKernelGGL((k_fwd_point_jvp<MDV, R>), dim3(grid), dim3(kThreads), tab, st, P, L, half, Ai, bi, dAi,  \
                       dbi, S, nwork);                                                                            \
    break;
    switch (Pl.MD) {
      FD_LAUNCH_JVP(1)
      FD_LAUNCH_JVP(2)
      FD_LAUNCH_JVP(3)
      FD_LAUNCH_JVP(4)
      FD_LAUNCH_JVP(5)
      FD_LAUNCH_JVP(6)
      FD_LAUNCH_JVP(7)
      FD_LAUNCH_JVP(8)
      default:
        return hipErrorInvalidValue;
    }
#undef FD_LAUNCH_JVP
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = launch_out_perm_t<R>(Pl, P, f0, rho, st)) != hipSuccess) return e;
  return launch_out_perm_t<R>(Pl, P, tf0, drho, st);
}

hipError_t run_jvp(const Plan& Pl, const void* A, const void* b, const void* c, const void* dA, const void* db,
                   const void* dc, void* rho, void* drho, void* ws, hipStream_t st) {
  const int64_t half = (int64_t)jvp_half_bytes(Pl);
  if (Pl.dt == FD_C64) return run_jvp_t<float>(Pl, A, b, c, dA, db, dc, rho, drho, (char*)ws, half, st);
  return run_jvp_t<double>(Pl, A, b, c, dA, db, dc, rho, drho, (char*)ws, half, st);
}

}  // namespace fd
