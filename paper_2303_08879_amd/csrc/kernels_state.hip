// State vectors of pure Gaussian states: psi[n] = <n|psi> for 0 <= n_j < C_j.
//
// The generating function of a pure state has one index per mode (D = M in
// Sec. 2.1), and its scaled Taylor coefficients obey the same recurrence as
// the density matrix's:
//   psi[n] = ( b_i psi[p] + sum_l sqrt(p_l) A_il psi[p - 1_l] ) / sqrt(n_i),
// p = n - 1_i, taken here with i the first mode where n_i > 0.  Targets of
// total photon number S read levels S - 1 and S - 2 only, so the sweep runs
// level by level over the lattice of n (the detected lattice of a plan whose
// modes are all detected: same rank / unrank tables, same level-major
// storage, same output permutation).  With b = 0 the odd levels vanish
// (Sec. 2.4): even levels read level S - 2 alone and odd levels are only
// cleared.
//
// One thread per target; its parent's rank is rdn[i] of the target, its
// parent's own neighbour ranks come from the parent's partial sums (those of
// the target less one up to mode i).
#include <algorithm>
#include <cstring>

#include "fd_device.h"

namespace fd {

struct StateModes {
  int MD;               // kept modes (cutoff >= 2)
  int mode[kMaxD];      // kept mode k -> caller's mode index
};

// A and b of the kept modes into the workspace (MD x MD, then MD), psi at
// the vacuum = c; non-finite inputs set status bit 0, a non-zero b under the
// b = 0 promise status bit 1.
template <typename R>
__global__ __launch_bounds__(64) void k_state_prep(int M, StateModes sm, const cx<R>* __restrict__ A,
                                                   const cx<R>* __restrict__ b, const cx<R>* __restrict__ c,
                                                   cx<R>* __restrict__ Ak, cx<R>* __restrict__ psi0, int check_b_zero,
                                                   int* status) {
  const int MD = sm.MD;
  int bad = 0;
  for (int i = threadIdx.x; i < MD * MD; i += blockDim.x) {
    const cx<R> v = ld(A + (size_t)sm.mode[i / MD] * M + sm.mode[i % MD]);
    if (!isfinite(v.x) || !isfinite(v.y)) bad |= 1;
    st(Ak + i, v);
  }
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    const cx<R> v = ld(b + i);
    if (!isfinite(v.x) || !isfinite(v.y)) bad |= 1;
    if (check_b_zero && (v.x != R(0) || v.y != R(0))) bad |= 2;
  }
  for (int i = threadIdx.x; i < MD; i += blockDim.x) st(Ak + MD * MD + i, ld(b + sm.mode[i]));
  if (threadIdx.x == 0) {
    const cx<R> cv = ld(c);
    if (!isfinite(cv.x) || !isfinite(cv.y)) bad |= 1;
    st(psi0, cv);
  }
  if (bad) atomicOr(status, bad);
}

// Level S of the sweep (S >= 1; S < 0: none) and, when zlevel >= 0, the
// clearing of level zlevel (an odd level under b = 0).  f0 is psi in level
// order; lvl[S] is the first entry of level S.
template <int MD, bool BZ, typename R>
__global__ __launch_bounds__(kThreads) void k_state_level(DevPlan P, const cx<R>* __restrict__ Ak,
                                                          cx<R>* __restrict__ f0, int S, int zlevel) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<R>* sA = reinterpret_cast<cx<R>*>(smem_raw);   // A (MD x MD) then b (MD)
  const cx<R>* sb = sA + MD * MD;
  R* sq = reinterpret_cast<R*>(sA + MD * MD + MD);
  R* isq = sq + (kMaxCut + 4);
  int* spn = reinterpret_cast<int*>(isq + (kMaxCut + 4));
  const int pnw = P.pnw;
  for (int i = threadIdx.x; i < (MD + 1) * pnw; i += blockDim.x) spn[i] = P.pn[i];
  for (int v = threadIdx.x; v < kMaxCut + 4; v += blockDim.x) {
    sq[v] = sqrt(R(v));
    isq[v] = v ? R(1) / sqrt(R(v)) : R(0);
  }
  for (int i = threadIdx.x; i < MD * MD + MD; i += blockDim.x) sA[i] = ld(Ak + i);
  __syncthreads();
  const int stride = gridDim.x * blockDim.x;
  if (zlevel >= 0) {
    cx<R>* z = f0 + P.lvl[zlevel];
    const int nz = (int)(P.lvl[zlevel + 1] - P.lvl[zlevel]);
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nz; r += stride) st(z + r, czero<R>());
  }
  if (S < 1) return;
  cx<R>* cur = f0 + P.lvl[S];
  const cx<R>* lv1 = f0 + P.lvl[S - 1];
  const cx<R>* lv2 = S >= 2 ? f0 + P.lvl[S - 2] : f0;
  const int n = (int)(P.lvl[S + 1] - P.lvl[S]);
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    int m[MD], s[MD + 1], rdn[MD], rup[MD];
    unrank<MD>(spn, pnw, P.CD, S, r, m, s);
    neighbour_ranks<MD>(spn, pnw, s, rdn, rup);
    // first mode with a photon: its index, the parent's rank and n_i
    // (selected with constant indices)
    int i = 0, rp = 0, ni = 1;
    bool found = false;
#pragma unroll
    for (int d = 0; d < MD; ++d)
      if (!found && m[d] > 0) {
        found = true;
        i = d;
        rp = rdn[d];
        ni = m[d];
      }
    // partial sums of the parent p = m - 1_i, then its neighbours at S - 2
    int sp[MD + 1], pdn[MD], pup[MD];
#pragma unroll
    for (int d = 0; d <= MD; ++d) sp[d] = s[d] - (d <= i ? 1 : 0);
    sp[MD] = 0;
    cx<R> acc = czero<R>();
    if (!BZ) cfma(acc, sb[i], ld(lv1 + rp));
    if (S >= 2) {
      neighbour_ranks<MD>(spn, pnw, sp, pdn, pup);
#pragma unroll
      for (int l = 0; l < MD; ++l) {
        const int pl = m[l] - (l == i ? 1 : 0);
        if (pl > 0) cfma(acc, sA[i * MD + l], cscale(ld(lv2 + pdn[l]), sq[pl]));
      }
    }
    st(cur + r, cscale(acc, isq[ni]));
  }
}

size_t state_ws_bytes(const Plan& Pl) {
  const size_t eb = elem_bytes(Pl.dt);
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  return al((size_t)Pl.nodes_total * eb) + al((size_t)(Pl.MD * Pl.MD + Pl.MD) * eb);
}

template <typename R>
static hipError_t run_state_fwd_t(const Plan& Pl, bool bz, const void* A, const void* b, const void* c, void* psi,
                                  void* ws, hipStream_t st) {
  const size_t eb = sizeof(cx<R>);
  cx<R>* f0 = static_cast<cx<R>*>(ws);
  cx<R>* Ak = reinterpret_cast<cx<R>*>(static_cast<char*>(ws) + (((size_t)Pl.nodes_total * eb + 255) & ~size_t(255)));
  StateModes sm;
  std::memset(&sm, 0, sizeof(sm));
  sm.MD = Pl.MD;
  for (int k = 0; k < Pl.MD; ++k) sm.mode[k] = Pl.dmodes[k];
  {
    KTimer kt(Pl, KK_PREP, st);
    hipLaunchKernelGGL((k_state_prep<R>), dim3(1), dim3(64), 0, st, Pl.M, sm, static_cast<const cx<R>*>(A),
                       static_cast<const cx<R>*>(b), static_cast<const cx<R>*>(c), Ak, f0, bz ? 1 : 0,
                       Pl.d_status);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const DevPlan P = make_devplan(Pl, !bz);
  const size_t shm = (size_t)(Pl.MD * Pl.MD + Pl.MD) * eb + 2 * (kMaxCut + 4) * sizeof(R) +
                     (size_t)(Pl.MD + 1) * (Pl.smax + 3) * sizeof(int);
  auto count = [&](int S) { return S >= 0 && S <= Pl.smax ? Pl.lvl[S + 1] - Pl.lvl[S] : int64_t(0); };
  auto launch = [&](int S, int zl) -> hipError_t {
    const int64_t work = std::max(count(S), count(zl));
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + kThreads - 1) / kThreads, 65536));
    KTimer kt(Pl, KK_FWD_LEVEL, st);
#define FD_STATE_LEVEL(MDV)                                                                                \
  case MDV:                                                                                                \
    if (bz)                                                                                                \
      hipLaunchKernelGGL((k_state_level<MDV, true, R>), dim3(grid), dim3(kThreads), shm, st, P, Ak, f0, S, zl); \
    else                                                                                                   \
      hipLaunchKernelGGL((k_state_level<MDV, false, R>), dim3(grid), dim3(kThreads), shm, st, P, Ak, f0, S, zl); \
    break;
    switch (Pl.MD) {
      FD_STATE_LEVEL(1)
      FD_STATE_LEVEL(2)
      FD_STATE_LEVEL(3)
      FD_STATE_LEVEL(4)
      FD_STATE_LEVEL(5)
      FD_STATE_LEVEL(6)
      FD_STATE_LEVEL(7)
      FD_STATE_LEVEL(8)
      default: return hipErrorInvalidValue;
    }
#undef FD_STATE_LEVEL
    return hipGetLastError();
  };
  for (int S = 1; S <= Pl.smax && Pl.MD > 0; ++S) {
    if (bz && (S & 1)) continue;   // odd level: cleared with the next even one
    if ((e = launch(S, bz ? S - 1 : -1)) != hipSuccess) return e;
  }
  if (bz && Pl.MD > 0 && (Pl.smax & 1))
    if ((e = launch(-1, Pl.smax)) != hipSuccess) return e;
  return launch_out_perm(Pl, f0, psi, st);
}

hipError_t run_state_fwd(const Plan& Pl, bool b_zero, const void* A, const void* b, const void* c, void* psi, void* ws,
                         hipStream_t st) {
  if (Pl.dt == FD_C64) return run_state_fwd_t<float>(Pl, b_zero, A, b, c, psi, ws, st);
  return run_state_fwd_t<double>(Pl, b_zero, A, b, c, psi, ws, st);
}

}  // namespace fd
