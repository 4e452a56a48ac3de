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
#include <vector>

#include "fd_device.h"

namespace fd {

struct StateModes {
  int MD;               // kept modes (cutoff >= 2)
  int mode[kMaxD];      // kept mode k -> caller's mode index
};

// A (symmetrised, (A + A^T)/2, as for density matrices) and b of the kept
// modes into the workspace (MD x MD, then MD), psi at the vacuum = c;
// non-finite inputs set status bit 0, a non-zero b under the b = 0 promise
// status bit 1.
template <typename R>
__global__ __launch_bounds__(64) void k_state_prep(int M, StateModes sm, const cx<R>* __restrict__ A,
                                                   const cx<R>* __restrict__ b, const cx<R>* __restrict__ c,
                                                   cx<R>* __restrict__ Ak, cx<R>* __restrict__ psi0, int check_b_zero,
                                                   int* status) {
  const int MD = sm.MD;
  int bad = 0;
  for (int i = threadIdx.x; i < MD * MD; i += blockDim.x) {
    const cx<R> v = ld(A + (size_t)sm.mode[i / MD] * M + sm.mode[i % MD]);
    const cx<R> w = ld(A + (size_t)sm.mode[i % MD] * M + sm.mode[i / MD]);
    if (!isfinite(v.x) || !isfinite(v.y)) bad |= 1;
    st(Ak + i, cmake<R>(R(0.5) * (v.x + w.x), R(0.5) * (v.y + w.y)));
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

// ---------------------------------------------------------------------------
// Derivatives.  The local gradients of Sec. 2.5 (the solutions of its tangent
// recurrences for b and A) have closed forms in the amplitudes:
//   d psi_k / d b_i   = sqrt(k_i) psi_{k - 1_i},
//   d psi_k / d A_il  = 1/2 sqrt(k_i (k_l - [i = l])) psi_{k - 1_i - 1_l},
//   d psi_k / d c     = psi_k / c,
// and every shifted amplitude lies inside the box.  Reverse mode: the
// cotangents bbar_i = sum_k g_k conj(d psi_k / d b_i) (g = dL/dpsi^*, Eqs.
// dL_dB, dL_dA) are weighted dot products of g with shifted copies of psi.
// Forward mode: the tangent along (dA, db, dc) is
//   dpsi_k = (dc / c) psi_k + sum_i db_i sqrt(k_i) psi_{k-1_i}
//          + sum_{i <= l} S_il w_il(k) psi_{k-1_i-1_l},
// S_il = dA_il + dA_li (i < l), dA_ii (i = l), w_il the weight above: the
// directional derivative for the symmetric part of dA, as A enters through
// (A + A^T)/2.
//
// Both kernels walk psi (C order, last kept mode fastest) by tiles: the
// trailing modes sp..MD-1 span a tile of T = prod_{d >= sp} C_d entries (at
// most the kernel's tile size) and the leading modes number the tiles, so entry x is
// entry x mod T of tile x / T.  A shifted amplitude of a tile-t entry lies in
// tile t (every mode of the shift trailing), in tile t - 1_i (one leading
// mode i) or in tile t - 1_i - 1_l (two leading modes).  A workgroup stages
// tile t in LDS and serves the terms of the first kind from it, then stages
// tile t - 1_i for each leading i with k_i >= 1 and serves the terms whose
// leading part is 1_i, reading the one amplitude of each two-leading-mode
// term straight from memory.  Each psi entry is so read 1 + (leading modes)
// + (leading pairs) times instead of once per term, and the tile order keeps
// those re-reads in cache: workgroup v runs on XCD v mod 8 and visits tile
// (v mod 8) * ntiles/8 + v / 8, so every XCD walks one contiguous range of
// tiles in order and finds tiles t - 1_i of the faster leading modes in its
// own L2.
// ---------------------------------------------------------------------------
// Tile geometry of each kernel (entries per tile, entries per lane, lanes per
// workgroup): the forward mode stages 64 KB tiles in sixteen-wavefront
// workgroups, the reverse mode 8 KB tiles in one-wavefront workgroups (the faster of the two shapes for each on the 8-mode cutoff-8
// state).
constexpr int kJvpTile = 4096, kJvpEPT = 4, kJvpThreads = kJvpTile / kJvpEPT;
constexpr int kVjpTile = 512, kVjpEPT = 8, kVjpThreads = kVjpTile / kVjpEPT;
constexpr int kVjpGrid = kVjpSlots;   // reverse-mode workgroups at most (one reduction slot each)
constexpr int kVjpCols = kMaxD + kMaxD * (kMaxD + 1) / 2 + 1;   // bbar, Abar (i <= l), c

struct StateTiles {
  int MD, sp, T, ntiles;
  int C[kMaxD], stride[kMaxD];   // kept cutoffs, C-order strides
  double inv_stride[kMaxD], inv_c[kMaxD];
};

static StateTiles state_tiles(const Plan& Pl, int max_tile) {
  StateTiles G;
  std::memset(&G, 0, sizeof(G));
  G.MD = Pl.MD;
  int64_t s = 1;
  for (int d = Pl.MD - 1; d >= 0; --d) {
    G.C[d] = Pl.CD[d];
    G.stride[d] = (int)s;
    G.inv_stride[d] = 1.0 / (double)s;
    G.inv_c[d] = 1.0 / (double)Pl.CD[d];
    s *= Pl.CD[d];
  }
  G.sp = Pl.MD;
  G.T = 1;
  while (G.sp > 0 && G.T * Pl.CD[G.sp - 1] <= max_tile) G.T *= Pl.CD[--G.sp];
  G.ntiles = (int)(s / G.T);
  return G;
}

// Digit (x / stride) mod C of a C-order index x < 2^31: (x + 1/2) / stride
// lies at least 1 / (2 stride) from an integer and the rounded product is off
// by less than (x / stride) 2^-51, so truncation is exact (and so for the mod).
__device__ __forceinline__ int cdigit(int x, int stride, int c, double inv_stride, double inv_c) {
  const int q = (int)((x + 0.5) * inv_stride);
  return q - c * (int)((q + 0.5) * inv_c);
}

// The tile of visit v (see above); in order when the tiles do not split into
// eight equal ranges.
__device__ __forceinline__ int state_tile_of(int ntiles, int v) {
  return (ntiles & 7) ? v : (v & 7) * (ntiles >> 3) + (v >> 3);
}

// Loads tile entries [src, src + T) of this lane (entry f = lane + e * lanes)
// into registers, every load issued before the first is waited on.
template <int NT, int EPT, typename R>
__device__ __forceinline__ void load_lane_entries(cx<R> (&v)[EPT], const cx<R>* __restrict__ src, int T) {
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int f = threadIdx.x + e * NT;
    v[e] = f < T ? ld(src + f) : czero<R>();
  }
}

// Stages tile entries [src, src + T) in LDS (loads first, then the writes).
template <int NT, int EPT, typename R>
__device__ __forceinline__ void stage_tile(cx<R>* buf, const cx<R>* __restrict__ src, int T) {
  cx<R> v[EPT];
  load_lane_entries<NT, EPT>(v, src, T);
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int f = threadIdx.x + e * NT;
    if (f < T) buf[f] = v[e];
  }
}

// acc += (w s) p for a double coefficient s and an amplitude p.
template <typename R>
__device__ __forceinline__ void cmac_w(double& ax, double& ay, double w, double2 s, const cx<R>& p) {
  const double sx = w * s.x, sy = w * s.y;
  ax += sx * (double)p.x - sy * (double)p.y;
  ay += sx * (double)p.y + sy * (double)p.x;
}

template <typename R>
size_t state_jvp_lds_bytes() {
  return (size_t)kJvpTile * sizeof(cx<R>) + (kMaxD * kMaxD + kMaxD) * sizeof(double2) +
         (kMaxCut + 1) * sizeof(double) + kMaxD * sizeof(int);
}

// Forward mode: one workgroup per tile, kJvpEPT entries per lane, the
// tangent accumulated in registers over the tile's phases; the modes are a
// template argument, so the term loops unroll with the strides in scalar
// registers.
template <int MD, typename R>
__global__ __launch_bounds__(kJvpThreads) void k_state_jvp(
    StateTiles G, StateModes sm, int M, const cx<R>* __restrict__ psi, const cx<R>* __restrict__ c,
    const cx<R>* __restrict__ tA, const cx<R>* __restrict__ tb, const cx<R>* __restrict__ tc,
    cx<R>* __restrict__ dpsi) {
  constexpr int MDA = MD > 0 ? MD : 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
  double2* sS = reinterpret_cast<double2*>(smem_raw + (size_t)kJvpTile * sizeof(cx<R>));   // kMaxD x kMaxD
  double2* sB = sS + kMaxD * kMaxD;
  double* sq = reinterpret_cast<double*>(sB + kMaxD);   // sqrt(0..kMaxCut)
  int* ks = reinterpret_cast<int*>(sq + kMaxCut + 1);  // leading digits of the tile
  const int sp = G.sp, T = G.T;
  for (int v = threadIdx.x; v <= kMaxCut; v += kJvpThreads) sq[v] = sqrt((double)v);
  for (int e = threadIdx.x; e < MD * MD; e += kJvpThreads) {
    const int i = e / MD, l = e % MD;
    const cx<R> a = ld(tA + (size_t)sm.mode[i] * M + sm.mode[l]);
    const cx<R> t = ld(tA + (size_t)sm.mode[l] * M + sm.mode[i]);
    sS[i * kMaxD + l] = i == l ? make_double2(a.x, a.y) : make_double2((double)a.x + t.x, (double)a.y + t.y);
  }
  for (int i = threadIdx.x; i < MD; i += kJvpThreads) {
    const cx<R> v = ld(tb + sm.mode[i]);
    sB[i] = make_double2(v.x, v.y);
  }
  const int x0 = state_tile_of(G.ntiles, blockIdx.x) * T;
  for (int d = threadIdx.x; d < sp; d += kJvpThreads)
    ks[d] = cdigit(x0, G.stride[d], G.C[d], G.inv_stride[d], G.inv_c[d]);
  stage_tile<kJvpThreads, kJvpEPT>(buf, psi + x0, T);
  __syncthreads();
  // dc / c
  const cx<R> cv = ld(c), dv = ld(tc);
  const double n2 = (double)cv.x * cv.x + (double)cv.y * cv.y;
  const double2 r = make_double2(((double)dv.x * cv.x + (double)dv.y * cv.y) / n2,
                                 ((double)dv.y * cv.x - (double)dv.x * cv.y) / n2);
  double ax[kJvpEPT], ay[kJvpEPT];
  // terms inside tile t: dc/c, db_i and the pairs of trailing modes
#pragma unroll
  for (int e = 0; e < kJvpEPT; ++e) {
    const int f = threadIdx.x + e * kJvpThreads;
    ax[e] = 0.0;
    ay[e] = 0.0;
    if (f >= T) continue;
    int k[MDA];
#pragma unroll
    for (int d = 0; d < MD; ++d) k[d] = d >= sp ? cdigit(f, G.stride[d], G.C[d], G.inv_stride[d], G.inv_c[d]) : 0;
    double x = 0.0, y = 0.0;
    cmac_w(x, y, 1.0, r, buf[f]);
#pragma unroll
    for (int i = 0; i < MD; ++i) {
      if (i < sp || k[i] < 1) continue;
      const int fi = f - G.stride[i];
      const double wi = sq[k[i]];
      cmac_w(x, y, wi, sB[i], buf[fi]);
#pragma unroll
      for (int l = i; l < MD; ++l) {
        const int kl = k[l] - (l == i ? 1 : 0);
        if (kl < 1) continue;
        cmac_w(x, y, 0.5 * wi * sq[kl], sS[i * kMaxD + l], buf[fi - G.stride[l]]);
      }
    }
    ax[e] = x;
    ay[e] = y;
  }
  // terms whose leading part is 1_i: tile t - 1_i (uniform over the workgroup)
#pragma unroll
  for (int i = 0; i < MD; ++i) {
    if (i >= sp) continue;
    const int ki = ks[i];
    if (ki < 1) continue;
    const int xs = x0 - G.stride[i];
    __syncthreads();
    stage_tile<kJvpThreads, kJvpEPT>(buf, psi + xs, T);
    __syncthreads();
    const double wi = sq[ki];
#pragma unroll
    for (int e = 0; e < kJvpEPT; ++e) {
      const int f = threadIdx.x + e * kJvpThreads;
      if (f >= T) continue;
      int k[MDA];
#pragma unroll
      for (int d = 0; d < MD; ++d) k[d] = d >= sp ? cdigit(f, G.stride[d], G.C[d], G.inv_stride[d], G.inv_c[d]) : 0;
      double x = ax[e], y = ay[e];
      cmac_w(x, y, wi, sB[i], buf[f]);
#pragma unroll
      for (int l = i + 1; l < MD; ++l) {
        if (l < sp || k[l] < 1) continue;
        cmac_w(x, y, 0.5 * wi * sq[k[l]], sS[i * kMaxD + l], buf[f - G.stride[l]]);
      }
      ax[e] = x;
      ay[e] = y;
    }
    // two leading modes: one amplitude per entry from memory
#pragma unroll
    for (int l = i; l < MD; ++l) {
      if (l >= sp) continue;
      const int kl = ks[l] - (l == i ? 1 : 0);
      if (kl < 1) continue;
      cx<R> p[kJvpEPT];
      load_lane_entries<kJvpThreads, kJvpEPT>(p, psi + (xs - G.stride[l]), T);
      const double w = 0.5 * wi * sq[kl];
      const double2 sc = sS[i * kMaxD + l];
#pragma unroll
      for (int e = 0; e < kJvpEPT; ++e) cmac_w(ax[e], ay[e], w, sc, p[e]);
    }
  }
#pragma unroll
  for (int e = 0; e < kJvpEPT; ++e) {
    const int f = threadIdx.x + e * kJvpThreads;
    if (f < T) st(dpsi + x0 + f, cmake<R>((R)ax[e], (R)ay[e]));
  }
}

// Column of each cotangent: bbar_i (i), Abar_il for i <= l (MD + the upper
// triangle row by row), sum g conj(psi) (last).
__host__ __device__ __forceinline__ int vjp_col_pair(int MD, int i, int l) { return MD + i * MD - i * (i - 1) / 2 + (l - i); }

template <typename R>
size_t state_vjp_lds_bytes() {
  return (size_t)kVjpTile * sizeof(cx<R>) + (size_t)(kVjpThreads / 64) * kVjpCols * sizeof(double2) +
         (kMaxCut + 1) * sizeof(double) + 2 * kMaxD * sizeof(int);
}

// Adds the wavefront's sum of (sx, sy) to *dst (a fixed butterfly, lane 0
// writes: bitwise reproducible).
__device__ __forceinline__ void wave_sum_into(double2* dst, double sx, double sy) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sx += __shfl_xor(sx, o);
    sy += __shfl_xor(sy, o);
  }
  if ((threadIdx.x & 63) == 0) {
    dst->x += sx;
    dst->y += sy;
  }
  // one term at a time: the scheduler keeps the next term's LDS reads behind
  // this one (interleaving them only raises the register count)
  __builtin_amdgcn_sched_barrier(0);
}

// sum over e of g_e conj(w_e p_e)
template <typename R>
__device__ __forceinline__ void dot_acc(double& sx, double& sy, double w, double gx, double gy, const cx<R>& p) {
  const double px = w * (double)p.x, py = w * (double)p.y;
  sx += gx * px + gy * py;
  sy += gy * px - gx * py;
}

// Reverse mode: workgroup w visits tiles w, w + grid, ... (grid a multiple of
// 8, so every visit of a workgroup stays on its XCD's range), each lane
// holding the cotangent of its kVjpEPT entries; per term the lanes sum
// their entries in order, each wavefront folds its lanes into its own LDS
// row, and at the end the workgroup adds its wavefront rows in order into
// slot (workgroup, column); the final kernel adds the slots of a column in
// order (bitwise reproducible).  Terms are walked by runtime loops over the
// modes, one term at a time (unrolled over the modes, the per-entry weights
// of every mode stay live and the register count grows with the modes).
template <typename R>
__global__ __launch_bounds__(kVjpThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_state_vjp(StateTiles G, const cx<R>* psi,
                                                             const cx<R>* __restrict__ g, double2* __restrict__ slots) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<R>* buf = reinterpret_cast<cx<R>*>(smem_raw);
  double2* red = reinterpret_cast<double2*>(smem_raw + (size_t)kVjpTile * sizeof(cx<R>));   // waves x kVjpCols
  double* sq = reinterpret_cast<double*>(red + (kVjpThreads / 64) * kVjpCols);
  int* ks = reinterpret_cast<int*>(sq + kMaxCut + 1);   // leading digits of the tile
  int* sst = ks + kMaxD;                                  // C-order strides
  const int MD = G.MD, sp = G.sp, T = G.T;
  const int ncol = MD + MD * (MD + 1) / 2 + 1;
  for (int v = threadIdx.x; v <= kMaxCut; v += kVjpThreads) sq[v] = sqrt((double)v);
  for (int p = threadIdx.x; p < (kVjpThreads / 64) * kVjpCols; p += kVjpThreads) red[p] = make_double2(0.0, 0.0);
  if (threadIdx.x < kMaxD) sst[threadIdx.x] = G.stride[threadIdx.x];
  double2* wred = red + (threadIdx.x >> 6) * kVjpCols;
  // trailing digits of this lane's tile entries (the same in every tile), 6
  // bits per mode; an entry beyond the tile gets digit 0 everywhere, which
  // zeroes every shifted term
  uint64_t kp[kVjpEPT];
#pragma unroll
  for (int e = 0; e < kVjpEPT; ++e) {
    const int f = threadIdx.x + e * kVjpThreads;
    uint64_t p = 0;
#pragma unroll
    for (int d = 0; d < kMaxD; ++d)
      if (f < T && d >= sp && d < MD)
        p |= (uint64_t)cdigit(f, G.stride[d], G.C[d], G.inv_stride[d], G.inv_c[d]) << (6 * d);
    kp[e] = p;
  }
  auto digit = [](uint64_t p, int d) { return (int)((p >> (6 * d)) & 63); };
  for (int v = blockIdx.x; v < G.ntiles; v += gridDim.x) {
    const int x0 = state_tile_of(G.ntiles, v) * T;
    __syncthreads();   // the previous tile's LDS reads are done
    if (threadIdx.x < sp) ks[threadIdx.x] = cdigit(x0, G.stride[threadIdx.x], G.C[threadIdx.x],
                                                   G.inv_stride[threadIdx.x], G.inv_c[threadIdx.x]);
    cx<R> gv[kVjpEPT];
    load_lane_entries<kVjpThreads, kVjpEPT>(gv, g + x0, T);
    stage_tile<kVjpThreads, kVjpEPT>(buf, psi + x0, T);
    double gx[kVjpEPT], gy[kVjpEPT];
#pragma unroll
    for (int e = 0; e < kVjpEPT; ++e) {
      gx[e] = (double)gv[e].x;
      gy[e] = (double)gv[e].y;
    }
    __syncthreads();
    // terms inside tile t
    {
      double sx = 0.0, sy = 0.0;
#pragma unroll
      for (int e = 0; e < kVjpEPT; ++e) {
        const int f = threadIdx.x + e * kVjpThreads;
        if (f < T) dot_acc(sx, sy, 1.0, gx[e], gy[e], buf[f]);
      }
      wave_sum_into(wred + ncol - 1, sx, sy);
    }
#pragma unroll 1
    for (int i = sp; i < MD; ++i) {
      const int si = sst[i];
      {
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int e = 0; e < kVjpEPT; ++e) {
          const int f = threadIdx.x + e * kVjpThreads;
          const int ki = digit(kp[e], i);
          if (ki >= 1) dot_acc(sx, sy, sq[ki], gx[e], gy[e], buf[f - si]);
        }
        wave_sum_into(wred + i, sx, sy);
      }
#pragma unroll 1
      for (int l = i; l < MD; ++l) {
        const int sil = si + sst[l];
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int e = 0; e < kVjpEPT; ++e) {
          const int f = threadIdx.x + e * kVjpThreads;
          const int ki = digit(kp[e], i), kl = digit(kp[e], l) - (l == i ? 1 : 0);
          if (ki >= 1 && kl >= 1) dot_acc(sx, sy, 0.5 * sq[ki] * sq[kl], gx[e], gy[e], buf[f - sil]);
        }
        wave_sum_into(wred + vjp_col_pair(MD, i, l), sx, sy);
      }
    }
    // terms whose leading part is 1_i: tile t - 1_i
#pragma unroll 1
    for (int i = 0; i < sp; ++i) {
      const int ki = ks[i];
      if (ki < 1) continue;   // uniform
      const int xs = x0 - sst[i];
      __syncthreads();
      stage_tile<kVjpThreads, kVjpEPT>(buf, psi + xs, T);
      __syncthreads();
      const double wi = sq[ki];
      {
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int e = 0; e < kVjpEPT; ++e) {
          const int f = threadIdx.x + e * kVjpThreads;
          if (f < T) dot_acc(sx, sy, wi, gx[e], gy[e], buf[f]);
        }
        wave_sum_into(wred + i, sx, sy);
      }
#pragma unroll 1
      for (int l = sp; l < MD; ++l) {
        const int sl = sst[l];
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int e = 0; e < kVjpEPT; ++e) {
          const int f = threadIdx.x + e * kVjpThreads;
          const int kl = digit(kp[e], l);
          if (kl >= 1) dot_acc(sx, sy, 0.5 * wi * sq[kl], gx[e], gy[e], buf[f - sl]);
        }
        wave_sum_into(wred + vjp_col_pair(MD, i, l), sx, sy);
      }
      // two leading modes: one amplitude per entry from memory
#pragma unroll 1
      for (int l = i; l < sp; ++l) {
        const int kl = ks[l] - (l == i ? 1 : 0);
        if (kl < 1) continue;   // uniform
        cx<R> p[kVjpEPT];
        load_lane_entries<kVjpThreads, kVjpEPT>(p, psi + (xs - sst[l]), T);
        const double w = 0.5 * wi * sq[kl];
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int e = 0; e < kVjpEPT; ++e) dot_acc(sx, sy, w, gx[e], gy[e], p[e]);
        wave_sum_into(wred + vjp_col_pair(MD, i, l), sx, sy);
      }
    }
  }
  __syncthreads();
  for (int p = threadIdx.x; p < ncol; p += kVjpThreads) {
    double sx = 0.0, sy = 0.0;
    for (int wv = 0; wv < kVjpThreads / 64; ++wv) {
      sx += red[wv * kVjpCols + p].x;
      sy += red[wv * kVjpCols + p].y;
    }
    slots[(size_t)blockIdx.x * ncol + p] = make_double2(sx, sy);
  }
}

// One workgroup per caller entry of dA (M x M), db (M), dc: the slots of its
// column added in order (zero for modes with cutoff 1), Abar mirrored.
struct StateVjpMap {
  int M, MD, ncol, nslots;
  int mode[kMaxD];
};

template <typename R>
__global__ __launch_bounds__(kThreads) void k_state_vjp_final(StateVjpMap m, const double2* __restrict__ slots,
                                                              const cx<R>* __restrict__ c, cx<R>* dA, cx<R>* db,
                                                              cx<R>* dc) {
  __shared__ double2 red[kThreads];
  const int e = blockIdx.x, M = m.M, MD = m.MD;
  int col = -1;
  if (e < M * M) {
    int ki = -1, kl = -1;
    for (int d = 0; d < MD; ++d) {
      if (m.mode[d] == e / M) ki = d;
      if (m.mode[d] == e % M) kl = d;
    }
    if (ki >= 0 && kl >= 0) {
      const int a = min(ki, kl), bb = max(ki, kl);
      col = MD + a * MD - a * (a - 1) / 2 + (bb - a);   // columns: bbar (MD), then the upper triangle row by row
    }
  } else if (e < M * M + M) {
    for (int d = 0; d < MD; ++d)
      if (m.mode[d] == e - M * M) col = d;
  } else {
    col = m.ncol - 1;
  }
  double sx = 0.0, sy = 0.0;
  if (col >= 0)
    for (int s = threadIdx.x; s < m.nslots; s += blockDim.x) {
      sx += slots[(size_t)s * m.ncol + col].x;
      sy += slots[(size_t)s * m.ncol + col].y;
    }
  red[threadIdx.x] = make_double2(sx, sy);
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[threadIdx.x].x += red[threadIdx.x + w].x;
      red[threadIdx.x].y += red[threadIdx.x + w].y;
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  double2 t = red[0];
  if (e < M * M) {
    st(dA + e, cmake<R>((R)t.x, (R)t.y));
  } else if (e < M * M + M) {
    st(db + (e - M * M), cmake<R>((R)t.x, (R)t.y));
  } else {
    // cbar = sum g conj(psi / c) = (sum g conj(psi)) / conj(c)
    const cx<R> cv = ld(c);
    const double cr = (double)cv.x, ci = (double)cv.y, n2 = cr * cr + ci * ci;
    st(dc, cmake<R>((R)((t.x * cr - t.y * ci) / n2), (R)((t.y * cr + t.x * ci) / n2)));
  }
}

template <int MD, typename R>
static void launch_state_jvp(const StateTiles& G, const StateModes& sm, int M, const void* psi, const void* c,
                             const void* dA, const void* db, const void* dc, void* dpsi, hipStream_t st) {
  const size_t shm = state_jvp_lds_bytes<R>();
  if (shm > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_state_jvp<MD, R>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipLaunchKernelGGL((k_state_jvp<MD, R>), dim3((unsigned)G.ntiles), dim3(kJvpThreads), shm, st, G, sm, M,
                     static_cast<const cx<R>*>(psi), static_cast<const cx<R>*>(c), static_cast<const cx<R>*>(dA),
                     static_cast<const cx<R>*>(db), static_cast<const cx<R>*>(dc), static_cast<cx<R>*>(dpsi));
}

template <typename R>
static hipError_t launch_state_jvp_md(const StateTiles& G, const StateModes& sm, int M, const void* psi,
                                      const void* c, const void* dA, const void* db, const void* dc, void* dpsi,
                                      hipStream_t st) {
  switch (G.MD) {
    case 0: launch_state_jvp<0, R>(G, sm, M, psi, c, dA, db, dc, dpsi, st); break;
    case 1: launch_state_jvp<1, R>(G, sm, M, psi, c, dA, db, dc, dpsi, st); break;
    case 2: launch_state_jvp<2, R>(G, sm, M, psi, c, dA, db, dc, dpsi, st); break;
    case 3: launch_state_jvp<3, R>(G, sm, M, psi, c, dA, db, dc, dpsi, st); break;
    case 4: launch_state_jvp<4, R>(G, sm, M, psi, c, dA, db, dc, dpsi, st); break;
    case 5: launch_state_jvp<5, R>(G, sm, M, psi, c, dA, db, dc, dpsi, st); break;
    case 6: launch_state_jvp<6, R>(G, sm, M, psi, c, dA, db, dc, dpsi, st); break;
    case 7: launch_state_jvp<7, R>(G, sm, M, psi, c, dA, db, dc, dpsi, st); break;
    case 8: launch_state_jvp<8, R>(G, sm, M, psi, c, dA, db, dc, dpsi, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t run_state_jvp(const Plan& Pl, const void* c, const void* psi, const void* dA, const void* db, const void* dc,
                         void* dpsi, hipStream_t st) {
  StateModes sm;
  std::memset(&sm, 0, sizeof(sm));
  sm.MD = Pl.MD;
  for (int k = 0; k < Pl.MD; ++k) sm.mode[k] = Pl.dmodes[k];
  const StateTiles G = state_tiles(Pl, kJvpTile);
  KTimer kt(Pl, KK_FWD_LEVEL, st);
  if (Pl.dt == FD_C64) return launch_state_jvp_md<float>(G, sm, Pl.M, psi, c, dA, db, dc, dpsi, st);
  return launch_state_jvp_md<double>(G, sm, Pl.M, psi, c, dA, db, dc, dpsi, st);
}

template <typename R>
static hipError_t run_state_vjp_t(const Plan& Pl, const void* c, const void* psi, const void* g, void* dA, void* db,
                                  void* dc, void* ws, hipStream_t st) {
  const int MD = Pl.MD, ncol = MD + MD * (MD + 1) / 2 + 1;
  double2* slots = static_cast<double2*>(ws);
  const StateTiles G = state_tiles(Pl, kVjpTile);
  // at most kVjpGrid <= kVjpSlots workgroups (a multiple of 8), one slot each
  static_assert(kVjpGrid <= kVjpSlots && kVjpGrid % 8 == 0, "reduction slots");
  const int grid = std::min(G.ntiles, kVjpGrid);
  {
    KTimer kt(Pl, KK_VJP_LEVEL, st);
    const size_t shm = state_vjp_lds_bytes<R>();
    hipLaunchKernelGGL((k_state_vjp<R>), dim3((unsigned)grid), dim3(kVjpThreads), shm, st, G,
                       static_cast<const cx<R>*>(psi), static_cast<const cx<R>*>(g), slots);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  StateVjpMap m;
  std::memset(&m, 0, sizeof(m));
  m.M = Pl.M;
  m.MD = MD;
  m.ncol = ncol;
  m.nslots = grid;
  for (int d = 0; d < MD; ++d) m.mode[d] = Pl.dmodes[d];
  KTimer kt(Pl, KK_VJP_FINAL, st);
  hipLaunchKernelGGL((k_state_vjp_final<R>), dim3(Pl.M * Pl.M + Pl.M + 1), dim3(kThreads), 0, st, m, slots,
                     static_cast<const cx<R>*>(c), static_cast<cx<R>*>(dA), static_cast<cx<R>*>(db),
                     static_cast<cx<R>*>(dc));
  return hipGetLastError();
}

hipError_t run_state_vjp(const Plan& Pl, const void* c, const void* psi, const void* g, void* dA, void* db, void* dc,
                         void* ws, hipStream_t st) {
  if (Pl.dt == FD_C64) return run_state_vjp_t<float>(Pl, c, psi, g, dA, db, dc, ws, st);
  return run_state_vjp_t<double>(Pl, c, psi, g, dA, db, dc, ws, st);
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
