// Host planner: validates a problem shape and builds the level tables of the
// selective schedule (Algorithm 1 over the detected modes, each node carrying
// the undetected block of Algorithm 2).  Host-only: no device call here
// except in ensure_device(), which uploads the tables on first use.
#include <algorithm>
#include <cstdlib>
#include <atomic>
#include <cstring>

#include "fd_internal.h"

namespace fd {

size_t elem_bytes(fd_dtype dt) { return dt == FD_C64 ? 8 : 16; }

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Lattice points n with 0 <= n_d <= ub[d] (no point if some ub[d] < 0) and
// |n| <= smax: a convolution over the modes.
static int64_t count_box_levels(const std::vector<int>& ub, int smax) {
  for (int u : ub)
    if (u < 0) return 0;
  std::vector<int64_t> cnt(smax + 1, 0), nxt(smax + 1, 0);
  cnt[0] = 1;
  for (int u : ub) {
    std::fill(nxt.begin(), nxt.end(), 0);
    for (int s = 0; s <= smax; ++s)
      for (int v = 0; v <= u && v <= s; ++v) nxt[s] += cnt[s - v];
    cnt.swap(nxt);
  }
  int64_t t = 0;
  for (int64_t x : cnt) t += x;
  return t;
}

namespace {
std::atomic<bool> g_unloading{false};
// Runs when the library is unloaded (process exit or dlclose): the HIP
// runtime may already be shutting down, so later releases skip device calls.
__attribute__((destructor)) void mark_unloading() { g_unloading.store(true); }
}  // namespace

bool unloading() { return g_unloading.load(); }

fd_status build_plan(int M, const int* cutoffs, uint32_t mask, fd_dtype dt, uint32_t flags, Plan* P,
                     std::string* err, int level_cap) {
  static std::atomic<uint64_t> next_uid{1};
  P->uid = next_uid.fetch_add(1);
  if (M < 1 || M > kMaxModes) {
    *err = "M must be in [1, 16]";
    return FD_ERR_INVALID_ARG;
  }
  if (!cutoffs) {
    *err = "cutoffs is NULL";
    return FD_ERR_INVALID_ARG;
  }
  if (dt != FD_C128 && dt != FD_C64) {
    *err = "dtype must be FD_C128 or FD_C64";
    return FD_ERR_INVALID_ARG;
  }
  if (flags > FD_B_GENERAL) {
    *err = "flags must be FD_B_AUTO, FD_B_ZERO or FD_B_GENERAL";
    return FD_ERR_INVALID_ARG;
  }
  if (M < 32 && (mask >> M) != 0) {
    *err = "detected_mask has bits at or above M";
    return FD_ERR_INVALID_ARG;
  }
  P->M = M;
  P->cut.assign(cutoffs, cutoffs + M);
  P->mask = mask;
  P->dt = dt;
  P->flags = flags;
  for (int j = 0; j < M; ++j) {
    if (cutoffs[j] < 1 || cutoffs[j] > kMaxCut) {
      *err = "every cutoff must be in [1, 64]";
      return FD_ERR_INVALID_ARG;
    }
  }
  P->umodes.clear();
  P->dmodes.clear();
  for (int j = 0; j < M; ++j) {
    if (cutoffs[j] < 2) continue;  // cutoff 1: vacuum only, no index moves
    if ((mask >> j) & 1u)
      P->dmodes.push_back(j);
    else
      P->umodes.push_back(j);
  }
  P->MU = (int)P->umodes.size();
  P->MD = (int)P->dmodes.size();
  if (P->MD > kMaxD) {
    *err = "at most 8 detected modes with cutoff >= 2 are supported";
    return FD_ERR_UNSUPPORTED;
  }
  if (P->MU > kMaxUq / 2) {
    *err = "at most 3 undetected modes with cutoff >= 2 are supported";
    return FD_ERR_UNSUPPORTED;
  }
  P->CU.clear();
  P->CD.clear();
  for (int j : P->umodes) P->CU.push_back(cutoffs[j]);
  for (int j : P->dmodes) P->CD.push_back(cutoffs[j]);
  P->nq = 2 * P->MU;
  P->npos = P->nq + 2 * P->MD;
  P->udims.clear();
  for (int q = 0; q < 2; ++q)
    for (int c : P->CU) P->udims.push_back(c);
  P->ustride.assign(P->nq, 1);
  int64_t B = 1;
  for (int q = P->nq - 1; q >= 0; --q) {
    P->ustride[q] = (int)B;
    B *= P->udims[q];
  }
  if (B > kMaxBlock) {
    *err = "undetected block prod C_u^2 exceeds 65536";
    return FD_ERR_UNSUPPORTED;
  }
  P->B = (int)B;
  // internal positions: U kets, U bras, then (ket, bra) per detected mode
  P->pos2blk.clear();
  for (int j : P->umodes) P->pos2blk.push_back(j);
  for (int j : P->umodes) P->pos2blk.push_back(M + j);
  for (int j : P->dmodes) {
    P->pos2blk.push_back(j);
    P->pos2blk.push_back(M + j);
  }
  // output size
  int64_t out = 1;
  if (level_cap < 0)
    for (int j = 0; j < M; ++j) out *= ((mask >> j) & 1u) ? cutoffs[j] : (int64_t)cutoffs[j] * cutoffs[j];
  P->out_elems = out;   // capped plans: set once the levels are counted
  if (level_cap >= 0 && P->MU > 0) {
    *err = "a total photon cutoff needs every mode with cutoff >= 2 detected";
    return FD_ERR_INVALID_ARG;
  }
  P->level_cap = level_cap;
  int64_t nt = 1;
  for (int c : P->CD) {
    nt *= c;
    if (level_cap < 0 && nt >= (int64_t(1) << 31)) {
      *err = "product of detected cutoffs must be < 2^31";
      return FD_ERR_UNSUPPORTED;
    }
    nt = std::min<int64_t>(nt, int64_t(1) << 40);
  }
  P->nodes_total = nt;
  if (P->B > 1 && nt > (int64_t(1) << 22)) {
    *err = "with undetected modes the product of detected cutoffs must be <= 2^22 (node records)";
    return FD_ERR_UNSUPPORTED;
  }
  const int MD = P->MD;
  int smax = 0;
  for (int c : P->CD) smax += c - 1;
  if (level_cap >= 0) smax = std::min(smax, level_cap);
  P->smax = smax;
  const int pnw = smax + 3;
  // ncnt[d][s] = #(n_d..n_{MD-1}) in the box with sum s
  P->ncnt.assign((size_t)(MD + 1) * (smax + 1), 0);
  auto NC = [&](int d, int s) -> int64_t& { return P->ncnt[(size_t)d * (smax + 1) + s]; };
  NC(MD, 0) = 1;
  for (int d = MD - 1; d >= 0; --d)
    for (int s = 0; s <= smax; ++s) {
      int64_t acc = 0;
      for (int v = 0; v < P->CD[d] && v <= s; ++v) acc += NC(d + 1, s - v);
      NC(d, s) = acc;
    }
  // PN[d][s+1] = sum_{s' <= s} ncnt[d][s'], s in [-1, smax+1]
  P->pn.assign((size_t)(MD + 1) * pnw, 0);
  for (int d = 0; d <= MD; ++d) {
    int64_t acc = 0;
    for (int s = -1; s <= smax + 1; ++s) {
      if (s >= 0 && s <= smax) acc += NC(d, s);
      P->pn[(size_t)d * pnw + (s + 1)] = (int)acc;
    }
  }
  // level offsets and group sizes
  const int G = std::max(MD, 1);
  P->lvl.assign((size_t)G * (smax + 2), 0);
  P->group_nodes.assign(G, 1);
  P->maxN.assign(G, 1);
  for (int g = 0; g < MD; ++g) {
    int64_t acc = 0, mx = 0;
    for (int S = 0; S <= smax + 1; ++S) {
      P->lvl[(size_t)g * (smax + 2) + S] = acc;
      if (S <= smax) {
        acc += NC(g, S);
        mx = std::max(mx, NC(g, S));
      }
    }
    P->group_nodes[g] = acc;
    P->maxN[g] = std::max<int64_t>(mx, 1);
  }
  if (level_cap >= 0) {
    // the lattice points of levels 0..smax, returned in level order
    nt = MD > 0 ? P->lvl[smax + 1] : 1;
    if (nt >= (int64_t(1) << 31)) {
      *err = "at most 2^31 - 1 lattice points below the total photon cutoff";
      return FD_ERR_UNSUPPORTED;
    }
    P->nodes_total = nt;
    P->out_elems = nt;
  }
  // the level kernels address a level's entries with 32-bit byte offsets
  if (MD > 0 && P->maxN[0] * P->B > (int64_t(1) << 28)) {
    *err = "a photon-number level (lattice points times undetected block) may hold at most 2^28 amplitudes";
    return FD_ERR_UNSUPPORTED;
  }
  // families
  P->nfam = 1 + 3 * MD + MD * (MD - 1);
  P->fam_group.assign(P->nfam, 0);
  for (int K = 0; K < MD; ++K) {
    P->fam_group[fam_f2(MD, K)] = K;
    for (int j = K + 1; j < MD; ++j) {
      P->fam_group[fam_1010(MD, K, j)] = K;
      P->fam_group[fam_1001(MD, K, j)] = K;
    }
  }
  // App. B counts (valid nodes per offset type; pivots of Algorithm 1)
  const std::vector<int>& C = P->CD;
  auto prod_except = [&](int a, int b2, int from) {
    int64_t p = 1;
    for (int i = from; i < MD; ++i)
      if (i != a && i != b2) p *= C[i];
    return p;
  };
  for (int i = 0; i < 6; ++i) P->stored[i] = 0;
  P->pivots = 0;
  if (MD > 0) {
    P->stored[F_F0] = nt;
    P->stored[F_F1K] += (C[0] - 1) * prod_except(0, -1, 0);
    P->stored[F_F1B] += std::max(C[0] - 2, 0) * prod_except(0, -1, 0);
    for (int j = 1; j < MD; ++j) {
      P->stored[F_F1K] += (int64_t)(C[0] - 1) * (C[j] - 1) * prod_except(0, j, 0);
      P->stored[F_F1B] += (int64_t)(C[0] - 1) * (C[j] - 1) * prod_except(0, j, 0);
    }
    for (int K = 0; K < MD; ++K) {
      P->stored[F_F2] += std::max(C[K] - 2, 0) * prod_except(K, -1, K);
      for (int j = K + 1; j < MD; ++j) {
        int64_t v = (int64_t)(C[K] - 1) * (C[j] - 1) * prod_except(K, j, K);
        P->stored[F_1010] += v;
        P->stored[F_1001] += v;
      }
    }
    P->pivots = (C[0] - 1) * prod_except(0, -1, 0);
    for (int K = 0; K < MD; ++K) P->pivots += (C[K] - 1) * prod_except(K, -1, K);
    if (level_cap >= 0) {
      // the same families and pivots, counted on the levels 0..smax
      auto ubox = [&]() { std::vector<int> u(MD); for (int d = 0; d < MD; ++d) u[d] = C[d] - 1; return u; };
      for (int i = 0; i < 6; ++i) P->stored[i] = 0;
      P->stored[F_F0] = nt;
      std::vector<int> u = ubox();
      u[0] = C[0] - 2;
      P->stored[F_F1K] += count_box_levels(u, smax);
      P->pivots = count_box_levels(u, smax);
      u[0] = C[0] - 3;
      P->stored[F_F1B] += count_box_levels(u, smax);
      for (int j = 1; j < MD; ++j) {
        u = ubox();
        u[0] = C[0] - 2;
        u[j] = C[j] - 2;
        P->stored[F_F1K] += count_box_levels(u, smax);
        P->stored[F_F1B] += count_box_levels(u, smax);
      }
      for (int K = 0; K < MD; ++K) {
        u = ubox();
        for (int d = 0; d < K; ++d) u[d] = 0;
        u[K] = C[K] - 2;
        P->pivots += count_box_levels(u, smax);
        u[K] = C[K] - 3;
        P->stored[F_F2] += count_box_levels(u, smax);
        for (int j = K + 1; j < MD; ++j) {
          u[K] = C[K] - 2;
          std::vector<int> w = u;
          w[j] = C[j] - 2;
          const int64_t v = count_box_levels(w, smax);
          P->stored[F_1010] += v;
          P->stored[F_1001] += v;
        }
      }
    }
  } else {
    P->stored[F_F0] = 1;
  }
  // undetected block entries by weight (fill order of step 1)
  P->wmax = 0;
  for (int q = 0; q < P->nq; ++q) P->wmax += P->udims[q] - 1;
  P->woff.assign(P->wmax + 2, 0);
  std::vector<int> wt(P->B, 0);
  for (int e = 0; e < P->B; ++e) {
    int rem = e, w = 0;
    for (int q = 0; q < P->nq; ++q) {
      w += rem / P->ustride[q];
      rem %= P->ustride[q];
    }
    wt[e] = w;
    P->woff[w + 1]++;
  }
  for (int w = 0; w <= P->wmax; ++w) P->woff[w + 1] += P->woff[w];
  P->elist.assign(P->B, 0);
  {
    std::vector<int> pos(P->woff.begin(), P->woff.end() - 1);
    for (int e = 0; e < P->B; ++e) P->elist[pos[wt[e]]++] = e;
  }
  // the block kernels and the block fills hold their rows in LDS where they
  // fit, else stream them from HBM
  if (P->B > 1) {
    const size_t rows = std::max(fwd_lds_bytes_for(*P, chunk_geo(*P)), fwd_lds_bytes_for(*P, chunk_geo(*P, kBT / 2)));
    P->st_fwd = P->MD > 0 && rows > kMaxLds;
    P->st_ufill = ufill_lds_bytes(*P, false) > kMaxLds;
    P->vjp_waves = kVjpWaves;
    if (vjp_lds_bytes(*P) > kMaxLds) P->vjp_waves = kVjpWavesLds;
    P->st_vjp = P->MD > 0 && vjp_lds_bytes(*P) > kMaxLds;
    P->st_ufill_vjp = ufill_lds_bytes(*P, true) > kMaxLds;
  }
  P->targets = -1;
  P->terms = -1;
  return FD_OK;
}

DevPlan make_devplan(const Plan& P, bool odd) {
  DevPlan d;
  std::memset(&d, 0, sizeof(d));
  d.MD = P.MD;
  d.MU = P.MU;
  d.nq = P.nq;
  d.npos = P.npos;
  d.B = P.B;
  d.smax = P.smax;
  d.pnw = P.smax + 3;
  d.odd = odd ? 1 : 0;
  for (int j = 0; j < P.MD; ++j) d.CD[j] = P.CD[j];
  for (int q = 0; q < P.nq; ++q) {
    d.udims[q] = P.udims[q];
    d.ustride[q] = P.ustride[q];
    d.uinv[q] = 1.0 / P.ustride[q];
  }
  for (int j = 0; j < P.MD; ++j) d.cinv[j] = 1.0 / P.CD[j];
  d.pn = P.d_pn;
  d.lvl = P.d_lvl;
  d.node = P.d_node;
  for (int g = 0; g < std::max(P.MD, 1); ++g) d.ringN[g] = P.maxN[g];
  return d;
}

size_t prep_core_bytes(const Plan& P) {
  size_t n = (size_t)P.npos * P.npos + P.npos + 1;
  return align256(n * elem_bytes(P.dt));
}

// The prep block of every workspace; a plan whose forward block rows stream
// from HBM keeps its workgroups' bridge pivot slots right after it.
size_t prep_bytes(const Plan& P) {
  size_t n = prep_core_bytes(P);
  if (P.st_fwd) n += align256((size_t)kStreamSlots * fwd_stream_entries(P) * elem_bytes(P.dt));
  return n;
}

size_t fwd_stream_entries(const Plan& P) {
  if (P.B == 1 || P.MD == 0) return 0;
  const ChunkGeo G = chunk_geo(P);   // the taller of the two chunk geometries
  return (size_t)P.MD * (G.RC + 1) * G.R0;
}

FwdLayout fwd_layout(const Plan& P, bool odd, bool store_all, size_t base) {
  FwdLayout L;
  const size_t eb = elem_bytes(P.dt);
  size_t off = base;
  L.prep = off;
  off += prep_bytes(P);
  L.f0 = off;
  off = align256(off + (size_t)P.nodes_total * P.B * eb);
  L.fam.assign(P.nfam, 0);
  const int MD = P.MD;
  for (int f = 1; f < P.nfam; ++f) {
    bool is_odd = (f < 1 + 2 * MD);
    if (is_odd && !odd) continue;
    int g = P.fam_group[f];
    size_t nodes = store_all ? (size_t)P.group_nodes[g] : 2 * (size_t)P.maxN[g];
    L.fam[f] = off;
    off = align256(off + nodes * P.B * eb);
  }
  L.total = off;
  return L;
}

// Chunks of whole rows of the first undetected coordinate, about `target`
// entries each, spread evenly over the rows (one (lattice point, chunk) unit
// per workgroup of the block kernels).
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

// Dynamic LDS of the block reverse kernel for a chunk geometry: the forward
// pivot rows, the undetected-neighbour terms, each wavefront's record
// staging batch and A, b (or the pair table of the final fold, if larger), then the
// square-root tables.
size_t vjp_lds_bytes_for(const Plan& Pl, const ChunkGeo& G) {
  const size_t eb = elem_bytes(Pl.dt), rb = eb / 2;
  const int MD = Pl.MD, NPD = 2 * MD, NR = Pl.npos + 1, WV = Pl.vjp_waves;
  const size_t rows = Pl.st_vjp ? 0 : (size_t)(G.RC + 1) * G.R0 + (size_t)Pl.nq * (G.RC + 2) * G.R0;
  const size_t ents = rows + (size_t)WV * (kBlockBatch + 1) * (NPD + NR);
  return std::max((ents + (size_t)Pl.npos * (Pl.npos + 1)) * eb, (size_t)WV * NPD * NR * 16) +
         2 * (kMaxCut + 4) * rb;
}

// Chunk geometry of a forward level with nwork lattice points (its units
// span kFwdWaves wavefronts): about kFwdChunk own entries, kFwdChunkSmall on
// levels with few units, and the one-wavefront heights where the taller
// chunk's rows do not fit the LDS (those fit whenever the plan's rows are not
// streamed).
ChunkGeo fwd_geo(const Plan& Pl, int64_t nwork) {
  ChunkGeo G = chunk_geo(Pl, kFwdChunk);
  if (nwork * G.nchunks < kSmallLevelUnits) G = chunk_geo(Pl, kFwdChunkSmall);
  if (fwd_lds_bytes_for(Pl, G) <= kMaxLds) return G;
  G = chunk_geo(Pl, kBT);
  if (nwork * G.nchunks < kSmallLevelUnits) G = chunk_geo(Pl, kBT / 2);
  return G;
}

// Row chunks of the reverse block kernel: own entries per unit on large
// levels, on levels with fewer than `small_units` units, and that threshold.
// Four wavefronts take 128 entries each (48 on small levels): a chunk's two
// halo rows then cost less of its time (5-mode conditional reverse 6.2 -> 5.7
// ms, 6-mode gradient circuit 12.9 -> 10.4 ms); two wavefronts keep 64 (32).
VjpChunking vjp_chunking(const Plan& Pl) {
  if (Pl.vjp_waves == kVjpWaves) return {128 * kVjpWaves, 48 * kVjpWaves, 1024};
  return {64 * Pl.vjp_waves, 32 * Pl.vjp_waves, kSmallLevelUnits};
}

// Chunk geometry of a reverse level with nwork lattice points.
ChunkGeo vjp_geo(const Plan& Pl, int64_t nwork) {
  const VjpChunking t = vjp_chunking(Pl);
  ChunkGeo G = chunk_geo(Pl, t.target);
  if (nwork * G.nchunks < t.small_units) G = chunk_geo(Pl, t.small);
  return G;
}

size_t fwd_stream_lds_bytes(const Plan& Pl) {
  return (size_t)Pl.npos * (Pl.npos + 1) * elem_bytes(Pl.dt) + 2 * (kMaxCut + 4) * (elem_bytes(Pl.dt) / 2);
}

size_t fwd_lds_bytes_for(const Plan& Pl, const ChunkGeo& G, bool jvp) {
  return (((size_t)(G.RC + 2) + (size_t)Pl.MD * (G.RC + 1)) * G.R0 + (size_t)Pl.npos * (Pl.npos + 1)) *
             elem_bytes(Pl.dt) * (jvp ? 2 : 1) +
         2 * (kMaxCut + 4) * (elem_bytes(Pl.dt) / 2);
}

size_t vjp_lds_bytes(const Plan& Pl) {
  const VjpChunking t = vjp_chunking(Pl);
  return std::max(vjp_lds_bytes_for(Pl, chunk_geo(Pl, t.target)), vjp_lds_bytes_for(Pl, chunk_geo(Pl, t.small)));
}

size_t jvp_half_bytes(const Plan& Pl) { return (fwd_layout(Pl, true, false, 0).total + 255) / 256 * 256; }

// State vectors: the amplitudes in level order plus A and b of the kept modes.
size_t state_ws_bytes(const Plan& Pl) {
  const size_t eb = elem_bytes(Pl.dt);
  return align256((size_t)Pl.nodes_total * eb) + align256((size_t)(Pl.MD * Pl.MD + Pl.MD) * eb);
}

// One double2 per reduction slot and cotangent term (bbar, upper triangle of
// Abar, sum g conj(psi)).
size_t state_vjp_ws_bytes(const Plan& Pl) {
  const int ncol = Pl.MD + Pl.MD * (Pl.MD + 1) / 2 + 1;
  return (size_t)kVjpSlots * ncol * sizeof(double2);
}

bool ckpt_keeps_family(const Plan& P, int f) {
  const bool odd_family = f >= 1 && f < 1 + 2 * P.MD;
  return f >= 1 && (!odd_family || P.odd_for(P.flags == FD_B_ZERO));
}

static int64_t level_nodes(const Plan& P, int g, int L) {
  return (L < 0 || L > P.smax) ? 0 : P.ncnt[(size_t)g * (P.smax + 1) + L];
}

int64_t seg_node(const Plan& P, int g, int seg_lo, int L) {
  int64_t n = 0;
  for (int l = std::max(seg_lo - 1, 0); l < L; ++l) n += level_nodes(P, g, l);
  return n;
}

CkptLayout ckpt_layout(const Plan& P) {
  CkptLayout L;
  const size_t eb = elem_bytes(P.dt);
  const int s = std::max(P.ckpt, 1);
  L.nseg = P.MD > 0 ? (P.smax + 1 + s - 1) / s : 1;
  // offset 0 means "not kept" in every layout: F0 starts after a 256-byte gap
  L.f0 = 256;
  size_t off = align256(L.f0 + (size_t)P.nodes_total * P.B * eb);
  L.ck.assign((size_t)std::max(L.nseg - 1, 0) * P.nfam, 0);
  for (int c = 1; c < L.nseg; ++c)
    for (int f = 1; f < P.nfam; ++f) {
      if (!ckpt_keeps_family(P, f)) continue;
      L.ck[(size_t)(c - 1) * P.nfam + f] = off;
      off = align256(off + (size_t)level_nodes(P, P.fam_group[f], c * s - 1) * P.B * eb);
    }
  L.total = off;
  return L;
}

SegLayout seg_layout(const Plan& P) {
  SegLayout L;
  const size_t eb = elem_bytes(P.dt);
  L.base = align256(vjp_layout(P, true, 0).total);
  size_t off = L.base;
  L.fam.assign(P.nfam, 0);
  const int s = std::max(P.ckpt, 1);
  for (int f = 1; f < P.nfam; ++f) {
    if (!ckpt_keeps_family(P, f)) continue;
    const int g = P.fam_group[f];
    int64_t most = 2 * P.maxN[g];   // the forward's ring
    for (int lo = 0; lo <= P.smax; lo += s) {
      const int hi = std::min(lo + s - 1, P.smax);
      most = std::max(most, seg_node(P, g, lo, hi + 1));
    }
    L.fam[f] = off;
    off = align256(off + (size_t)most * P.B * eb);
  }
  L.total = off;
  return L;
}

size_t saved_bytes(const Plan& P) {
  return P.ckpt > 0 ? ckpt_layout(P).total : fwd_layout(P, true, true, 0).total;
}

size_t vjp_ws_bytes(const Plan& P) {
  return P.ckpt > 0 ? seg_layout(P).total : vjp_layout(P, true, 0).total;
}

VjpLayout vjp_layout(const Plan& P, bool odd, size_t base) {
  VjpLayout L;
  const size_t eb = elem_bytes(P.dt);
  size_t off = base;
  L.prep = off;
  off += prep_bytes(P);
  L.g0 = off;
  off = align256(off + (size_t)P.nodes_total * P.B * eb);
  L.gfam.assign(P.nfam, 0);
  const int MD = P.MD;
  for (int f = 0; f < P.nfam; ++f) {
    bool is_odd = (f >= 1 && f < 1 + 2 * MD);
    if (is_odd && !odd) continue;
    int g = P.fam_group[f];
    L.gfam[f] = off;
    off = align256(off + 2 * (size_t)P.maxN[g] * P.B * eb);
  }
  L.partial = off;
  off = align256(off + (size_t)kPartialSlots * P.npos * (P.npos + 1) * 16);
  if (P.B > 1 && P.MD > 0) {
    L.priv = off;
    off = align256(off + (size_t)(P.st_vjp ? kStreamSlots : kPartialSlots) * vjp_private_entries(P) * eb);
  }
  if (P.st_ufill_vjp) {
    L.ublk = off;
    off = align256(off + (size_t)P.B * eb);
  }
  L.total = off;
  return L;
}

size_t vjp_private_entries(const Plan& P) {
  if (P.B == 1 || P.MD == 0) return 0;
  const ChunkGeo G = chunk_geo(P, vjp_chunking(P).target);   // the taller of the launcher's two chunk heights
  return (size_t)(P.MD + 1) * (G.RC + 1) * G.R0 + (size_t)G.RC * G.R0 +
         (P.st_vjp ? (size_t)P.nq * (G.RC + 2) * G.R0 : 0);
}


// Rank of lattice point v within its level (lexicographic, first mode
// slowest): sum over d of #points of sub-box d+1 whose sum lies in
// (s_d - v_d, s_d], with s_d the sum of v over modes d...MD-1.
static int64_t host_rank(const Plan& P, const int* v) {
  const int pnw = P.smax + 3;
  int sd = 0;
  for (int j = 0; j < P.MD; ++j) sd += v[j];
  int64_t r = 0;
  for (int d = 0; d < P.MD; ++d) {
    r += P.pn[(size_t)(d + 1) * pnw + sd + 1] - P.pn[(size_t)(d + 1) * pnw + sd - v[d] + 1];
    sd -= v[d];
  }
  return r;
}

// Node records of an Algorithm 2 plan: for every lattice point m (level-major
// order) m itself, the rank of m - 1_j at level |m| - 1 (-1 if m_j = 0) and
// the rank of m + 1_j at level |m| + 1 (-1 outside the box).  The block
// kernels read a unit's record with one scalar load instead of unranking.
static bool build_node_table(const Plan& P, std::vector<int>* out, std::string* err) {
  const int MD = P.MD;
  out->assign((size_t)P.nodes_total * kNodeStride, -1);
  std::vector<int> m(MD, 0), v(MD);
  for (int64_t it = 0; it < P.nodes_total; ++it) {
    int S = 0;
    for (int j = 0; j < MD; ++j) S += m[j];
    const int64_t r = host_rank(P, m.data());
    const int64_t id = P.lvl[S] + r;
    if (r < 0 || r >= P.ncnt[S] || id >= P.nodes_total || (*out)[(size_t)id * kNodeStride] != -1) {
      *err = "internal: lattice ranks are not a bijection";
      return false;
    }
    int* rec = out->data() + (size_t)id * kNodeStride;
    for (int j = 0; j < MD; ++j) {
      rec[j] = m[j];
      v = m;
      v[j] -= 1;
      rec[MD + j] = m[j] > 0 ? (int)host_rank(P, v.data()) : -1;
      v[j] += 2;
      rec[2 * MD + j] = m[j] + 1 < P.CD[j] ? (int)host_rank(P, v.data()) : -1;
    }
    for (int j = MD - 1; j >= 0; --j) {
      if (++m[j] < P.CD[j]) break;
      m[j] = 0;
    }
  }
  return true;
}

fd_status ensure_device(Plan* P, std::string* err) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    *err = "hipGetDevice failed";
    return FD_ERR_HIP;
  }
  if (P->d_pn && P->device == dev) return FD_OK;
  if (P->d_pn) {
    *err = "plan was initialised on another device";
    return FD_ERR_INVALID_ARG;
  }
  size_t npn = P->pn.size() * sizeof(int);
  size_t nlvl = P->lvl.size() * sizeof(int64_t);
  size_t nel = P->elist.size() * sizeof(int), nwo = P->woff.size() * sizeof(int);
  if (hipMalloc((void**)&P->d_pn, npn) != hipSuccess || hipMalloc((void**)&P->d_lvl, nlvl) != hipSuccess ||
      hipMalloc((void**)&P->d_status, 256) != hipSuccess || hipMalloc((void**)&P->d_elist, nel) != hipSuccess ||
      hipMalloc((void**)&P->d_woff, nwo) != hipSuccess) {
    *err = "hipMalloc of plan tables failed";
    return FD_ERR_OOM;
  }
  if (hipMemcpy(P->d_pn, P->pn.data(), npn, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P->d_lvl, P->lvl.data(), nlvl, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P->d_elist, P->elist.data(), nel, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(P->d_woff, P->woff.data(), nwo, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(P->d_status, 0, 256) != hipSuccess) {
    *err = "upload of plan tables failed";
    return FD_ERR_HIP;
  }
  if (P->MD > 0 && P->B == 1 &&
      hipMalloc((void**)&P->d_mass, (size_t)(P->smax + 1) * kMassParts * sizeof(double)) != hipSuccess) {
    *err = "hipMalloc of the level masses failed";
    return FD_ERR_OOM;
  }
  if (P->B > 1 && P->MD > 0) {
    std::vector<int> nt;
    if (!build_node_table(*P, &nt, err)) return FD_ERR_HIP;
    if (hipMalloc((void**)&P->d_node, nt.size() * sizeof(int)) != hipSuccess) {
      *err = "hipMalloc of the node table failed";
      return FD_ERR_OOM;
    }
    if (hipMemcpy(P->d_node, nt.data(), nt.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
      *err = "upload of the node table failed";
      return FD_ERR_HIP;
    }
  }
  P->device = dev;
  return FD_OK;
}

}  // namespace fd

namespace fd {

// Computed amplitudes and A-terms of one forward sweep (for FLOP accounting):
// every valid target of every applied pivot, times the block size; a term is
// one read with a non-zero sqrt coefficient (undetected neighbours included),
// plus the pivot's b-term when b != 0.
void count_work(const Plan& P, bool b_zero, int64_t* targets, int64_t* terms) {
  const int MD = P.MD;
  const bool odd = P.odd_for(b_zero);
  double unb = 0.0;  // undetected-neighbour terms per target block
  for (int q = 0; q < P.nq; ++q) unb += (double)P.B * (1.0 - 1.0 / P.udims[q]);
  const double bterm = b_zero ? 0.0 : (double)P.B;
  int64_t T = (P.B > 1) ? (P.B - 1) : 0;   // undetected block fill
  double W = 0.0;
  if (P.B > 1) W += (double)P.B * 2.0;     // rough: <= 2 reads per fill entry
  if (MD == 0 || P.nodes_total > (int64_t(1) << 27)) {
    *targets = MD == 0 ? T : -1;
    *terms = MD == 0 ? (int64_t)W : -1;
    return;
  }
  const std::vector<int>& C = P.CD;
  std::vector<int> m(MD, 0);
  int msum = 0;   // |m|: the walk skips points above level smax (capped plans)
  for (int64_t it = 0; it < P.nodes_total; ++it) {
    int nz = 0;
    for (int j = 0; j < MD; ++j) nz += m[j] > 0;
    if (odd && m[0] <= C[0] - 2) {
      int t = 0;
      for (int j = 0; j < MD; ++j) {
        if (j == 0 || m[j] <= C[j] - 2) ++t;                                   // F1k(j)
        if ((j == 0) ? (m[0] <= C[0] - 3) : (m[j] <= C[j] - 2)) ++t;          // F1b(j)
      }
      T += (int64_t)t * P.B;
      W += (double)t * (2.0 * nz * P.B + unb + bterm);
    }
    int K0 = MD;
    for (int d = MD - 1; d >= 0; --d)
      if (m[d] > 0) K0 = d;
    for (int K = 0; K < MD && K <= K0; ++K) {
      if (m[K] > C[K] - 2) continue;
      int reads = 1 + (m[K] > 0);
      for (int j = K + 1; j < MD; ++j) reads += 2 * (m[j] > 0);
      // the F0 target d(m + 1_K) lies above a total photon cutoff's last level
      const bool f0_target = !(P.level_cap >= 0 && msum == P.smax);
      int t = (f0_target ? 1 : 0) + (m[K] <= C[K] - 3);
      for (int j = K + 1; j < MD; ++j) t += 2 * (m[j] <= C[j] - 2);
      T += (int64_t)t * P.B;
      W += (double)t * ((double)reads * P.B + (odd ? unb + bterm : 0.0));
    }
    for (int j = MD - 1; j >= 0; --j) {
      ++m[j];
      ++msum;
      if (m[j] < C[j] && msum <= P.smax) break;
      msum -= m[j];
      m[j] = 0;
    }
  }
  *targets = T;
  *terms = (int64_t)W;
}

}  // namespace fd
