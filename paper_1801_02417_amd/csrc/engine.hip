// Host side of the library: set-up (visibility sorting and tile binning, tables), device
// memory of one solve, the pass sequence of one Algorithm-1 iteration captured as a HIP
// graph, the FP64 power iteration, the stopping quantities, and the C ABI.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <limits>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "common.hpp"
#include "engine.hpp"
#include "graph_key.hpp"
#include "launch.hpp"
#include "psara.h"

namespace psara {

std::vector<double> daubechies(int p);
double kb_beta(int taps, double alpha);
double kb_hat(int taps, double beta, double nu);
std::vector<double> kb_poly(int taps, double beta, int deg);

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(PSARA_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Host <-> device copy ordered on `stream` and waited for.  Never the legacy default stream:
// a synchronous hipMemcpy there would have to wait for every blocking stream, which breaks a
// graph capture that another thread (the request server) may have in progress.
static void copy_sync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t stream, const char* what) {
  hip_check(hipMemcpyAsync(dst, src, bytes, kind, stream), what);
  hip_check(hipStreamSynchronize(stream), what);
}

// ------------------------------------------------------------------------------------------------
// geometry: window starts, fractional offsets, sorting by grid tile, per-tile lists
Geometry build_geometry(int n, int64_t M, const double* uv, int alpha, int T) {
  Geometry g;
  g.n = n; g.K = alpha * n; g.T = T; g.M = M;
  g.ts = degrid_tile(g.K);
  g.nts = g.K / g.ts;
  g.ntsg = g.K / kGridTile;
  g.beta = kb_beta(T, alpha);
  const int K = g.K, ts = g.ts, nts = g.nts;
  const int ntiles = nts * nts;
  std::vector<int> k1(M), k2(M), tile(M);
  std::vector<double> f1(M), f2(M);
  for (int64_t m = 0; m < M; ++m) {
    const double w0 = uv[2 * m], w1 = uv[2 * m + 1];
    if (!(w0 >= -M_PI && w0 < M_PI && w1 >= -M_PI && w1 < M_PI))
      throw Error(PSARA_EINVAL, "uv point outside [-pi, pi)");
    const double t1 = (double)K * w0 / (2.0 * M_PI), t2 = (double)K * w1 / (2.0 * M_PI);
    const double c1 = std::ceil(t1 - T / 2.0), c2 = std::ceil(t2 - T / 2.0);
    f1[m] = t1 - c1; f2[m] = t2 - c2;
    k1[m] = ((int)c1) & (K - 1);
    k2[m] = ((int)c2) & (K - 1);
    tile[m] = (k1[m] / ts) * nts + k2[m] / ts;
  }
  // rows sorted by de-gridding tile, then by the gridding tile (kGridTile-sided, inside it) that
  // holds their window start, then by window start: each gridding tile's rows are then one
  // contiguous range, so the gridding reads its rows without an index list
  const int tg0 = kGridTile, ntsg0 = K / kGridTile;
  std::vector<int> gtile(M);
  for (int64_t m = 0; m < M; ++m) gtile[m] = (k1[m] / tg0) * ntsg0 + k2[m] / tg0;
  std::vector<int64_t> order(M);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    if (tile[a] != tile[b]) return tile[a] < tile[b];
    if (gtile[a] != gtile[b]) return gtile[a] < gtile[b];
    if (k1[a] != k1[b]) return k1[a] < k1[b];
    return k2[a] < k2[b];
  });
  g.perm = order;
  g.k0.resize(M);
  g.frac.resize(2 * M);
  g.own_ptr.assign(ntiles + 1, 0);
  for (int64_t p = 0; p < M; ++p) {
    const int64_t m = order[p];
    g.k0[p] = (k1[m] << 16) | k2[m];
    g.frac[2 * p] = f1[m];
    g.frac[2 * p + 1] = f2[m];
    g.own_ptr[tile[m] + 1]++;
  }
  for (int t = 0; t < ntiles; ++t) g.own_ptr[t + 1] += g.own_ptr[t];
  // gridding: every visibility belongs to the kGridTile x kGridTile tile that holds its window
  // start; a gridding tile lies inside one de-gridding tile, so by the sort its rows are one
  // contiguous range, in (k1, k2) order
  const int tg = kGridTile, ntsg = g.ntsg, ntg = ntsg * ntsg;
  auto owner = [&](int64_t p) { return ((g.k0[p] >> 16) / tg) * ntsg + (g.k0[p] & 0xffff) / tg; };
  g.row_beg.assign(ntg, 0);
  g.row_end.assign(ntg, 0);
  std::vector<int> count(ntg, 0);
  for (int64_t p = 0; p < M; ++p) {
    const int t = owner(p);
    if (count[t]++ == 0) g.row_beg[t] = (int)p;
    g.row_end[t] = (int)p + 1;
  }
  for (int t = 0; t < ntg; ++t)
    if (g.row_end[t] - g.row_beg[t] != count[t]) throw Error(PSARA_EINVAL, "internal: a gridding tile's rows are not contiguous");
  build_grid_chunks(g, kChunkEntries);
  return g;
}

void build_grid_chunks(Geometry& g, int chunk_entries) {
  const int ntg = g.ntsg * g.ntsg;
  g.run_pack.clear();
  g.chunks.clear(); g.chunk_ent.clear(); g.tile_slots.clear(); g.slot_box.clear(); g.tile_box.clear(); g.small_ids.clear();
  g.n_slots = 0;
  g.chunk_entries = chunk_entries;
  // runs: consecutive rows of a tile with the same window start (their taps hit the
  // same cells), split at kRunMax; chunks of whole runs with <= chunk_entries entries, runs
  // ordered longest first inside a chunk so the lanes of a wave loop for similar lengths.
  // Every chunk accumulates its tile plus the T-1 halo in its own slot; the column inverse
  // FFT sums the slots of a cell's tile and of the three tiles whose halos reach it.
  for (int t = 0; t < ntg; ++t) {
    std::vector<std::pair<int, int>> runs;
    for (int e = g.row_beg[t]; e < g.row_end[t];) {
      int f = e + 1;
      while (f < g.row_end[t] && f - e < kRunMax && g.k0[f] == g.k0[e]) ++f;
      runs.push_back({e, f - e});
      e = f;
    }
    const int first_slot = g.n_slots;
    int u_lo1 = 255, u_hi1 = 0, u_lo2 = 255, u_hi2 = 0;   // union of the tile's boxes (empty: none)
    size_t r = 0;
    while (r < runs.size()) {
      const size_t r0 = r;
      int entries = 0;
      while (r < runs.size() && (entries + runs[r].second <= chunk_entries || r == r0)) entries += runs[r++].second;
      std::stable_sort(runs.begin() + r0, runs.begin() + r,
                       [](const std::pair<int, int>& x, const std::pair<int, int>& y) { return x.second > y.second; });
      const int base = (int)g.run_pack.size();
      int lo = g.row_end[t], hi = g.row_beg[t];
      for (size_t q = r0; q < r; ++q) {
        lo = std::min(lo, runs[q].first);
        hi = std::max(hi, runs[q].first + runs[q].second);
      }
      // the cells the chunk's windows cover, as offsets in the tile's region
      const int b1 = (t / g.ntsg) * kGridTile, b2 = (t % g.ntsg) * kGridTile;
      int lo1 = kGridTile, hi1 = 0, lo2 = kGridTile, hi2 = 0;
      for (size_t q = r0; q < r; ++q) {
        const int pk = g.k0[runs[q].first];
        g.run_pack.push_back(pack_run(runs[q].first - lo, runs[q].second, (pk >> 16) - b1, (pk & 0xffff) - b2));
        lo1 = std::min(lo1, (pk >> 16) - b1);
        hi1 = std::max(hi1, (pk >> 16) - b1);
        lo2 = std::min(lo2, (pk & 0xffff) - b2);
        hi2 = std::max(hi2, (pk & 0xffff) - b2);
      }
      g.slot_box.push_back(pack_box(lo1, hi1 + g.T - 1, lo2, hi2 + g.T - 1));
      u_lo1 = std::min(u_lo1, lo1); u_hi1 = std::max(u_hi1, hi1 + g.T - 1);
      u_lo2 = std::min(u_lo2, lo2); u_hi2 = std::max(u_hi2, hi2 + g.T - 1);
      g.chunks.push_back(make_int4(t, base, base + (int)(r - r0), g.n_slots++));
      g.chunk_ent.push_back(make_int2(lo, hi));
    }
    g.tile_slots.push_back(make_int2(first_slot, g.n_slots - first_slot));
    g.tile_box.push_back(pack_box(u_lo1, u_hi1, u_lo2, u_hi2));
  }
  // the small chunks, gridded one per wave, heaviest first
  for (int c = 0; c < (int)g.chunks.size(); ++c)
    if (g.chunk_ent[c].y - g.chunk_ent[c].x <= kSmallChunk) g.small_ids.push_back(c);
  std::stable_sort(g.small_ids.begin(), g.small_ids.end(), [&](int a, int b) {
    return g.chunk_ent[a].y - g.chunk_ent[a].x > g.chunk_ent[b].y - g.chunk_ent[b].x;
  });
}

void check_tuning(const Tuning& t, int K) {
  if (t.grid_chunk != 256 && t.grid_chunk != 512 && t.grid_chunk != 1024)
    throw Error(PSARA_EINVAL, "grid_chunk must be 256, 512 or 1024");
  if (t.degrid_item < 64 || t.degrid_item > 1024 || (t.degrid_item & (t.degrid_item - 1)))
    throw Error(PSARA_EINVAL, "degrid_item must be a power of two in [64, 1024]");
  if (t.ana_wide < 0 || t.ana_wide > (kAnaWide | kAnaAllBases))
    throw Error(PSARA_EINVAL, "analysis_wide must be 0, 1, 2 or 3");
  if (t.fft_cells != 0 && ((t.fft_cells != 512 && t.fft_cells != 1024 && t.fft_cells != 2048) || t.fft_cells < K))
    throw Error(PSARA_EINVAL, "fft_cells must be 0 or 512, 1024 or 2048, and at least the grid side 2n");
}

// ------------------------------------------------------------------------------------------------
// work lists (appended per problem, so batches concatenate them)

// Orders gridding items: the factor items first, then the chunks by decreasing work (entries
// plus a flush cost per run), so the heaviest start first and the tail is short, then the items
// of small chunks (eight chunks each, one per wave) by decreasing entries of their first chunk.
// geo_of(prob) gives the geometry of an item's problem.
template <typename It, typename GeoOf>
void order_grid_items(It begin, It end, GeoOf geo_of) {
  auto cost = [&](const int4& it) -> long long {
    if (it.y == kGridFactorItem) return std::numeric_limits<long long>::max();
    const Geometry& g = *geo_of(it.x);
    if (it.y == kGridSmallItem) {
      const int c = g.small_ids[it.z];
      return (long long)(g.chunk_ent[c].y - g.chunk_ent[c].x) - (1LL << 40);
    }
    return (g.chunk_ent[it.y].y - g.chunk_ent[it.y].x) + 3LL * (g.chunks[it.y].z - g.chunks[it.y].y);
  };
  std::stable_sort(begin, end, [&](const int4& a, const int4& b) { return cost(a) > cost(b); });
}
// Orders de-grid items for the eight XCDs that workgroups are dealt to in turn: the items of
// one tile (which stage overlapping k1 bands of the same window) all take positions of one XCD,
// where they share its L2 lines; tiles go to the XCD with the fewest rows so far, largest
// first, and each XCD's items run fullest first, so the tail of the launch is made of the short
// ones.  (An item keeps its partial index, so the norm's reduction order does not change.)
template <typename It>
void order_degrid_items(It begin, It end) {
  std::vector<int4> v(begin, end);
  if (v.size() < 2) return;
  auto rows = [](const int4& a) { return a.y >> 16; };
  auto key = [](const int4& a) { return std::make_pair(a.x, a.y & 0xffff); };   // (problem, tile)
  std::stable_sort(v.begin(), v.end(), [&](const int4& a, const int4& b) { return key(a) < key(b); });
  struct Group { size_t beg, end; long long rows; };
  std::vector<Group> groups;
  for (size_t i = 0; i < v.size();) {
    size_t j = i;
    long long r = 0;
    while (j < v.size() && key(v[j]) == key(v[i])) r += rows(v[j++]);
    groups.push_back({i, j, r});
    i = j;
  }
  std::stable_sort(groups.begin(), groups.end(), [](const Group& a, const Group& b) { return a.rows > b.rows; });
  constexpr int kXcds = 8;
  std::vector<int4> q[kXcds];
  long long load[kXcds] = {};
  for (const Group& g : groups) {
    const int x = (int)(std::min_element(load, load + kXcds) - load);
    q[x].insert(q[x].end(), v.begin() + g.beg, v.begin() + g.end);
    load[x] += g.rows;
  }
  size_t longest = 0;
  for (auto& qx : q) {
    std::stable_sort(qx.begin(), qx.end(), [&](const int4& a, const int4& b) { return rows(a) > rows(b); });
    longest = std::max(longest, qx.size());
  }
  It out = begin;
  for (size_t j = 0; j < longest; ++j)
    for (int x = 0; x < kXcds; ++x)
      if (j < q[x].size()) *out++ = q[x][j];
}
void add_operator_items(ItemSet& S, int prob, const Geometry& g, int cells, int rcells, int dg_item, int* n_p6) {
  const int n = g.n, K = g.K, N = n * n;
  const int lines = cells / K, rlines = rcells / K;
  for (int b = 0; b < (N + 255) / 256; ++b) S.img.push_back(make_int4(prob, b, 0, 0));
  for (int l = 0; l < n; l += rlines) S.rows.push_back(make_int4(prob, l, 0, 0));
  for (int l = 0; l < K; l += lines) S.cols.push_back(make_int4(prob, l, 0, 0));
  const int ntiles = g.nts * g.nts;
  const size_t first_p6 = S.p6.size();
  int part = 0;
  for (int t = 0; t < ntiles; ++t) {
    // (a de-grid item packs its tile and row count in one int: tiles < 2^16, rows < 2^15)
    if (ntiles > 0xffff || dg_item > 0x7fff) throw Error(PSARA_EINVAL, "de-grid tiling out of range");
    for (int v = g.own_ptr[t]; v < g.own_ptr[t + 1]; v += dg_item) {
      const int rows = std::min(dg_item, g.own_ptr[t + 1] - v);
      // the k1 band of the tile window the item's rows use: their smallest and largest window
      // starts k1, relative to the tile
      const int b1 = (t / g.nts) * g.ts;
      int lo = g.ts, hi = 0;
      for (int p = v; p < v + rows; ++p) {
        lo = std::min(lo, (g.k0[p] >> 16) - b1);
        hi = std::max(hi, (g.k0[p] >> 16) - b1);
      }
      if (part >= (1 << 20) || g.ts > 32) throw Error(PSARA_EINVAL, "de-grid item fields out of range");
      S.p6.push_back(make_int4(prob, t | (rows << 16), v, part++ | (lo << 20) | (hi << 25)));
    }
  }
  order_degrid_items(S.p6.begin() + first_p6, S.p6.end());
  // gridding: first the item that stores the pass's scalar factor, then the chunks heaviest
  // first so the tail is short, a chunk item carrying its entry range; the grid pass takes the
  // small chunks eight to an item {prob, kGridSmallItem, first of small_ids, count}, the fused
  // de-grid + grid pass every chunk as an item of its own
  const Geometry* geo = &g;
  const size_t first = S.p7.size(), first_f = S.p7f.size();
  S.p7.push_back(make_int4(prob, kGridFactorItem, 0, 0));
  S.p7f.push_back(make_int4(prob, kGridFactorItem, 0, 0));
  for (size_t c = 0; c < g.chunks.size(); ++c) {
    const int4 item = make_int4(prob, (int)c, g.chunk_ent[c].x, g.chunk_ent[c].y);
    S.p7f.push_back(item);
    if (item.w - item.z > kSmallChunk) S.p7.push_back(item);
  }
  const int ns = (int)g.small_ids.size(), per = kGridThreads / 64;
  for (int i = 0; i < ns; i += per) S.p7.push_back(make_int4(prob, kGridSmallItem, i, std::min(per, ns - i)));
  order_grid_items(S.p7.begin() + first, S.p7.end(), [geo](int) { return geo; });
  order_grid_items(S.p7f.begin() + first_f, S.p7f.end(), [geo](int) { return geo; });
  *n_p6 = part;
}

// Tile order of the SARA work lists.  Workgroups are dealt to the eight XCDs in turn, so a
// list whose j-th item takes tile xcd_tiles(tps)[j] runs every tile of one horizontal band
// (an eighth of the tile rows) on the same XCD, where neighbouring tiles share the L2 lines of
// their overlapping halos; the per-basis lists (a multiple of eight items each) keep every
// basis of a tile on its band's XCD.  The identity where the tile rows do not split into
// eight bands.
static std::vector<int> xcd_tiles(int tps) {
  std::vector<int> ord(tps * tps);
  std::iota(ord.begin(), ord.end(), 0);
  if (tps % 8 != 0) return ord;
  const int per = tps * tps / 8;                   // tiles per band, row-major
  for (int j = 0; j < per; ++j)
    for (int b = 0; b < 8; ++b) ord[j * 8 + b] = b * per + j;
  return ord;
}

void add_prior_items(ItemSet& S, int prob, int n, int levels, int nwav, const int* wav_len, bool fp64, int c_level,
                     int ana_wide, int* n_ana_parts) {
  const int N = n * n;
  const bool wide = (ana_wide & kAnaWide) != 0;
  // kAnaAllBases: the iterations' level-1 dual items take every basis of a tile at once
  const bool all_bases = (ana_wide & kAnaAllBases) != 0 && nwav > 0 && 1 < c_level;
  int part = 0;
  for (int b = 0; b < (N + 255) / 256; ++b) S.dirac.push_back(make_int4(prob, b, 0, part++));
  for (int l = 1; l <= levels; ++l) {
    const int h = n >> l;
    const int to = fp64 ? dwt_ana_tile<double>(h, wide) : dwt_ana_tile<float>(h, wide), tps = h / to;
    const std::vector<int> ord = xcd_tiles(tps);
    for (int w = 0; w < nwav; ++w)
      for (int t : ord) {
        S.ana[l].push_back(make_int4(prob, w, t, part + w * tps * tps + t));   // partials in tile order
        if (l < c_level && !(l == 1 && all_bases)) S.ana_d[l].push_back(S.ana[l].back());
      }
    part += nwav * tps * tps;
    if (l == 1 && all_bases)
      for (int t : ord) S.ana_d[1].push_back(make_int4(prob, kAllBases, t, 0));
  }
  for (int l = 2; l <= levels; ++l) {
    const int m = n >> (l - 1);
    const int to = fp64 ? dwt_syn_tile<double>(m) : dwt_syn_tile<float>(m), tps = m / to;
    const std::vector<int> ord = xcd_tiles(tps);
    for (int w = 0; w < nwav; ++w)
      for (int t : ord) {
        S.syn[l].push_back(make_int4(prob, w, t, 0));
        if (l < c_level) S.syn_d[l].push_back(S.syn[l].back());
      }
  }
  // the coarse items channel-major over eight basis places (an empty place is an item with
  // basis -1, which does nothing): workgroups are dealt to the eight XCDs in turn, so the four
  // channel workgroups of a basis run on one XCD and share its L2 lines (each reads and writes
  // one component of the same four-component elements); a problem's 32 items keep the
  // alignment when a batch concatenates the lists
  static_assert(kMaxBases - 1 <= 8, "eight basis places");
  if (c_level <= levels)
    for (int ch = 0; ch < 4; ++ch)
      for (int w = 0; w < 8; ++w) S.coarse.push_back(make_int4(prob, w < nwav ? w : -1, ch, c_level));
  {
    const int to = fp64 ? dwt_syn_tile<double>(n) : dwt_syn_tile<float>(n), tps = n / to;
    // the split: longest filters first, each to the lighter part (work ~ filter length plus the
    // window fetch, taken as 8 taps)
    std::vector<int> order(nwav);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return wav_len[a] > wav_len[b]; });
    int mask[2] = {0, 0}, work[2] = {0, 0};
    for (int w : order) {
      const int p = work[1] < work[0] ? 1 : 0;
      mask[p] |= 1 << w;
      work[p] += wav_len[w] + 8;
    }
    const int all = (1 << nwav) - 1;
    const std::vector<int> ord = xcd_tiles(tps);
    for (int t : ord) S.synfinal.push_back(make_int4(prob, t, 0, all));
    if (nwav < 2) {
      for (int t : ord) S.synsplit.push_back(make_int4(prob, t, 0, all));
    } else {
      for (int p = 0; p < 2; ++p)
        for (int t : ord) S.synsplit.push_back(make_int4(prob, t, p, mask[p]));
    }
  }
  *n_ana_parts = part;
}

// ------------------------------------------------------------------------------------------------
// Engine<R>
template <typename R>
Engine<R>::Engine(const Geometry& g, hipStream_t stream) : geo_(g), s0_(stream) {
  hip_check(hipStreamCreateWithFlags(&s1_, hipStreamNonBlocking), "hipStreamCreate");
  hip_check(hipEventCreateWithFlags(&ev_fork_, hipEventDisableTiming), "hipEventCreate");
  hip_check(hipEventCreateWithFlags(&ev_join_, hipEventDisableTiming), "hipEventCreate");
  std::memset(&h_, 0, sizeof(h_));
  const int n = g.n, K = g.K, N = n * n;
  const int64_t M = g.M;
  cells_ = std::max(512, K);
  rcells_ = std::max(512, K);
  h_.n = n; h_.K = K; h_.T = g.T; h_.M = M;
  h_.ts = g.ts; h_.ntile_side = g.nts; h_.ntile_side_g = g.ntsg;
  h_.deg = KbDeg<R>::value;
  for (int s = 0; s < IMG_Z; ++s) h_.img[s] = dalloc<V4<R>>(N);
  h_.img[IMG_Z] = dalloc<V2<R>>(N);
  h_.img[IMG_D] = dalloc<V2<R>>(N);
  for (int s = 0; s < NUM_VIS; ++s) h_.vis[s] = dalloc<Cell<R>>(M);
  h_.grid = dalloc<Cell<R>>((size_t)K * K);
  h_.half = dalloc<Cell<R>>((size_t)K * n);
  // geometry
  h_.vis_k0 = upload<int>(g.k0.data(), M);
  h_.vis_frac = upload_conv(g.frac.data(), 2 * M);
  h_.own_ptr = upload<int>(g.own_ptr.data(), g.own_ptr.size());
  upload_chunks();
  // tables
  std::vector<double> poly = kb_poly(g.T, g.beta, h_.deg);
  h_.kbpoly = upload_conv(poly.data(), poly.size());
  std::vector<double> tw(2 * K);
  for (int j = 0; j < K; ++j) {
    const double a = -2.0 * M_PI * (double)j / (double)K;
    tw[2 * j] = std::cos(a);
    tw[2 * j + 1] = std::sin(a);
  }
  h_.twiddle = upload_conv(tw.data(), tw.size());
  std::vector<double> s(n);
  for (int j = 0; j < n; ++j) s[j] = 1.0 / kb_hat(g.T, g.beta, (double)(j - n / 2) / (double)K);
  h_.deapod = upload_conv(s.data(), n);
  set_grid_kernel_limits<R>(g.ts, g.T);
  h_.dg_item = tuning_.degrid_item;
  h_.ana_wide = tuning_.ana_wide;
  // items of the operator passes
  build_operator_items();
  gen_parts_ = (N + 255) / 256;
  realloc_partials();
  h_.scal = dalloc<double>(NUM_SCALARS);
  zero(h_.scal, NUM_SCALARS * sizeof(double));
  zero_state();
  upload_items();
}

template <typename R>
Engine<R>::~Engine() {
  (void)hipStreamSynchronize(s0_);
  (void)hipStreamSynchronize(s1_);
  for (auto& kv : graphs_) if (kv.second) (void)hipGraphExecDestroy(kv.second);
  graphs_.clear();
  for (void* p : allocs_) (void)hipFree(p);
  if (h_active_) (void)hipHostFree(h_active_);
  for (hipEvent_t e : ev_active_) if (e) (void)hipEventDestroy(e);
  (void)hipEventDestroy(ev_fork_);
  (void)hipEventDestroy(ev_join_);
  (void)hipStreamDestroy(s1_);
}

template <typename R>
template <typename T>
T* Engine<R>::dalloc(size_t count) {
  void* p = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(&p, count * sizeof(T)) != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error(PSARA_ENOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
  }
  allocs_.push_back(p);
  bytes_ += count * sizeof(T);
  return (T*)p;
}

template <typename R>
void Engine<R>::dfree(void* p) {
  if (!p) return;
  auto it = std::find(allocs_.begin(), allocs_.end(), p);
  if (it != allocs_.end()) { allocs_.erase(it); (void)hipFree(p); }
}

template <typename R>
template <typename T>
T* Engine<R>::upload(const T* host, size_t count) {
  T* d = dalloc<T>(count);
  if (host) copy_sync(d, host, count * sizeof(T), hipMemcpyHostToDevice, s0_, "hipMemcpy H2D");
  else zero(d, std::max<size_t>(count, 1) * sizeof(T));   // an empty list's placeholder
  return d;
}

template <typename R>
R* Engine<R>::upload_conv(const double* host, size_t count) {
  std::vector<R> tmp(count);
  for (size_t i = 0; i < count; ++i) tmp[i] = (R)host[i];
  return upload<R>(tmp.data(), count);
}

template <typename R>
void Engine<R>::zero(void* p, size_t bytes) {
  hip_check(hipMemsetAsync(p, 0, bytes, s0_), "hipMemsetAsync");
}

template <typename R>
void Engine<R>::realloc_partials() {
  const int stride = std::max(gen_parts_, 1);
  h_.gen_stride = stride;
  const size_t count = 2 * ((size_t)h_.n_p6 + (size_t)kGenQ * stride + (size_t)h_.n_slots);
  if (h_.partials) dfree(h_.partials);
  h_.partials = dalloc<double>(count);
  zero(h_.partials, count * sizeof(double));
}

// Workgroups are dealt to the eight XCDs round-robin (workgroup b to XCD b % 8), each XCD with
// its own L2.  Reorders a work list so that every XCD takes one contiguous run of it: adjacent
// image rows, whose transposed accesses to the intermediate array share cache lines, then meet
// in the same L2 instead of fetching the same line into up to four of them.
static std::vector<int4> xcd_contiguous(const std::vector<int4>& v) {
  const size_t G = v.size(), q = G / 8, r = G % 8;
  std::vector<int4> out(G);
  for (size_t b = 0; b < G; ++b) {
    const size_t x = b % 8, j = b / 8;
    out[b] = v[x * q + std::min(x, r) + j];
  }
  return out;
}

// The geometry's runs, chunks and per-tile slot ranges on the device, with the partial slots.
template <typename R>
void Engine<R>::upload_chunks() {
  const Geometry& g = geo_;
  dfree((void*)h_.run_pack);
  dfree((void*)h_.chunk_ent); dfree((void*)h_.tile_slots); dfree((void*)h_.chunks); dfree((void*)h_.slot_box);
  dfree((void*)h_.tile_box); dfree((void*)h_.small_ids); dfree(h_.gpart);
  h_.run_pack = upload<int>(g.run_pack.data(), std::max<size_t>(1, g.run_pack.size()));
  h_.chunk_ent = upload<int2>(g.chunk_ent.data(), std::max<size_t>(1, g.chunk_ent.size()));
  h_.tile_slots = upload<int2>(g.tile_slots.data(), std::max<size_t>(1, g.tile_slots.size()));
  h_.chunks = upload<int4>(g.chunks.data(), std::max<size_t>(1, g.chunks.size()));
  h_.slot_box = upload<int>(g.slot_box.data(), std::max<size_t>(1, g.slot_box.size()));
  h_.tile_box = upload<int>(g.tile_box.data(), std::max<size_t>(1, g.tile_box.size()));
  h_.small_ids = upload<int>(g.small_ids.data(), std::max<size_t>(1, g.small_ids.size()));
  // the gridding writes only the cells of a slot's box; the rest stay zero from here on
  const size_t cells = (size_t)std::max(g.n_slots, 1) * (kGridTile + g.T - 1) * (kGridTile + g.T - 1);
  h_.gpart = dalloc<Cell<R>>(cells);
  zero(h_.gpart, cells * sizeof(Cell<R>));
  h_.n_slots = g.n_slots;
}

template <typename R>
void Engine<R>::build_operator_items() {
  items_.img.clear(); items_.rows.clear(); items_.cols.clear(); items_.p6.clear(); items_.p7.clear();
  items_.p7f.clear();
  add_operator_items(items_, 0, geo_, cells_, rcells_, tuning_.degrid_item, &h_.n_p6);
}

// The SARA work lists of the current prior (none for the TV priors or without a prior).
template <typename R>
void Engine<R>::build_prior_items() {
  const int N = geo_.n * geo_.n;
  items_.dirac.clear(); items_.synfinal.clear(); items_.synsplit.clear(); items_.coarse.clear();
  for (int l = 0; l <= kMaxLevels; ++l) {
    items_.ana[l].clear(); items_.syn[l].clear(); items_.ana_d[l].clear(); items_.syn_d[l].clear();
  }
  int nap = 0;
  if (h_.tv_kind == 0 && h_.coef[COEF_A] && h_.levels > 0)
    add_prior_items(items_, 0, geo_.n, h_.levels, h_.nwav, h_.wav_len, std::is_same<R, double>::value, c_level_,
                    tuning_.ana_wide, &nap);
  ana_parts_ = nap;
  gen_parts_ = std::max((N + 255) / 256, nap);
}

template <typename R>
void Engine<R>::set_tuning(const Tuning& t) {
  check_tuning(t, geo_.K);
  hip_check(hipStreamSynchronize(s0_), "tuning sync");
  hip_check(hipStreamSynchronize(s1_), "tuning sync");
  if (t.grid_chunk != geo_.chunk_entries) {
    build_grid_chunks(geo_, t.grid_chunk);
    upload_chunks();
  }
  tuning_ = t;
  cells_ = t.fft_cells ? t.fft_cells : std::max(512, geo_.K);
  rcells_ = cells_;
  h_.dg_item = t.degrid_item;
  h_.ana_wide = t.ana_wide;
  build_operator_items();
  build_prior_items();
  realloc_partials();
  upload_items();
  invalidate_graphs();
  hip_check(hipStreamSynchronize(s0_), "tuning");
}

template <typename R>
void Engine<R>::upload_items() {
  auto up = [&](DevItems& d, const std::vector<int4>& v) {
    if (d.ptr) dfree(d.ptr);
    d.ptr = nullptr;
    d.count = (int)v.size();
    if (!v.empty()) d.ptr = upload<int4>(v.data(), v.size());
  };
  up(d_img_, items_.img); up(d_rows_, xcd_contiguous(items_.rows)); up(d_cols_, items_.cols);
  up(d_p6_, items_.p6); up(d_p7_, items_.p7); up(d_p7f_, items_.p7f);
  up(d_dirac_, items_.dirac); up(d_synfinal_, items_.synfinal); up(d_synsplit_, items_.synsplit);
  up(d_coarse_, items_.coarse);
  for (int l = 0; l <= kMaxLevels; ++l) {
    up(d_ana_[l], items_.ana[l]); up(d_syn_[l], items_.syn[l]);
    up(d_ana_d_[l], items_.ana_d[l]); up(d_syn_d_[l], items_.syn_d[l]);
  }
  if (!d_desc_) d_desc_ = dalloc<ProbDesc>(1);
  desc_dirty_ = true;
  pl_.descs = d_desc_;
  pl_.img = d_img_; pl_.rows = d_rows_; pl_.cols = d_cols_; pl_.p6 = d_p6_; pl_.p7 = d_p7_; pl_.p7f = d_p7f_;
  pl_.synfinal = d_synsplit_; pl_.coarse = d_coarse_;
  for (int l = 0; l <= kMaxLevels; ++l) { pl_.ana_d[l] = d_ana_d_[l]; pl_.syn_d[l] = d_syn_d_[l]; }
  pl_.cells = cells_; pl_.rcells = rcells_;
  pl_.max_ts = geo_.ts; pl_.taps = geo_.T; pl_.max_levels = h_.levels;
  pl_.max_n = h_.n;
  pl_.ana_wide = tuning_.ana_wide;
  pl_.grid_ce = geo_.chunk_entries;
  pl_.sparse = h_.coef[COEF_A] != nullptr && h_.nwav > 0;
  pl_.tv = h_.tv_kind != 0;
}

template <typename R>
void Engine<R>::sync_desc() {
  if (!desc_dirty_) return;
  hip_check(hipMemcpyAsync(d_desc_, &h_, sizeof(ProbDesc), hipMemcpyHostToDevice, s0_), "desc upload");
  hip_check(hipStreamSynchronize(s0_), "desc upload sync");
  desc_dirty_ = false;
}

template <typename R>
void Engine<R>::zero_state() {
  const size_t N = (size_t)geo_.n * geo_.n;
  for (int s = 0; s < IMG_Z; ++s) zero(h_.img[s], N * sizeof(V4<R>));
  zero(h_.img[IMG_Z], N * sizeof(V2<R>));
  zero(h_.img[IMG_D], N * sizeof(V2<R>));
  zero(h_.vis[VIS_BV], (size_t)geo_.M * sizeof(Cell<R>));
  zero(h_.vis[VIS_R], (size_t)geo_.M * sizeof(Cell<R>));
  if (h_.coef[COEF_A]) zero(h_.coef[COEF_A], coef_elems_ * sizeof(V4<R>));
  zero(h_.scal, NUM_SCALARS * sizeof(double));
  hip_check(hipStreamSynchronize(s0_), "zero state");
}

template <typename R>
void Engine<R>::set_data(const double* Y_sorted, double eps) {
  const int64_t M = geo_.M;
  std::vector<R> tmp((size_t)M * 8);
  for (size_t i = 0; i < tmp.size(); ++i) tmp[i] = (R)Y_sorted[i];
  copy_sync(h_.vis[VIS_Y], tmp.data(), tmp.size() * sizeof(R), hipMemcpyHostToDevice, s0_, "Y upload");
  h_.eps = eps;
  desc_dirty_ = true;
}

template <typename R>
bool Engine<R>::set_data_dev(const double* Y_dev, double eps) {
  const int64_t M = geo_.M;
  if (M > std::numeric_limits<int>::max()) throw Error(PSARA_EINVAL, "too many rows for the device upload");
  if (!d_flag_) d_flag_ = dalloc<int>(1);
  if (!d_perm_) {
    std::vector<int> p((size_t)std::max<int64_t>(M, 1), 0);
    for (int64_t i = 0; i < M; ++i) p[(size_t)i] = (int)geo_.perm[(size_t)i];
    d_perm_ = upload<int>(p.data(), p.size());
  }
  zero(d_flag_, sizeof(int));
  launch_nonfinite(Y_dev, (size_t)M * 8, d_flag_, s0_);
  hip_check(hipGetLastError(), "finite check launch");
  int bad = 0;
  copy_sync(&bad, d_flag_, sizeof(int), hipMemcpyDeviceToHost, s0_, "finite check");
  if (bad) return false;
  launch_gather_rows<R>(Y_dev, d_perm_, h_.vis[VIS_Y], (long long)M, s0_);
  hip_check(hipGetLastError(), "Y gather launch");
  hip_check(hipStreamSynchronize(s0_), "Y gather");
  h_.eps = eps;
  desc_dirty_ = true;
  return true;
}

template <typename R>
void Engine<R>::set_mixing(const double* mix_sorted) {
  dfree((void*)h_.mix);
  h_.mix = nullptr;
  if (mix_sorted) h_.mix = upload_conv(mix_sorted, (size_t)geo_.M * 32);
  desc_dirty_ = true;
  zero_state();
}

template <typename R>
void Engine<R>::set_prior_tv(int kind, const double* tv_weight, const double* l1_weight) {
  const int n = geo_.n, N = n * n;
  set_prior(1u, 1, nullptr, 1.0);      // releases a previous prior; replaced below
  for (int c = 0; c < NUM_COEF; ++c) { dfree(h_.coef[c]); h_.coef[c] = nullptr; }
  items_.dirac.clear();
  for (int l = 0; l <= kMaxLevels; ++l) {
    items_.ana[l].clear(); items_.syn[l].clear(); items_.ana_d[l].clear(); items_.syn_d[l].clear();
  }
  items_.synfinal.clear(); items_.synsplit.clear(); items_.coarse.clear();
  h_.tv_kind = kind;
  for (int i = 0; i < 4; ++i) {
    h_.tvw[i] = tv_weight[i];
    h_.l1w[i] = (kind == 2 && l1_weight) ? l1_weight[i] : 0.0;
  }
  h_.has_dirac = 0; h_.nwav = 0; h_.nbases = 1; h_.levels = 0; h_.norm = 1.0; h_.gamma = 1.0;
  coef_elems_ = (size_t)(kind == 2 ? 3 : 2) * N;     // dual blocks [d1, d2] or [Dirac, d1, d2]
  for (int c = 0; c < NUM_COEF; ++c) h_.coef[c] = dalloc<V4<R>>(coef_elems_);
  for (int c = 0; c < NUM_COEF; ++c) zero(h_.coef[c], coef_elems_ * sizeof(V4<R>));
  ana_parts_ = 0;
  gen_parts_ = (N + 255) / 256;
  realloc_partials();
  upload_items();
  invalidate_graphs();
  zero(h_.img[IMG_PSIA], (size_t)N * sizeof(V4<R>));
  zero(h_.img[IMG_PSIA2], (size_t)N * sizeof(V4<R>));
  hip_check(hipStreamSynchronize(s0_), "set_prior_tv");
}

template <typename R>
void Engine<R>::set_prior(uint32_t mask, int levels, const double* weights, double gamma) {
  const int n = geo_.n, N = n * n;
  h_.tv_kind = 0;
  // release a previous prior
  for (int c = 0; c < NUM_COEF; ++c) { dfree(h_.coef[c]); h_.coef[c] = nullptr; }
  dfree(h_.ll); h_.ll = nullptr;
  dfree((void*)h_.filters); h_.filters = nullptr;
  items_.dirac.clear(); items_.synfinal.clear(); items_.synsplit.clear(); items_.coarse.clear();
  for (int l = 0; l <= kMaxLevels; ++l) {
    items_.ana[l].clear(); items_.syn[l].clear(); items_.ana_d[l].clear(); items_.syn_d[l].clear();
  }
  h_.has_dirac = (mask & 1u) ? 1 : 0;
  int nwav = 0;
  std::vector<double> filt(8 * kMaxFilter, 0.0);
  for (int p = 1; p <= 8; ++p)
    if (mask & (1u << p)) {
      std::vector<double> hf = daubechies(p);
      for (int j = 0; j < 2 * p; ++j) filt[nwav * kMaxFilter + j] = hf[j];
      h_.wav_len[nwav] = 2 * p;
      ++nwav;
    }
  h_.nwav = nwav;
  h_.nbases = nwav + h_.has_dirac;
  h_.levels = levels;
  h_.norm = 1.0 / std::sqrt((double)h_.nbases);
  h_.gamma = gamma;
  h_.filters = upload_conv(filt.data(), filt.size());
  coef_elems_ = (size_t)h_.nbases * N;
  for (int c = 0; c < NUM_COEF; ++c) h_.coef[c] = dalloc<V4<R>>(coef_elems_);
  long long off = 0;
  h_.ll_off[0] = 0;
  for (int l = 1; l <= kMaxLevels; ++l) {
    h_.ll_off[l] = off;
    if (l < levels) off += (long long)(n >> l) * (n >> l);
  }
  h_.ll_stride = std::max<long long>(off, 1);
  h_.ll = dalloc<V4<R>>((size_t)std::max(nwav, 1) * h_.ll_stride);
  // thresholds gamma * W
  std::vector<R> gw(coef_elems_ * 4);
  for (size_t i = 0; i < gw.size(); ++i) gw[i] = (R)(gamma * (weights ? weights[i] : 1.0));
  copy_sync(h_.coef[COEF_GW], gw.data(), gw.size() * sizeof(R), hipMemcpyHostToDevice, s0_, "weights upload");
  zero(h_.coef[COEF_A], coef_elems_ * sizeof(V4<R>));
  c_level_ = coarse_level<R>(n, levels);
  build_prior_items();
  realloc_partials();
  upload_items();
  invalidate_graphs();
  // the state's Psi A is zero again
  zero(h_.img[IMG_PSIA], (size_t)N * sizeof(V4<R>));
  zero(h_.img[IMG_PSIA2], (size_t)N * sizeof(V4<R>));
  hip_check(hipStreamSynchronize(s0_), "set_prior");
}

template <typename R>
void Engine<R>::set_steps(double tau, double r1, double r2, double r3) {
  h_.tau = tau; h_.rho1 = r1; h_.rho2 = r2; h_.rho3 = r3;
  desc_dirty_ = true;
}

template <typename R>
LaunchArgs Engine<R>::la(const DevItems& d, hipStream_t s) const {
  LaunchArgs a;
  a.descs = d_desc_;
  a.items = d.ptr;
  a.nitems = d.count;
  a.stream = s ? s : s0_;
  a.max_n = h_.n;
  a.ana_wide = tuning_.ana_wide;
  a.grid_ce = geo_.chunk_entries;
  return a;
}

// ---- passes --------------------------------------------------------------------------------------
template <typename R> void Engine<R>::p1(int mode, hipStream_t s) { launch_primal<R>(mode, la(d_img_, s)); }
template <typename R> void Engine<R>::p2(hipStream_t s) {
  for (int l = 1; l <= h_.levels; ++l) launch_analysis<R>(AM_DUAL, l, la(d_ana_[l], s), IMG_X, COEF_A);
}
template <typename R> void Engine<R>::p3(int src_coef, int dst_slot, int add_dirac, hipStream_t s) {
  for (int l = h_.levels; l >= 2; --l) launch_synthesis<R>(l, h_.levels, la(d_syn_[l], s), src_coef, 0);
  launch_synthesis_final<R>(la(d_synfinal_, s), src_coef, dst_slot, add_dirac, dst_slot);
}
template <typename R> void Engine<R>::p23(hipStream_t s) { launch_sara_dual<R>(pl_, s ? s : s0_); }

// ---- the iteration over a set of problems -------------------------------------------------------
static LaunchArgs lists_la(const PassLists& L, const DevItems& d, hipStream_t s) {
  LaunchArgs a;
  a.descs = L.descs;
  a.items = d.ptr;
  a.nitems = d.count;
  a.stream = s;
  a.max_n = L.max_n;
  a.ana_wide = L.ana_wide;
  a.grid_ce = L.grid_ce;
  return a;
}

template <typename R>
void launch_sara_dual(const PassLists& L, hipStream_t s) {
  for (int l = 1; l <= L.max_levels; ++l) launch_analysis<R>(AM_DUAL, l, lists_la(L, L.ana_d[l], s), IMG_X, COEF_A);
  launch_coarse<R>(lists_la(L, L.coarse, s));
  for (int l = L.max_levels; l >= 2; --l) launch_synthesis<R>(l, L.max_levels, lists_la(L, L.syn_d[l], s), COEF_A, 0);
  launch_synthesis_final<R>(lists_la(L, L.synfinal, s), COEF_A, IMG_PSIA, 0, IMG_PSIA2);
}

// Whether the iterations of `mode` run P6 and P7 as one fused pass: only when no SARA branch runs
// beside them (the initialisation stage, Algorithm 3).  Alone the fused pass is the faster
// (one launch, 50 against 26 + 32 us on the 256^2 / 2e5 workload), but beside the SARA kernels
// its large workgroups share the CUs worse than the two separate passes, and the iteration is
// about 5 % slower with it.
inline bool fused_p6_p7(const PassLists& L, int mode) { return pm_tv(mode) || mode == PM_INIT || !L.sparse; }

// P6, P7 and P8 of one iteration (the dual B step or Algorithm 3's residual, its gridding, and
// the column inverse FFT, which takes the factor of the gridded values from the partials of the
// fused pass, as one for the TV residual, or as the grid pass stored it)
template <typename R>
void launch_p6_p8(const PassLists& L, int mode, hipStream_t s) {
  const bool tvm = pm_tv(mode);
  if (fused_p6_p7(L, mode)) {
    if (tvm) launch_degrid_grid<R>(GR_STOKES, lists_la(L, L.p7f, s), L.taps, VIS_Y, VIS_R);
    else launch_degrid_grid<R>(GR_DUAL, lists_la(L, L.p7f, s), L.taps, VIS_BV, VIS_BV);
    launch_fft<R>(2, lists_la(L, L.cols, s), L.cells, tvm ? 2 : 1, 0);
  } else {
    launch_degrid<R>(DG_DUAL, lists_la(L, L.p6, s), L.max_ts, L.taps, VIS_BV, VIS_BV);
    launch_grid<R>(GR_DUAL, lists_la(L, L.p7, s), L.taps, VIS_BV, 0);
    launch_fft<R>(2, lists_la(L, L.cols, s), L.cells, 0, 0);
  }
}

template <typename R>
void launch_iterations(const PassLists& L, int mode, int count, hipStream_t s0, hipStream_t s1, hipEvent_t fork,
                       hipEvent_t join) {
  if (count <= 0) return;
  // P1 fused into P4: the row-FFT workgroups run the primal step of their rows
  launch_primal_fft<R>(mode, lists_la(L, L.rows, s0), L.rcells);
  // Algorithm 3 (TV modes): the sparsity branch is the TV dual step and its synthesis, and
  // P5..P8 evaluate the data term's gradient at S_new (the row FFT after the primal step
  // transforms S_new): residual Phi S - Y L^{-1} per Stokes map, gridded without mixing
  const bool tvm = pm_tv(mode);
  const bool sparse = tvm || ((mode != PM_INIT) && L.sparse);
  for (int k = 0; k < count; ++k) {
    // P5 is captured before the other branch's launches (it depends on the same row pass): the
    // graph then issues it first, and the branch with less slack starts earlier
    if (sparse) hip_check(hipEventRecord(fork, s0), "event record");
    launch_fft<R>(1, lists_la(L, L.cols, s0), L.cells, 0, 0);                        // P5
    if (sparse) {
      hip_check(hipStreamWaitEvent(s1, fork, 0), "stream wait");
      if (tvm) {
        launch_tv_dual<R>(lists_la(L, L.img, s1));
        launch_tv_synth<R>(lists_la(L, L.img, s1));
      } else {
        launch_sara_dual<R>(L, s1);
      }
      hip_check(hipEventRecord(join, s1), "event record");
    }
    launch_p6_p8<R>(L, mode, s0);
    if (sparse) hip_check(hipStreamWaitEvent(s0, join, 0), "stream wait");
    if (k + 1 < count) launch_fused_rows<R>(mode, lists_la(L, L.rows, s0), L.rcells);  // P9 + next P1, P4
    else launch_fft<R>(3, lists_la(L, L.rows, s0), L.rcells, 0, IMG_PHIB);          // P9
  }
}
// The stopping quantities of Sec. 4.6 for every problem in L, into each problem's scalars,
// with no host synchronisation: the residual ||phi(S) - Y||^2, N_p (its threshold zeta from the
// residual image Re phi^dagger (Y - phi(S))), and the relative variation of the last iteration
// from S and X = 2 S_new - S_old.  Uses the grid, VIS_R and IMG_TMP, none of which carries
// iteration state between the iterations of a chain.
template <typename R>
void launch_check(const PassLists& L, int nprob, hipStream_t s) {
  launch_fft<R>(0, lists_la(L, L.rows, s), L.rcells, IMG_S, 0);                       // phi(S)
  launch_fft<R>(1, lists_la(L, L.cols, s), L.cells, 0, 0);
  launch_degrid<R>(DG_RESIDUAL, lists_la(L, L.p6, s), L.max_ts, L.taps, VIS_BV, VIS_R);
  launch_finalize(L.descs, nprob, -1, 0, SC_RES2, s);
  launch_grid<R>(GR_PLAIN, lists_la(L, L.p7, s), L.taps, VIS_R, 0);                   // phi^dagger
  launch_fft<R>(2, lists_la(L, L.cols, s), L.cells, 0, 0);
  launch_fft<R>(3, lists_la(L, L.rows, s), L.rcells, 0, IMG_TMP);
  launch_img_sumsq<R>(lists_la(L, L.img, s), IMG_TMP, 0, 0);
  launch_finalize(L.descs, nprob, 0, -1, SC_RIMG2, s);
  launch_finalize_zeta(L.descs, nprob, s);
  launch_npcount<R>(lists_la(L, L.img, s));
  launch_finalize(L.descs, nprob, 0, -1, SC_NPCOUNT, s);
  launch_relvar<R>(lists_la(L, L.img, s));
  for (int q = 0; q < 4; ++q) {
    launch_finalize(L.descs, nprob, q, -1, SC_RV0 + q, s);
    launch_finalize(L.descs, nprob, 4 + q, -1, SC_SN0 + q, s);
  }
}

// Host side of an adaptive run: launches chunks of `check_every` iterations, each followed by
// the check and the decision, and looks at the number of running problems one chunk behind (an
// asynchronous copy into pinned memory), so it never waits for the chunk it has just queued;
// chunks queued after every problem has halted do nothing.  `graph(k)` returns the captured
// chunk of k iterations.  Returns when the work has drained.
template <class G>
void adaptive_loop(G&& graph, int max_iters, int check_every, hipStream_t s, int* d_active, int* h_active,
                   hipEvent_t* ev) {
  int left = max_iters, c = 0;
  bool done = false;
  while (left > 0 && !done) {
    const int k = std::min(left, check_every);
    hip_check(hipGraphLaunch(graph(k), s), "graph launch");
    hip_check(hipMemcpyAsync(h_active + (c & 1), d_active, sizeof(int), hipMemcpyDeviceToHost, s), "active D2H");
    hip_check(hipEventRecord(ev[c & 1], s), "event record");
    left -= k;
    if (c >= 1) {
      hip_check(hipEventSynchronize(ev[(c - 1) & 1]), "event sync");
      done = h_active[(c - 1) & 1] == 0;
    }
    ++c;
  }
  hip_check(hipStreamSynchronize(s), "adaptive sync");
}

template void launch_iterations<float>(const PassLists&, int, int, hipStream_t, hipStream_t, hipEvent_t, hipEvent_t);
template void launch_iterations<double>(const PassLists&, int, int, hipStream_t, hipStream_t, hipEvent_t, hipEvent_t);
template void launch_sara_dual<float>(const PassLists&, hipStream_t);
template void launch_sara_dual<double>(const PassLists&, hipStream_t);
template <typename R> void Engine<R>::p4(int src, hipStream_t s) { launch_fft<R>(0, la(d_rows_, s), rcells_, src, 0); }
template <typename R> void Engine<R>::p5(hipStream_t s) { launch_fft<R>(1, la(d_cols_, s), cells_, 0, 0); }
template <typename R> void Engine<R>::p6(int mode, int src, int out, hipStream_t s) {
  launch_degrid<R>(mode, la(d_p6_, s), geo_.ts, geo_.T, src, out);
}
template <typename R> void Engine<R>::p7(int mode, int src, int use_cfac, hipStream_t s) {
  launch_grid<R>(mode, la(d_p7_, s), geo_.T, src, use_cfac);
}
template <typename R> void Engine<R>::p8(hipStream_t s) { launch_fft<R>(2, la(d_cols_, s), cells_, 0, 0); }
template <typename R> void Engine<R>::p9(int dst, hipStream_t s) { launch_fft<R>(3, la(d_rows_, s), rcells_, 0, dst); }

template <typename R>
void Engine<R>::forward(int src_img, int mode, int out_vis) {
  p4(src_img); p5(); p6(mode, VIS_BV, out_vis);
}
template <typename R>
void Engine<R>::adjoint(int src_vis, int use_cfac, int dst_img) {
  p7(GR_PLAIN, src_vis, use_cfac); p8(); p9(dst_img);
}

// Algorithm 3 keeps, between iterations, the data term's gradient Re phi~^dagger (phi~ S - Y~)
// where Algorithm 1 keeps Re phi^dagger B, and Psi A; both are recomputed from the state before
// a run, since the state (S, A) may have been set or reset since the last one.
template <typename R>
void Engine<R>::prime(int mode) {
  if (!pm_tv(mode)) return;
  sync_desc();
  launch_fft<R>(0, la(d_rows_), rcells_, IMG_S, 0);
  p5();
  p6(DG_STOKES, VIS_Y, VIS_R);
  p7(GR_STOKES, VIS_R, 0);
  p8();
  p9(IMG_PHIB);
  launch_tv_synth<R>(la(d_img_));
  hip_check(hipGetLastError(), "prime");
}

template <typename R>
void Engine<R>::launch_iterations(int mode, int count) {
  ::psara::launch_iterations<R>(pl_, mode, count, s0_, s1_, ev_fork_, ev_join_);
}

template <typename R>
void Engine<R>::stop_begin(const double* stop, int max_iters) {
  sync_desc();
  const double v[6] = {0.0, 0.0, stop[0], stop[1], stop[2], (double)max_iters};   // SC_HALT .. SC_STOP_MAXIT
  copy_sync(h_.scal + SC_HALT, v, sizeof(v), hipMemcpyHostToDevice, s0_, "stop set-up");
}

template <typename R>
void Engine<R>::stop_poll(bool* halted_out, int* iters) {
  double v[2] = {0.0, 0.0};                                     // SC_HALT, SC_ITERS
  copy_sync(v, h_.scal + SC_HALT, sizeof(v), hipMemcpyDeviceToHost, s0_, "stop read");
  *halted_out = v[0] != 0.0;
  *iters = (int)v[1];
}

template <typename R>
int Engine<R>::stop_end() {
  double v[2] = {0.0, 0.0};                                     // SC_HALT, SC_ITERS
  copy_sync(v, h_.scal + SC_HALT, sizeof(v), hipMemcpyDeviceToHost, s0_, "stop read");
  const double z = 0.0;
  copy_sync(h_.scal + SC_HALT, &z, sizeof(z), hipMemcpyHostToDevice, s0_, "stop reset");
  return (int)v[1];
}

template <typename R>
void Engine<R>::adaptive_buffers() {
  if (!d_active_) d_active_ = dalloc<int>(1);
  if (!h_active_) {
    void* p = nullptr;
    if (hipHostMalloc(&p, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess || !p) {
      (void)hipGetLastError();
      throw Error(PSARA_ENOMEM, "pinned host allocation failed");
    }
    h_active_ = (int*)p;
    for (int i = 0; i < 2; ++i) hip_check(hipEventCreateWithFlags(&ev_active_[i], hipEventDisableTiming), "event");
  }
}

template <typename R>
int Engine<R>::run_adaptive(int mode, int max_iters, int check_every, const double* stop) {
  adaptive_buffers();
  stop_begin(stop);
  if (max_iters > 0) prime(mode);
  auto graph = [&](int count) -> hipGraphExec_t {
    const uint64_t key = graph_key(true, mode, count);
    auto it = graphs_.find(key);
    if (it != graphs_.end()) return it->second;
    hipGraph_t g = nullptr;
    hip_check(hipStreamBeginCapture(s0_, hipStreamCaptureModeRelaxed), "begin capture");
    launch_iterations(mode, count);
    launch_check<R>(pl_, 1, s0_);
    launch_stop_decide(d_desc_, 1, count, d_active_, s0_);
    hip_check(hipStreamEndCapture(s0_, &g), "end capture");
    hipGraphExec_t exec = nullptr;
    hip_check(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0), "graph instantiate");
    (void)hipGraphDestroy(g);
    graphs_[key] = exec;
    return exec;
  };
  adaptive_loop(graph, max_iters, check_every, s0_, d_active_, h_active_, ev_active_);
  return stop_end();
}

template <typename R>
void Engine<R>::invalidate_graphs() {
  for (auto& kv : graphs_) if (kv.second) (void)hipGraphExecDestroy(kv.second);
  graphs_.clear();
}

template <typename R>
hipGraphExec_t Engine<R>::chain_graph(int mode, int count) {
  const uint64_t key = graph_key(false, mode, count);
  auto it = graphs_.find(key);
  if (it != graphs_.end()) return it->second;
  hipGraph_t graph = nullptr;
  hip_check(hipStreamBeginCapture(s0_, hipStreamCaptureModeRelaxed), "begin capture");
  launch_iterations(mode, count);
  hip_check(hipStreamEndCapture(s0_, &graph), "end capture");
  hipGraphExec_t exec = nullptr;
  hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate");
  (void)hipGraphDestroy(graph);
  graphs_[key] = exec;
  return exec;
}

// A run of `iters` iterations replays chains of kChain captured iterations (the chain's first
// and last iterations run the unfused row passes, and each launch costs a few microseconds),
// then one chain of the remaining iters mod kChain; so every run length uses at most two graphs,
// whose per-iteration cost differs little.
template <typename R>
void Engine<R>::capture(int mode, int iters) {
  sync_desc();
  if (iters >= kChain) chain_graph(mode, kChain);
  if (iters % kChain) chain_graph(mode, iters % kChain);
}

template <typename R>
void Engine<R>::run(int mode, int iters) {
  sync_desc();
  if (iters <= 0) return;
  prime(mode);
  int left = iters;
  if (left >= kChain) {
    hipGraphExec_t g = chain_graph(mode, kChain);
    while (left >= kChain) { hip_check(hipGraphLaunch(g, s0_), "graph launch"); left -= kChain; }
  }
  if (left > 0) hip_check(hipGraphLaunch(chain_graph(mode, left), s0_), "graph launch");
  hip_check(hipGetLastError(), "iteration launch");
}

template <typename R>
size_t Engine<R>::scratch_bytes() const {
  const size_t rg = kGridTile + geo_.T - 1;
  const size_t slots = (size_t)std::max(geo_.n_slots, 1) * rg * rg * sizeof(Cell<R>);
  const size_t parts = 2 * ((size_t)h_.n_p6 + (size_t)kGenQ * h_.gen_stride + (size_t)h_.n_slots) * sizeof(double);
  return ((slots + 255) & ~(size_t)255) + parts;
}

template <typename R>
void Engine<R>::run_in_scratch(int mode, int iters, void* scr, size_t cap) {
  const size_t need = scratch_bytes();
  if (need > cap)
    throw Error(PSARA_EINVAL, "this problem needs " + std::to_string(need) + " bytes of iteration scratch, more than the " +
                                  std::to_string(cap) + " the allocation-free entry point holds");
  sync_desc();
  void* own_gpart = h_.gpart;
  double* own_partials = h_.partials;
  const size_t rg = kGridTile + geo_.T - 1;
  const size_t slots = (size_t)std::max(geo_.n_slots, 1) * rg * rg * sizeof(Cell<R>);
  h_.gpart = scr;
  h_.partials = (double*)((unsigned char*)scr + ((slots + 255) & ~(size_t)255));
  desc_dirty_ = true;
  try {
    sync_desc();
    // the gridding writes only the cells of each slot's box and the column inverse FFT reads
    // the rest of a tile's region as zero, so the slots are cleared, and the partial sums with
    // them, by a kernel (so the call records no memset node when a caller captures it)
    launch_fill<double>(scr, need / sizeof(double), s0_);
    if (iters > 0) prime(mode);
    launch_iterations(mode, iters);
    hip_check(hipGetLastError(), "iteration launch");
  } catch (...) {
    h_.gpart = own_gpart;
    h_.partials = own_partials;
    desc_dirty_ = true;
    throw;
  }
  h_.gpart = own_gpart;
  h_.partials = own_partials;
  desc_dirty_ = true;
  sync_desc();          // queued after the iterations; waits for them
}

template <typename R>
void Engine<R>::run_eager(int mode, int iters) {
  sync_desc();
  if (iters > 0) prime(mode);
  launch_iterations(mode, iters);
  hip_check(hipGetLastError(), "iteration launch");
}

// ---- reductions ---------------------------------------------------------------------------------
template <typename R>
void Engine<R>::finalize(int q, int count, int scalar) { launch_finalize(d_desc_, 1, q, count, scalar, s0_); }

template <typename R>
void Engine<R>::read_scalars(double* out) {
  hip_check(hipMemcpyAsync(out, h_.scal, NUM_SCALARS * sizeof(double), hipMemcpyDeviceToHost, s0_), "scalars D2H");
  hip_check(hipStreamSynchronize(s0_), "scalars sync");
}

template <typename R>
void Engine<R>::write_scalar(int idx, double v) {
  hip_check(hipMemcpyAsync(h_.scal + idx, &v, sizeof(double), hipMemcpyHostToDevice, s0_), "scalar H2D");
  hip_check(hipStreamSynchronize(s0_), "scalar sync");
}

template <typename R>
void Engine<R>::report(psara_report* r) {
  sync_desc();
  const int nimg = d_img_.count;
  // residual ||phi(S) - Y|| and the residual image
  forward(IMG_S, DG_RESIDUAL, VIS_R);
  finalize(-1, 0, SC_RES2);
  adjoint(VIS_R, 0, IMG_TMP);
  launch_img_sumsq<R>(la(d_img_), IMG_TMP, 0, 0);
  finalize(0, nimg, SC_RIMG2);
  launch_finalize_zeta(d_desc_, 1, s0_);
  launch_npcount<R>(la(d_img_));
  finalize(0, nimg, SC_NPCOUNT);
  launch_relvar<R>(la(d_img_));
  for (int q = 0; q < 4; ++q) { finalize(q, nimg, SC_RV0 + q); finalize(4 + q, nimg, SC_SN0 + q); }
  const bool prior = h_.coef[COEF_A] != nullptr;
  if (h_.tv_kind) {
    launch_tv_objective<R>(la(d_img_));
    finalize(0, nimg, SC_OBJ);
  } else if (prior) {
    if (h_.has_dirac) launch_dirac<R>(AM_OBJECTIVE, la(d_dirac_), IMG_S, 0);
    for (int l = 1; l <= h_.levels; ++l) launch_analysis<R>(AM_OBJECTIVE, l, la(d_ana_[l]), IMG_S, 0);
    finalize(0, ana_parts_, SC_OBJ);
  }
  hip_check(hipGetLastError(), "report launch");
  double sc[NUM_SCALARS];
  read_scalars(sc);
  const double N = (double)geo_.n * geo_.n;
  r->residual = std::sqrt(std::max(sc[SC_RES2], 0.0));
  r->epsilon = h_.eps;
  for (int q = 0; q < 4; ++q) {
    const double num = std::sqrt(sc[SC_RV0 + q]), den = std::sqrt(sc[SC_SN0 + q]);
    r->rel_var[q] = den > 0.0 ? num / den : INFINITY;
  }
  r->zeta = sc[SC_ZETA];
  r->n_p = 100.0 * sc[SC_NPCOUNT] / N;
  r->objective = h_.tv_kind ? sc[SC_OBJ] : (prior ? sc[SC_OBJ] / h_.gamma : 0.0);
  r->vnorm = std::sqrt(std::max(sc[SC_VNORM2], 0.0));
}

template <typename R>
double Engine<R>::coef_std() {
  sync_desc();
  if (h_.has_dirac) launch_dirac<R>(AM_MOMENTS, la(d_dirac_), IMG_S, 0);
  for (int l = 1; l <= h_.levels; ++l) launch_analysis<R>(AM_MOMENTS, l, la(d_ana_[l]), IMG_S, 0);
  finalize(0, ana_parts_, SC_MEAN);
  finalize(1, ana_parts_, SC_SQ);
  hip_check(hipGetLastError(), "moments launch");
  double sc[NUM_SCALARS];
  read_scalars(sc);
  const double cnt = 4.0 * (double)coef_elems_;
  const double mean = sc[SC_MEAN] / cnt;
  return std::sqrt(std::max(sc[SC_SQ] / cnt - mean * mean, 0.0));
}

template <typename R>
double Engine<R>::data_max_coef() {
  sync_desc();
  adjoint(VIS_Y, 0, IMG_TMP);
  if (h_.has_dirac) launch_dirac<R>(AM_MAXABS, la(d_dirac_), IMG_TMP, 0);
  for (int l = 1; l <= h_.levels; ++l) launch_analysis<R>(AM_MAXABS, l, la(d_ana_[l]), IMG_TMP, 0);
  launch_finalize_max(d_desc_, 1, 0, ana_parts_, SC_DOT, s0_);
  hip_check(hipGetLastError(), "max-coefficient launch");
  double sc[NUM_SCALARS];
  read_scalars(sc);
  return sc[SC_DOT];
}

template <typename R>
void Engine<R>::set_gamma(double gamma) {
  launch_scale<R>(h_.coef[COEF_GW], coef_elems_ * 4, gamma / h_.gamma, s0_);
  hip_check(hipGetLastError(), "threshold scale");
  hip_check(hipStreamSynchronize(s0_), "threshold scale sync");
  h_.gamma = gamma;
  desc_dirty_ = true;
}

template <typename R>
void Engine<R>::reweight(double delta) {
  h_.delta = delta;
  desc_dirty_ = true;
  sync_desc();
  if (h_.has_dirac) launch_dirac<R>(AM_REWEIGHT, la(d_dirac_), IMG_S, 0);
  for (int l = 1; l <= h_.levels; ++l) launch_analysis<R>(AM_REWEIGHT, l, la(d_ana_[l]), IMG_S, 0);
  hip_check(hipGetLastError(), "reweight launch");
  hip_check(hipStreamSynchronize(s0_), "reweight sync");
}

// FP64 power iteration of S -> Re phi^dagger phi S (Rayleigh quotient of a unit vector)
template <typename R>
double Engine<R>::opnorm(int max_iter, double rtol, int* iters_out) {
  sync_desc();
  const size_t N = (size_t)geo_.n * geo_.n;
  std::mt19937_64 rng(12345);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<R> x0(N * 4);
  for (auto& v : x0) v = (R)nd(rng);
  copy_sync(h_.img[IMG_TMP2], x0.data(), x0.size() * sizeof(R), hipMemcpyHostToDevice, s0_, "x0 upload");
  const int nimg = d_img_.count;
  launch_img_dot<R>(la(d_img_), IMG_TMP2, IMG_TMP2);
  finalize(1, nimg, SC_NRM2);
  launch_img_scale<R>(la(d_img_), IMG_TMP2, IMG_TMP2, SC_NRM2);
  double lam = 0.0;
  int it = 0;
  for (; it < max_iter; ++it) {
    forward(IMG_TMP2, DG_FORWARD, VIS_R);
    adjoint(VIS_R, 0, IMG_TMP);
    launch_img_dot<R>(la(d_img_), IMG_TMP2, IMG_TMP);
    finalize(0, nimg, SC_DOT);
    finalize(1, nimg, SC_NRM2);
    launch_img_scale<R>(la(d_img_), IMG_TMP2, IMG_TMP, SC_NRM2);
    hip_check(hipGetLastError(), "power iteration launch");
    double sc[NUM_SCALARS];
    read_scalars(sc);
    const double lam_new = sc[SC_DOT];
    if (it > 0 && std::fabs(lam_new - lam) <= rtol * std::fabs(lam_new)) { lam = lam_new; ++it; break; }
    lam = lam_new;
  }
  if (iters_out) *iters_out = it;
  return lam;
}

// ---- host <-> device images, coefficients, visibilities ------------------------------------------
template <typename R>
void Engine<R>::put_img(int slot, const double* src, int comps) {
  const size_t cnt = (size_t)geo_.n * geo_.n * comps;
  std::vector<R> tmp(cnt);
  for (size_t i = 0; i < cnt; ++i) tmp[i] = (R)src[i];
  copy_sync(h_.img[slot], tmp.data(), cnt * sizeof(R), hipMemcpyHostToDevice, s0_, "image upload");
}
template <typename R>
void Engine<R>::get_img(int slot, double* dst, int comps) {
  hip_check(hipStreamSynchronize(s0_), "sync");
  const size_t cnt = (size_t)geo_.n * geo_.n * comps;
  std::vector<R> tmp(cnt);
  copy_sync(tmp.data(), h_.img[slot], cnt * sizeof(R), hipMemcpyDeviceToHost, s0_, "image download");
  for (size_t i = 0; i < cnt; ++i) dst[i] = (double)tmp[i];
}
template <typename R>
void Engine<R>::get_img_dev(int slot, double* dst_dev, int comps) {
  hip_check(hipStreamSynchronize(s0_), "sync");
  launch_to_double<R>(h_.img[slot], dst_dev, (size_t)geo_.n * geo_.n * comps, s0_);
  hip_check(hipGetLastError(), "image conversion launch");
  hip_check(hipStreamSynchronize(s0_), "image conversion");
}
template <typename R>
void Engine<R>::put_coef(int slot, const double* src) {
  std::vector<R> tmp(coef_elems_ * 4);
  for (size_t i = 0; i < tmp.size(); ++i) tmp[i] = (R)src[i];
  copy_sync(h_.coef[slot], tmp.data(), tmp.size() * sizeof(R), hipMemcpyHostToDevice, s0_, "coef upload");
}
template <typename R>
void Engine<R>::get_coef(int slot, double* dst) {
  hip_check(hipStreamSynchronize(s0_), "sync");
  std::vector<R> tmp(coef_elems_ * 4);
  copy_sync(tmp.data(), h_.coef[slot], tmp.size() * sizeof(R), hipMemcpyDeviceToHost, s0_, "coef download");
  for (size_t i = 0; i < tmp.size(); ++i) dst[i] = (double)tmp[i];
}
// visibilities: caller order <-> sorted order, optional scale
template <typename R>
void Engine<R>::put_vis(int slot, const double* src) {
  const int64_t M = geo_.M;
  std::vector<R> tmp((size_t)M * 8);
  for (int64_t p = 0; p < M; ++p) {
    const double* s = src + 8 * geo_.perm[p];
    for (int k = 0; k < 8; ++k) tmp[8 * p + k] = (R)s[k];
  }
  copy_sync(h_.vis[slot], tmp.data(), tmp.size() * sizeof(R), hipMemcpyHostToDevice, s0_, "vis upload");
}
template <typename R>
void Engine<R>::get_vis(int slot, double* dst, double scale) {
  hip_check(hipStreamSynchronize(s0_), "sync");
  const int64_t M = geo_.M;
  std::vector<R> tmp((size_t)M * 8);
  copy_sync(tmp.data(), h_.vis[slot], tmp.size() * sizeof(R), hipMemcpyDeviceToHost, s0_, "vis download");
  for (int64_t p = 0; p < M; ++p) {
    double* d = dst + 8 * geo_.perm[p];
    for (int k = 0; k < 8; ++k) d[k] = scale * (double)tmp[8 * p + k];
  }
}

template <typename R>
void Engine<R>::apply_phi(const double* S, double* Y) {
  sync_desc();
  put_img(IMG_TMP, S, 4);
  forward(IMG_TMP, DG_FORWARD, VIS_R);
  hip_check(hipGetLastError(), "phi launch");
  get_vis(VIS_R, Y, 1.0);
}
template <typename R>
void Engine<R>::apply_phi_adjoint(const double* B, double* S) {
  sync_desc();
  put_vis(VIS_R, B);
  adjoint(VIS_R, 0, IMG_TMP);
  hip_check(hipGetLastError(), "phi adjoint launch");
  get_img(IMG_TMP, S, 4);
}
template <typename R>
void Engine<R>::apply_psi_adjoint(const double* S, double* A) {
  sync_desc();
  put_img(IMG_TMP, S, 4);
  if (h_.has_dirac) launch_dirac<R>(AM_STORE, la(d_dirac_), IMG_TMP, COEF_TMP);
  for (int l = 1; l <= h_.levels; ++l) launch_analysis<R>(AM_STORE, l, la(d_ana_[l]), IMG_TMP, COEF_TMP);
  hip_check(hipGetLastError(), "psi adjoint launch");
  get_coef(COEF_TMP, A);
}
template <typename R>
void Engine<R>::apply_psi(const double* A, double* S) {
  sync_desc();
  put_coef(COEF_TMP, A);
  p3(COEF_TMP, IMG_TMP, 1, s0_);
  hip_check(hipGetLastError(), "psi launch");
  get_img(IMG_TMP, S, 4);
}

// state: S, Z, A, B (caller order), C, D
template <typename R>
void Engine<R>::get_state(double* buf) {
  const size_t N = (size_t)geo_.n * geo_.n;
  double sc[NUM_SCALARS];
  read_scalars(sc);
  double* p = buf;
  get_img(IMG_S, p, 4); p += 4 * N;
  get_img(IMG_Z, p, 2); p += 2 * N;
  if (coef_elems_) get_coef(COEF_A, p);
  p += 4 * coef_elems_;
  get_vis(VIS_BV, p, sc[SC_CFAC]); p += 8 * (size_t)geo_.M;
  get_img(IMG_C, p, 4); p += 4 * N;
  get_img(IMG_D, p, 2);
}
template <typename R>
void Engine<R>::set_state(const double* buf) {
  sync_desc();
  const size_t N = (size_t)geo_.n * geo_.n;
  const double* p = buf;
  put_img(IMG_S, p, 4); put_img(IMG_X, p, 4); p += 4 * N;
  put_img(IMG_Z, p, 2); p += 2 * N;
  if (coef_elems_) put_coef(COEF_A, p);
  p += 4 * coef_elems_;
  put_vis(VIS_BV, p); p += 8 * (size_t)geo_.M;
  put_img(IMG_C, p, 4); p += 4 * N;
  put_img(IMG_D, p, 2);
  write_scalar(SC_CFAC, 1.0);
  // the two operator images the next primal step reads: Re phi^dagger(B) and the wavelet part of Psi A
  adjoint(VIS_BV, 1, IMG_PHIB);
  if (coef_elems_ && h_.nwav > 0) p3(COEF_A, IMG_PSIA, 0, s0_);
  else zero(h_.img[IMG_PSIA], N * sizeof(V4<R>));
  zero(h_.img[IMG_PSIA2], N * sizeof(V4<R>));
  hip_check(hipGetLastError(), "state prime");
  hip_check(hipStreamSynchronize(s0_), "set_state");
}

// Run `iters` iterations of every problem in L with every pass on stream s, bracketed by HIP
// events, and return the average duration of each pass (P1..P9, with P6 and P7 as separate
// passes) in milliseconds in ms[0..8]; then `iters` iterations in the captured graphs' order,
// returning the average durations of the fused P9 + P1 + P4 pass in ms[9] and, in the modes
// whose iterations fuse P6 and P7, of that pass in ms[10] (0 otherwise).
template <typename R>
void profile_iterations(const PassLists& L, int mode, int iters, hipStream_t s, double* ms) {
  constexpr int NP = 9;
  hipEvent_t ev[NP + 1];
  for (int i = 0; i <= NP; ++i) hip_check(hipEventCreate(&ev[i]), "event");
  for (int i = 0; i <= NP + 1; ++i) ms[i] = 0.0;
  const bool sparse = (mode != PM_INIT) && L.sparse;
  auto p5_p8 = [&](bool timed) {
    launch_fft<R>(1, lists_la(L, L.cols, s), L.cells, 0, 0);
    if (timed) hip_check(hipEventRecord(ev[5], s), "event record");
    launch_degrid<R>(DG_DUAL, lists_la(L, L.p6, s), L.max_ts, L.taps, VIS_BV, VIS_BV);
    if (timed) hip_check(hipEventRecord(ev[6], s), "event record");
    launch_grid<R>(GR_DUAL, lists_la(L, L.p7, s), L.taps, VIS_BV, 0);
    if (timed) hip_check(hipEventRecord(ev[7], s), "event record");
    launch_fft<R>(2, lists_la(L, L.cols, s), L.cells, 0, 0);
    if (timed) hip_check(hipEventRecord(ev[8], s), "event record");
  };
  // P5 .. P8 as the iterations run them, with the fused P6 + P7 pass timed where they use it
  const bool fused = fused_p6_p7(L, mode);
  auto p5_p8_run = [&]() {
    launch_fft<R>(1, lists_la(L, L.cols, s), L.cells, 0, 0);
    hip_check(hipEventRecord(ev[2], s), "event record");
    if (fused) launch_degrid_grid<R>(GR_DUAL, lists_la(L, L.p7f, s), L.taps, VIS_BV, VIS_BV);
    hip_check(hipEventRecord(ev[3], s), "event record");
    if (fused) launch_fft<R>(2, lists_la(L, L.cols, s), L.cells, 1, 0);
    else launch_p6_p8<R>(L, mode, s);
  };
  for (int k = 0; k < iters; ++k) {
    hip_check(hipEventRecord(ev[0], s), "event record");
    launch_primal_fft<R>(mode, lists_la(L, L.rows, s), L.rcells);   // P1 fused into P4: timed as P1
    hip_check(hipEventRecord(ev[1], s), "event record");
    if (sparse) launch_sara_dual<R>(L, s);   // P2 and P3 with the fused coarse levels: timed as P2
    hip_check(hipEventRecord(ev[2], s), "event record");
    p5_p8(true);
    launch_fft<R>(3, lists_la(L, L.rows, s), L.rcells, 0, IMG_PHIB);
    hip_check(hipEventRecord(ev[9], s), "event record");
    hip_check(hipEventSynchronize(ev[9]), "event sync");
    for (int i = 0; i < NP; ++i) {
      if (i == 2 || i == 3) continue;          // P3 runs inside P2's launches, P4 inside P1's
      float t = 0.f;
      hip_check(hipEventElapsedTime(&t, ev[i == 4 ? 2 : i], ev[i + 1]), "elapsed");
      ms[i] += t;
    }
  }
  for (int i = 0; i < NP; ++i) ms[i] /= std::max(iters, 1);
  // the pass fusing P9 with the next P1+P4, timed inside a chain of iterations in graph order
  if (iters > 0) launch_primal_fft<R>(mode, lists_la(L, L.rows, s), L.rcells);
  for (int k = 0; k < iters; ++k) {
    if (sparse) launch_sara_dual<R>(L, s);
    p5_p8_run();
    float t = 0.f;
    if (k + 1 < iters) {
      hip_check(hipEventRecord(ev[0], s), "event record");
      launch_fused_rows<R>(mode, lists_la(L, L.rows, s), L.rcells);
      hip_check(hipEventRecord(ev[1], s), "event record");
      hip_check(hipEventSynchronize(ev[1]), "event sync");
      hip_check(hipEventElapsedTime(&t, ev[0], ev[1]), "elapsed");
      ms[NP] += t;
    } else {
      launch_fft<R>(3, lists_la(L, L.rows, s), L.rcells, 0, IMG_PHIB);
      hip_check(hipEventSynchronize(ev[3]), "event sync");
    }
    if (fused) {
      hip_check(hipEventElapsedTime(&t, ev[2], ev[3]), "elapsed");
      ms[NP + 1] += t;
    }
  }
  if (iters > 1) ms[NP] /= iters - 1;
  if (iters > 0) ms[NP + 1] /= iters;
  hip_check(hipStreamSynchronize(s), "profile sync");
  for (int i = 0; i <= NP; ++i) (void)hipEventDestroy(ev[i]);
}

template <typename R>
void Engine<R>::profile(int mode, int iters, double* ms) {
  sync_desc();
  profile_iterations<R>(pl_, mode, iters, s0_, ms);
}

template struct Engine<float>;
template struct Engine<double>;

// ---- Batch<R> ------------------------------------------------------------------------------------
template <typename R>
Batch<R>::Batch(const std::vector<Engine<R>*>& members, hipStream_t stream) : members_(members), s0_(stream) {
  if (members_.empty()) throw Error(PSARA_EINVAL, "empty batch");
  const int T = members_[0]->geometry().T;
  // the FFT launches take the most cells per workgroup any member's tuning asks for (at least
  // the largest grid side); the gridding staging is sized for the largest chunk
  int cells = 512, max_ts = 0, max_levels = 0, max_n = 0, grid_ce = 0, ana_wide = 0;
  bool sparse = true;
  for (Engine<R>* e : members_) {
    const Geometry& g = e->geometry();
    if (g.T != T) throw Error(PSARA_EINVAL, "batch members must share the tap count");
    cells = std::max(cells, std::max(g.K, e->fft_cells()));
    max_ts = std::max(max_ts, g.ts);
    max_n = std::max(max_n, g.n);
    max_levels = std::max(max_levels, e->desc().levels);
    grid_ce = std::max(grid_ce, g.chunk_entries);
    ana_wide = ana_wide | e->tuning().ana_wide;
    sparse = sparse && e->has_prior();
  }
  ItemSet S;
  for (size_t i = 0; i < members_.size(); ++i) {
    Engine<R>* e = members_[i];
    const Geometry& g = e->geometry();
    int np6 = 0;
    add_operator_items(S, (int)i, g, cells, cells, e->tuning().degrid_item, &np6);
    if (np6 != e->desc().n_p6) throw Error(PSARA_EDEVICE, "inconsistent de-grid partition");
    if (e->has_prior()) {
      int nap = 0;
      add_prior_items(S, (int)i, g.n, e->desc().levels, e->desc().nwav, e->desc().wav_len,
                      std::is_same<R, double>::value, e->c_level(), e->tuning().ana_wide, &nap);
    }
  }
  // the gridding launches take the heaviest chunks of all members first
  order_degrid_items(S.p6.begin(), S.p6.end());
  order_grid_items(S.p7.begin(), S.p7.end(), [this](int prob) { return &members_[prob]->geometry(); });
  order_grid_items(S.p7f.begin(), S.p7f.end(), [this](int prob) { return &members_[prob]->geometry(); });
  auto up = [&](DevItems& d, const std::vector<int4>& v) {
    d.count = (int)v.size();
    d.ptr = nullptr;
    if (v.empty()) return;
    void* p = nullptr;
    if (hipMalloc(&p, v.size() * sizeof(int4)) != hipSuccess || !p) {
      (void)hipGetLastError();
      throw Error(PSARA_ENOMEM, "batch work-list allocation failed");
    }
    allocs_.push_back(p);
    copy_sync(p, v.data(), v.size() * sizeof(int4), hipMemcpyHostToDevice, s0_, "work-list upload");
    d.ptr = (int4*)p;
  };
  up(pl_.img, S.img); up(pl_.rows, xcd_contiguous(S.rows)); up(pl_.cols, S.cols);
  up(pl_.p6, S.p6); up(pl_.p7, S.p7); up(pl_.p7f, S.p7f); up(pl_.synfinal, S.synsplit); up(pl_.coarse, S.coarse);
  for (int l = 0; l <= kMaxLevels; ++l) { up(pl_.ana_d[l], S.ana_d[l]); up(pl_.syn_d[l], S.syn_d[l]); }
  void* p = nullptr;
  if (hipMalloc(&p, members_.size() * sizeof(ProbDesc)) != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error(PSARA_ENOMEM, "batch descriptor allocation failed");
  }
  allocs_.push_back(p);
  d_descs_ = (ProbDesc*)p;
  pl_.descs = d_descs_;
  pl_.cells = cells; pl_.rcells = cells;
  pl_.max_ts = max_ts; pl_.taps = T; pl_.max_levels = max_levels;
  pl_.max_n = max_n;
  pl_.ana_wide = ana_wide;
  pl_.grid_ce = grid_ce;
  pl_.sparse = sparse;
  set_grid_kernel_limits<R>(max_ts, T);
  hip_check(hipStreamCreateWithFlags(&s1_, hipStreamNonBlocking), "hipStreamCreate");
  hip_check(hipEventCreateWithFlags(&ev_fork_, hipEventDisableTiming), "hipEventCreate");
  hip_check(hipEventCreateWithFlags(&ev_join_, hipEventDisableTiming), "hipEventCreate");
}

template <typename R>
Batch<R>::~Batch() {
  (void)hipStreamSynchronize(s0_);
  if (s1_) (void)hipStreamSynchronize(s1_);
  for (auto& kv : graphs_) if (kv.second) (void)hipGraphExecDestroy(kv.second);
  for (void* p : allocs_) (void)hipFree(p);
  if (h_active_) (void)hipHostFree(h_active_);
  for (hipEvent_t e : ev_active_) if (e) (void)hipEventDestroy(e);
  if (ev_fork_) (void)hipEventDestroy(ev_fork_);
  if (ev_join_) (void)hipEventDestroy(ev_join_);
  if (s1_) (void)hipStreamDestroy(s1_);
}

template <typename R>
hipGraphExec_t Batch<R>::graph(int mode, int count) {
  const uint64_t key = graph_key(false, mode, count);
  auto it = graphs_.find(key);
  if (it != graphs_.end()) return it->second;
  hipGraph_t g = nullptr;
  hip_check(hipStreamBeginCapture(s0_, hipStreamCaptureModeRelaxed), "begin capture");
  launch_iterations<R>(pl_, mode, count, s0_, s1_, ev_fork_, ev_join_);
  hip_check(hipStreamEndCapture(s0_, &g), "end capture");
  hipGraphExec_t exec = nullptr;
  hip_check(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0), "graph instantiate");
  (void)hipGraphDestroy(g);
  graphs_[key] = exec;
  return exec;
}

template <typename R>
void Batch<R>::capture(int mode) {
  if ((mode != PM_INIT) && !pl_.sparse) throw Error(PSARA_ESTATE, "every batch member needs a wavelet prior in this mode");
  graph(mode, kBatchChunk);
  graph(mode, 1);
}

template <typename R>
void Batch<R>::run(int mode, int iters) {
  if ((mode != PM_INIT) && !pl_.sparse) throw Error(PSARA_ESTATE, "every batch member needs a wavelet prior in this mode");
  // the members' current descriptors (scalars may have changed since the last run)
  std::vector<ProbDesc> d(members_.size());
  for (size_t i = 0; i < members_.size(); ++i) {
    members_[i]->sync();
    d[i] = members_[i]->desc();
    hip_check(hipStreamSynchronize(members_[i]->stream()), "member sync");
  }
  copy_sync(d_descs_, d.data(), d.size() * sizeof(ProbDesc), hipMemcpyHostToDevice, s0_, "descriptors upload");
  if (iters <= 0) return;
  int left = iters;
  if (left >= kBatchChunk) {
    hipGraphExec_t g = graph(mode, kBatchChunk);
    while (left >= kBatchChunk) { hip_check(hipGraphLaunch(g, s0_), "graph launch"); left -= kBatchChunk; }
  }
  if (left > 0) {
    hipGraphExec_t g = graph(mode, 1);
    for (; left > 0; --left) hip_check(hipGraphLaunch(g, s0_), "graph launch");
  }
  hip_check(hipGetLastError(), "batch iteration launch");
}

template <typename R>
void Batch<R>::adaptive_buffers() {
  if (d_active_) return;
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(int)) != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error(PSARA_ENOMEM, "batch flag allocation failed");
  }
  allocs_.push_back(p);
  d_active_ = (int*)p;
  if (hipHostMalloc(&p, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error(PSARA_ENOMEM, "pinned host allocation failed");
  }
  h_active_ = (int*)p;
  for (int i = 0; i < 2; ++i) hip_check(hipEventCreateWithFlags(&ev_active_[i], hipEventDisableTiming), "event");
}

// The captured chunk of an adaptive run: `count` iterations, the check, the decision.
template <typename R>
hipGraphExec_t Batch<R>::adaptive_graph(int mode, int count) {
  const uint64_t key = graph_key(true, mode, count);
  auto it = graphs_.find(key);
  if (it != graphs_.end()) return it->second;
  adaptive_buffers();
  const int nprob = (int)members_.size();
  hipGraph_t g = nullptr;
  hip_check(hipStreamBeginCapture(s0_, hipStreamCaptureModeRelaxed), "begin capture");
  launch_iterations<R>(pl_, mode, count, s0_, s1_, ev_fork_, ev_join_);
  launch_check<R>(pl_, nprob, s0_);
  launch_stop_decide(pl_.descs, nprob, count, d_active_, s0_);
  hip_check(hipStreamEndCapture(s0_, &g), "end capture");
  hipGraphExec_t exec = nullptr;
  hip_check(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0), "graph instantiate");
  (void)hipGraphDestroy(g);
  graphs_[key] = exec;
  return exec;
}

template <typename R>
void Batch<R>::capture_adaptive(int mode, int check_every) {
  if ((mode != PM_INIT) && !pl_.sparse) throw Error(PSARA_ESTATE, "every batch member needs a wavelet prior in this mode");
  adaptive_graph(mode, check_every);
}

template <typename R>
void Batch<R>::launch_adaptive(int mode, int chunks, int check_every) {
  run(mode, 0);                      // uploads the members' current descriptors
  for (int c = 0; c < chunks; ++c) hip_check(hipGraphLaunch(adaptive_graph(mode, check_every), s0_), "graph launch");
}

template <typename R>
void Batch<R>::run_adaptive(int mode, int max_iters, int check_every, const double* stop, int* iters_out) {
  if ((mode != PM_INIT) && !pl_.sparse) throw Error(PSARA_ESTATE, "every batch member needs a wavelet prior in this mode");
  for (Engine<R>* e : members_) e->stop_begin(stop);
  run(mode, 0);                      // uploads the members' current descriptors
  adaptive_buffers();
  auto graph = [&](int count) { return adaptive_graph(mode, count); };
  adaptive_loop(graph, max_iters, check_every, s0_, d_active_, h_active_, ev_active_);
  for (size_t i = 0; i < members_.size(); ++i) {
    const int it = members_[i]->stop_end();
    if (iters_out) iters_out[i] = it;
  }
}

template <typename R>
void Batch<R>::profile(int mode, int iters, double* ms) {
  run(mode, 0);                      // uploads the members' current descriptors
  profile_iterations<R>(pl_, mode, iters, s0_, ms);
}

template struct Batch<float>;
template struct Batch<double>;

}  // namespace psara
