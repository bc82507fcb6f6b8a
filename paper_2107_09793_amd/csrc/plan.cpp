// Contraction plan (host only).
//
// Bit model: every index of dimension 2^w is w bits.  A tensor is addressed
// by its bits, each with a power-of-two stride, so every transpose of the
// TTGT decomposition (Sec. 3.1) is a bit permutation and every operand of a
// step can be read in place through its bit strides.
//
// Slicing with shared work (Sec. 2.4, Sec. 3.2): a sliced index is never
// summed where its two tensors meet; it stays a bit of every node above them
// and is summed at the very end.  A node therefore carries exactly the sliced
// bits of the leaves below it -- its instance set S_v -- and is computed for
// 2^|S_v| instances instead of once per slice; a node with S_v empty is the
// shared work of Fig. 5 and runs once.  In a step, a sliced bit held by both
// operands is a batch bit, one held by one operand folds into that operand's
// free (row or column) bits.
//
// Resident / outer split (Sec. 4, Fig. 8 discussion: only a subset of slices
// is held in memory, its size fixed a priori): the sliced indices are split
// into resident ones (kept as bits in HBM) and outer ones (looped over).
// Steps that depend on no outer index run once and their results stay
// resident for all outer iterations; the others run once per iteration.
//
// Deletion of intermediates (Fig. 8): every result is freed after its single
// consumer ran; arena offsets come from a best-fit allocator simulated here.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <functional>
#include <numeric>

namespace tn {
namespace {

using Bits = std::vector<int32_t>;

Bits inter(const Bits& a, const Bits& b) {
  Bits r;
  std::set_intersection(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
  return r;
}
Bits unite(const Bits& a, const Bits& b) {
  Bits r;
  std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
  return r;
}
Bits minus(const Bits& a, const Bits& b) {
  Bits r;
  std::set_difference(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
  return r;
}

int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Best-fit arena with coalescing free list.
struct Arena {
  std::map<int64_t, int64_t> free_;  // offset -> size
  int64_t top = 0;
  int64_t alloc(int64_t bytes) {
    bytes = align_up(std::max<int64_t>(bytes, 256), 256);
    auto best = free_.end();
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes && (best == free_.end() || it->second < best->second)) best = it;
    if (best != free_.end()) {
      int64_t off = best->first, sz = best->second;
      free_.erase(best);
      if (sz > bytes) free_[off + bytes] = sz - bytes;
      return off;
    }
    // grow; absorb a trailing free block
    if (!free_.empty()) {
      auto last = std::prev(free_.end());
      if (last->first + last->second == top) {
        int64_t off = last->first;
        free_.erase(last);
        top = off + bytes;
        return off;
      }
    }
    int64_t off = top;
    top += bytes;
    return off;
  }
  void release(int64_t off, int64_t bytes) {
    bytes = align_up(std::max<int64_t>(bytes, 256), 256);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Layout {  // executed bits of a node with strides (bit id -> log2 stride)
  std::map<int32_t, int8_t> s;
};

struct StepBits {  // global bit ids of a step's classes, in stride-array order
  Bits batch, M, N, K;
};


// LDS bank spread of a matrix-core chain step.  The chain kernel's LDS
// address of tile position x is 8 swz(x) bytes, swz(x) = x ^ ((x >> 5 ^
// x >> 9) & 31), so with 64 four-byte banks the bank pair of x is
// swz(x) & 31, an XOR-linear function: a tile slot contributes a fixed
// 5-bit vector.  Thirty-two lanes that vary over five slot bits hit
// 2^(5 - rank) times the same bank pair.  The step's roles can be chosen
// freely: which four row slots form a 16-row block (and which of them is
// the lane group's low output-row bit), which summed slot the lane group's
// low bit takes, and which four new slots the 16 lanes of a column block
// cover; this picks the choice with the fewest repeated banks for the
// block's reads and writes.
static uint32_t bank_vec(int slot) {
  const uint32_t x = 1u << slot;
  return (x ^ (x >> 5) ^ (x >> 9)) & 31u;
}

static int gf2_rank(std::vector<uint32_t> v) {
  int r = 0;
  for (int bit = 31; bit >= 0; --bit) {
    int piv = -1;
    for (int i = r; i < (int)v.size(); ++i)
      if ((v[i] >> bit) & 1u) {
        piv = i;
        break;
      }
    if (piv < 0) continue;
    std::swap(v[r], v[piv]);
    for (int i = 0; i < (int)v.size(); ++i)
      if (i != r && ((v[i] >> bit) & 1u)) v[i] ^= v[r];
    ++r;
  }
  return r;
}

static void bank_tune(ChainStepDesc& d, bool split) {
  const int nk = (int)d.kslot.size(), nn = (int)d.nslot.size(), nrow = (int)d.rslot.size();
  if (nrow < 4) return;
  // lane group g's low bit is summed bit g0pos of the step (see the kernels)
  const int g0pos = split ? 1 : nk - 2;
  const int kg = nk >= 2 ? nk : 0;
  const int CB = (1 << nn) / 8;
  const int reads = split ? 2 * std::max(1, (1 << nk) / 8) : (1 << nk) / 4;
  const int writes = CB >= 2 ? 2 * CB : 4;
  double best = 1e30;
  std::vector<int8_t> bR;
  int bG = -1, bX = -1;
  for (int a = 0; a < nrow; ++a)
    for (int b = a + 1; b < nrow; ++b)
      for (int c = b + 1; c < nrow; ++c)
        for (int e = c + 1; e < nrow; ++e) {
          const int four[4] = {a, b, c, e};
          for (int r2 = 0; r2 < 4; ++r2) {
            const int8_t R2 = d.rslot[four[r2]];
            // writes: 32 lanes = 16 column lanes x the low lane-group bit
            double wbest = 1e30;
            int wx = -1;
            for (int x = (nn == 5 ? 0 : -1); x < (nn == 5 ? 5 : 0); ++x) {
              std::vector<uint32_t> v;
              if (CB >= 2) {
                for (int t = 0; t < nn; ++t)
                  if (t != x && (int)v.size() < 4) v.push_back(bank_vec(d.nslot[t]));
              } else {
                for (int t = 0; t < 3 && t < nn; ++t) v.push_back(bank_vec(d.nslot[t]));
              }
              v.push_back(bank_vec(R2));
              const double m = (double)(1 << ((int)v.size() - gf2_rank(v)));
              if (m < wbest) {
                wbest = m;
                wx = x;
              }
            }
            for (int gk = 0; gk < kg; ++gk) {
              std::vector<uint32_t> v;
              for (int t = 0; t < 4; ++t) v.push_back(bank_vec(d.rslot[four[t]]));
              v.push_back(bank_vec(d.kslot[gk]));
              const double rm = (double)(1 << (5 - gf2_rank(v)));
              const double cost = reads * rm + writes * wbest;
              if (cost < best - 1e-9) {
                best = cost;
                bR.clear();
                for (int t = 0; t < 4; ++t)
                  if (t != r2) bR.push_back(d.rslot[four[t]]);
                bR.insert(bR.begin() + 2, R2);   // rows: r bits 0, 1, then g bits
                bG = gk;
                bX = wx;
              }
            }
          }
        }
  if (bG < 0) return;
  std::vector<int8_t> rest;
  for (int8_t s : d.rslot)
    if (std::find(bR.begin(), bR.end(), s) == bR.end()) rest.push_back(s);
  d.rslot = bR;
  d.rslot.insert(d.rslot.end(), rest.begin(), rest.end());
  if (g0pos >= 0 && g0pos < nk && bG != g0pos) {
    std::swap(d.kslot[g0pos], d.kslot[bG]);
    std::swap(d.kB[g0pos], d.kB[bG]);
  }
  if (bX >= 0 && bX != 4) {
    std::swap(d.nslot[4], d.nslot[bX]);
    std::swap(d.nB[4], d.nB[bX]);
  }
}

// Tile of a chain candidate first..last (see ChainGroup); returns false when
// it does not fit the LDS tile or a summed / batch bit is misplaced.
bool build_chain(const Plan& p, const std::vector<Layout>& lay, const std::vector<StepBits>& sb,
                 int first, int last, ChainGroup& g) {
  const int n = p.n_tensors;
  const int X = p.steps[first].a, Y = n + last;
  const Bits& E0 = p.node_ebits[X];
  // input bits summed inside the chain, bits created inside it
  Bits in_act, created;
  for (int k = first; k <= last; ++k) {
    Bits K = sb[k].K;
    std::sort(K.begin(), K.end());
    in_act = unite(in_act, inter(K, E0));
    Bits N = sb[k].N;
    std::sort(N.begin(), N.end());
    created = unite(created, N);
  }
  // batch bits must stay outside the tile; simulate the live tile bits
  Bits live = in_act;
  int max_live = (int)live.size();
  Bits batch_all;
  for (int k = first; k <= last; ++k) {
    Bits K = sb[k].K, N = sb[k].N, B = sb[k].batch;
    std::sort(K.begin(), K.end());
    std::sort(N.begin(), N.end());
    std::sort(B.begin(), B.end());
    if (minus(K, live).size()) return false;          // summed bit not in the tile
    if (!inter(B, unite(in_act, created)).empty()) return false;
    batch_all = unite(batch_all, B);
    live = unite(minus(live, K), N);
    max_live = std::max(max_live, (int)live.size());
  }
  const Bits out_created = live;   // created bits that reach the output
  const Bits pas = minus(E0, in_act);
  // low-stride passive bits go into the tile so loads and stores run over
  // at least 2^3 consecutive elements; more when room is left
  auto low_bits = [&](int node) {
    std::vector<std::pair<int, int32_t>> v;
    for (const auto& kv : lay[node].s) v.push_back({kv.second, kv.first});
    std::sort(v.begin(), v.end());
    Bits r;
    for (auto& x : v) r.push_back(x.second);
    return r;
  };
  const Bits xo = low_bits(X), yo = low_bits(Y);
  Bits ptile;
  int want = 5;
  for (; want >= 3; --want) {
    ptile.clear();
    bool ok = true;
    for (const Bits* o : {&xo, &yo}) {
      for (int i = 0; i < want && i < (int)o->size(); ++i) {
        int b = (*o)[i];
        bool in_tile = std::binary_search(in_act.begin(), in_act.end(), b) ||
                       std::binary_search(out_created.begin(), out_created.end(), b);
        if (in_tile) continue;
        if (std::binary_search(batch_all.begin(), batch_all.end(), b)) { ok = false; break; }
        if (std::find(ptile.begin(), ptile.end(), b) == ptile.end()) ptile.push_back(b);
      }
    }
    if (ok && max_live + (int)ptile.size() <= kChainTileBits) break;
  }
  if (want < 3) return false;
  // then further passive bits, lowest input stride first, until the tile has
  // its full size: every thread of the workgroup gets rows to work on and
  // the per-tile costs are spread over more elements
  for (int32_t b : xo) {
    if (max_live + (int)ptile.size() >= kChainTileBits) break;
    if (std::binary_search(in_act.begin(), in_act.end(), b) ||
        std::binary_search(batch_all.begin(), batch_all.end(), b) ||
        std::find(ptile.begin(), ptile.end(), b) != ptile.end())
      continue;
    ptile.push_back(b);
  }
  std::sort(ptile.begin(), ptile.end());
  const Bits pt = minus(pas, ptile);   // passive bits that enumerate tiles
  if ((int)pt.size() > kChainPassive) return false;
  // LDS slots: tile passive bits lowest, then input bits; a new bit takes
  // the lowest free slot after the step's summed bits are released
  std::map<int32_t, int> slot;
  std::vector<uint8_t> used(kChainTileBits, 0);
  auto take = [&](int32_t b) {
    for (int q = 0; q < kChainTileBits; ++q)
      if (!used[q]) {
        used[q] = 1;
        slot[b] = q;
        return true;
      }
    return false;
  };
  for (int32_t b : ptile) take(b);
  Bits in_sorted = in_act;
  std::sort(in_sorted.begin(), in_sorted.end(),
            [&](int32_t a, int32_t b) { return lay[X].s.at(a) < lay[X].s.at(b); });
  for (int32_t b : in_sorted) take(b);
  g = ChainGroup();
  g.first = first;
  g.last = last;
  g.phase = p.steps[first].phase;
  Bits tile_live = unite(in_act, ptile);
  int64_t staged_f = 0, staged_v = 0;
  for (int k = first; k <= last; ++k) {
    const StepDesc& S = p.steps[k];
    ChainStepDesc d;
    d.step = k;
    Bits K = sb[k].K;
    std::sort(K.begin(), K.end());
    Bits rows = minus(tile_live, K);
    for (int32_t b : sb[k].K) d.kslot.push_back((int8_t)slot.at(b));
    for (int32_t b : K) used[slot.at(b)] = 0;
    for (int32_t b : sb[k].N)
      if (!take(b)) return false;
    for (int32_t b : sb[k].N) d.nslot.push_back((int8_t)slot.at(b));
    std::vector<int8_t> rs;
    for (int32_t b : rows) rs.push_back((int8_t)slot.at(b));
    std::sort(rs.begin(), rs.end());
    d.rslot = rs;
    d.nrow = (int32_t)rs.size();
    // shapes only the matrix-core step runs need 16-row blocks; the small
    // operands of all steps are staged together
    const int nk = (int)sb[k].K.size(), nn = (int)sb[k].N.size();
    const bool on_mfma = chain_step_mfma(nk, nn, d.nrow, p.flags);
    if ((nk > 4 || nn > 4) && !on_mfma) return false;
    staged_f += chain_staged_floats(nk, nn, on_mfma);
    if (!on_mfma) staged_v += 1 << (nk + nn);
    if (staged_f > kChainBFloats || staged_v > kChainVElems) return false;
    d.kB = S.kB;
    d.nB = S.nB;
    d.bB = S.bB;
    if (on_mfma) bank_tune(d, p.precision == PREC_SPLIT_BF16);
    for (int32_t b : sb[k].batch) {
      auto it = std::find(pt.begin(), pt.end(), b);
      if (it == pt.end()) return false;
      d.bpas.push_back((int8_t)(it - pt.begin()));
    }
    Bits N = sb[k].N;
    std::sort(N.begin(), N.end());
    tile_live = unite(rows, N);
    g.st.push_back(d);
  }
  int tb = 0;
  for (const auto& kv : slot) tb = std::max(tb, kv.second + 1);
  g.tile_bits = tb;
  // input tile bits in input-stride order, output tile bits in output order
  Bits in_tile = unite(in_act, ptile), out_tile = unite(out_created, ptile);
  std::sort(in_tile.begin(), in_tile.end(),
            [&](int32_t a, int32_t b) { return lay[X].s.at(a) < lay[X].s.at(b); });
  std::sort(out_tile.begin(), out_tile.end(),
            [&](int32_t a, int32_t b) { return lay[Y].s.at(a) < lay[Y].s.at(b); });
  // slots at load / store time: input bits keep their first slot; output
  // bits hold the slot they had after the last step
  std::map<int32_t, int> first_slot;
  for (int32_t b : ptile) first_slot[b] = slot.at(b);
  {
    // recompute the input slots (slot[] was overwritten for reused bits only
    // if a bit id repeats, which it cannot: bit ids are unique in the chain)
    for (int32_t b : in_act) first_slot[b] = slot.at(b);
  }
  for (int32_t b : in_tile) {
    g.in_slot.push_back((int8_t)first_slot.at(b));
    g.in_log2.push_back(lay[X].s.at(b));
  }
  for (int32_t b : out_tile) {
    g.out_slot.push_back((int8_t)slot.at(b));
    g.out_log2.push_back(lay[Y].s.at(b));
  }
  for (int32_t b : pt) {
    g.pas_in.push_back(lay[X].s.at(b));
    g.pas_out.push_back(lay[Y].s.at(b));
  }
  return true;
}

}  // namespace

// Kernel family for a step of the given shape (bit counts of the batch, row,
// column and summed classes).
int32_t choose_kind(int nb, int nm, int nn, int nk, uint32_t flags, int32_t* chunks,
                    int64_t* scratch) {
  int out_bits = nb + nm + nn;
  *chunks = 0;
  *scratch = 0;
  if (nk >= 8 && out_bits <= 12) {
    if (nm >= 5 && nn >= 3 && !(flags & 2u)) {
      // few output tiles, long sums: MFMA tiles over chunks of k (about 2^11
      // workgroups in all, at least one 32-wide k tile per chunk), partial
      // tiles added up in a fixed order afterwards
      const int tiles_log2 = std::max(0, out_bits - 12);
      const int cl = std::max(0, std::min(11 - tiles_log2, nk - 5));
      *chunks = 1 << cl;
      *scratch = cl > 0 ? (int64_t)8 << (out_bits + cl) : 0;
      return KIND_GEMM;
    }
    int cl = std::max(8, nk - 10);  // log2 chunk length
    if (cl > nk) cl = nk;
    *chunks = 1 << (nk - cl);
    *scratch = (int64_t)8 << (out_bits + (nk - cl));
    return KIND_SPLITK;
  }
  if (flags & 2u) return KIND_SIMPLE;
  if (nk >= 8 && nm >= 5 && nn >= 3 && out_bits - 13 < 8) {
    // fewer than 2^8 output tiles of 128 x 64 and long sums: chunks of k
    // bring the launch to about 2^10 workgroups, each chunk summing at least
    // 2^7 values so that writing and re-reading the partial tiles (16 bytes
    // per output and chunk) costs less than half the products' time
    const int tiles_log2 = std::max(0, out_bits - 13);
    const int cl = std::min(10 - tiles_log2, nk - 7);
    if (cl >= 1) {
      *chunks = 1 << cl;
      *scratch = (int64_t)8 << (out_bits + cl);
    }
    return KIND_GEMM;
  }
  if (nk <= 4 && nn <= 4 && nb <= 12) return KIND_STREAM;
  if (nm >= 5 && nn >= 3 && nk >= 3) return KIND_GEMM;
  // many rows against a few columns and many summed values: the GEMM
  // kernel with its narrowest tile (partial columns) streams the rows
  if (nm >= 12 && nn >= 1 && nk >= 5) return KIND_GEMM;
  return KIND_SIMPLE;
}

int32_t choose_tile(const Plan& p, int nm, int nn, int nk) {
  if (p.gemm_config >= 0) return p.gemm_config;
  int best = -1, best_d = 1 << 30;
  for (size_t i = 0; i + 4 < p.tune.size(); i += 5) {
    const int32_t* e = &p.tune[i];
    if (e[0] != p.precision || e[2] != nn || e[4] < 0 || e[4] >= kNumGemmConfigs) continue;
    int d = std::abs(e[1] - nm) + 4 * std::abs(e[3] - nk);
    if (d < best_d) {
      best_d = d;
      best = e[4];
    }
  }
  if (best >= 0) return best;
  // many rows: the stream kernels (three real products in complex64), which
  // fall back to the one-tile rule on shapes they do not take
  if (nm >= 18 && nn >= 4) return p.precision == PREC_C64 ? kGemmStreamGauss : kGemmStream;
  return rule_tile(nn);
}

int32_t rule_tile(int nn) {
  if (nn >= 6) return 0;   // 128 x 64
  if (nn == 5) return 1;   // 128 x 32
  return 7;                // 128 x 16
}

// The stream kernel: one batch, whole 32-row bands, at least one 16-column
// block, no split k, and a column tile of 2^ln columns whose B block (all k)
// fits the 64 KiB buffer: 8 bytes per complex entry in complex64 (ln <= 7,
// k tiles of 16 at 128 columns, else 32), 16 in split-BF16 (the embedded hi
// and lo operands; ln <= min(6, 12 - nk), k tiles of 32).
void stream_gemm_tile(int nn, int nk, int32_t precision, int* ln, int* lkt) {
  if (precision == PREC_SPLIT_BF16) {
    *ln = std::min(std::min(nn, 6), 12 - nk);
    *lkt = 5;
  } else {
    *ln = std::min(nn, 7);
    *lkt = *ln == 7 ? 4 : 5;
  }
}

bool stream_gemm_shape(int nb, int nm, int nn, int nk, int32_t chunks, int32_t precision) {
  if (nb != 0 || nm < 10 || nn < 4 || chunks > 1 || nk > 9) return false;
  int ln, lkt;
  stream_gemm_tile(nn, nk, precision, &ln, &lkt);
  if (ln < 4 || nn - ln > 10 || nk < lkt) return false;
  return ln + nk <= (precision == PREC_SPLIT_BF16 ? 12 : 13);
}

// The three-product stream kernel: complex64, column tiles of
// 2^min(nn, 6, 12 - nk) >= 32 columns, k tiles of 32, B's three planes of
// 4-byte entries (at most 2^12 entries per plane).
bool stream_gauss_shape(int nb, int nm, int nn, int nk, int32_t chunks, int32_t precision) {
  if (precision != PREC_C64 || nb != 0 || nm < 10 || chunks > 1 || nk < 5 || nk > 7) return false;
  const int ln = std::min(std::min(nn, 6), 12 - nk);
  return ln >= 5 && nn - ln <= 10;
}

int32_t tile_run(int32_t tile, int nb, int nm, int nn, int nk, int32_t chunks, int32_t precision) {
  if (tile == kGemmStreamGauss) {
    if (stream_gauss_shape(nb, nm, nn, nk, chunks, precision)) return tile;
    tile = kGemmStream;
  }
  if (tile == kGemmStream) {
    if (stream_gemm_shape(nb, nm, nn, nk, chunks, precision)) return tile;
    tile = rule_tile(nn);
  }
  return tile;
}

// Kernel launches of one execution of a step: split-k runs two kernels; a
// GEMM step runs one launch per 2^23 output tiles (a dispatch holds fewer
// than 2^32 work-items of 256-thread workgroups).
static int32_t step_launches(const StepDesc& S, int32_t precision) {
  if (S.kind == KIND_SPLITK) return 2;
  if (S.kind == KIND_GEMM && S.splitk_chunks > 1) return 2;   // partial tiles, then their sum
  if (S.kind != KIND_GEMM || S.tile < 0 || S.tile >= kNumGemmConfigs) return 1;
  const int nb = (int)S.bA.size(), nm = (int)S.mA.size(), nn = (int)S.nB.size();
  const int tile = tile_run(S.tile, nb, nm, nn, (int)S.kA.size(), S.splitk_chunks, precision);
  if (tile >= kGemmStream) return 1;
  static const int lm[kGemmStream] = {7, 7, 8, 7, 8, 7, 7, 7};   // log2 tile rows
  static const int ln[kGemmStream] = {6, 5, 4, 7, 6, 6, 5, 4};   // log2 tile columns
  const int t = nb + std::max(0, nm - lm[tile]) + std::max(0, nn - ln[tile]);
  return t > 23 ? 1 << std::min(t - 23, 24) : 1;
}

// Build schedule for a given outer set; fills steps, sched, memory, stats.
static void schedule_pass(Plan& p);

// Two planning passes when chains are on: the first finds the chains, the
// second lays out every chain input with the bits its chain sums over lowest
// (and forms the chains again on those layouts).  Results of stream steps put
// their new (column) bits lowest when chains are on, so a chain's output
// tile -- the bits the chain created -- is one contiguous block.
static void schedule(Plan& p) {
  p.chain_in_low.clear();
  schedule_pass(p);
  if (p.chains.empty()) return;
  for (const ChainGroup& g : p.chains) {
    const int X = p.steps[g.first].a;
    if (X < p.n_tensors) continue;   // leaf layouts are the caller's
    // a GEMM result keeps its tile-friendly layout (columns, then rows,
    // lowest): moving the chain's summed bits lowest would scatter the GEMM
    // epilogue's stores, and the chain's tile still holds low-stride bits
    // of its input for contiguous loads
    if (p.steps[X - p.n_tensors].kind == KIND_GEMM) continue;
    Bits in;
    for (int k = g.first; k <= g.last; ++k)
      for (int32_t b : p.chain_sum_bits[k]) in.push_back(b);
    std::sort(in.begin(), in.end());
    p.chain_in_low[X] = inter(in, p.node_ebits[X]);
  }
  schedule_pass(p);
}

static void schedule_pass(Plan& p) {
  const int n = p.n_tensors;
  const int nsteps = n - 1;
  const int nn_nodes = n + nsteps;
  bool no_reuse = p.flags & 1u;
  p.bit_outer.assign(p.n_bits, 0);
  for (int e : p.outer_idx)
    for (int j = 0; j < p.index_w[e]; ++j) p.bit_outer[p.index_bit0[e] + j] = 1;
  Bits outer_bits_set;
  for (int b = 0; b < p.n_bits; ++b)
    if (p.bit_outer[b]) outer_bits_set.push_back(b);

  p.node_ebits.assign(nn_nodes, {});
  p.node_layout.assign(nn_nodes, {});
  p.node_log2s.assign(nn_nodes, {});
  p.node_phase.assign(nn_nodes, 0);
  std::vector<Layout> lay(nn_nodes);

  // leaves: executed layout = leaf layout without outer bits
  for (int t = 0; t < n; ++t) {
    LeafDesc& L = p.leaves[t];
    L.outer_bits.clear();
    L.outer_log2s.clear();
    for (size_t i = 0; i < L.bits.size(); ++i) {
      int b = L.bits[i];
      if (p.bit_outer[b]) {
        L.outer_bits.push_back(b);
        L.outer_log2s.push_back(L.log2s[i]);
      } else {
        lay[t].s[b] = L.log2s[i];
        p.node_layout[t].push_back(b);
      }
    }
    p.node_ebits[t] = minus(p.node_bits[t], outer_bits_set);
    p.node_phase[t] = L.outer_bits.empty() ? 0 : 1;
  }

  p.steps.assign(nsteps, StepDesc());
  std::vector<StepBits> sbits(nsteps);
  p.chain_sum_bits.assign(nsteps, {});
  for (int k = 0; k < nsteps; ++k) {
    int a = p.path[2 * k], b = p.path[2 * k + 1], v = n + k;
    StepDesc& S = p.steps[k];
    // the larger operand is A (rows); the smaller B (columns)
    if (p.node_ebits[b].size() > p.node_ebits[a].size()) std::swap(a, b);
    S.a = a;
    S.b = b;
    S.c = v;
    const Bits& eA = p.node_ebits[a];
    const Bits& eB = p.node_ebits[b];
    Bits common = inter(eA, eB);
    Bits batch, K;
    for (int x : common) (p.bit_kept[x] ? batch : K).push_back(x);
    Bits M = minus(eA, common), N = minus(eB, common);
    auto by = [&](Bits v2, const Layout& L) {
      std::sort(v2.begin(), v2.end(), [&](int x, int y) { return L.s.at(x) < L.s.at(y); });
      return v2;
    };
    M = by(M, lay[a]);
    N = by(N, lay[b]);
    batch = by(batch, lay[a]);
    K = by(K, lay[a]);
    int nb = (int)batch.size(), nm = (int)M.size(), nnb = (int)N.size(), nk = (int)K.size();
    sbits[k] = StepBits{batch, M, N, K};
    p.chain_sum_bits[k] = K;
    S.kind = choose_kind(nb, nm, nnb, nk, p.flags, &S.splitk_chunks, &S.scratch_bytes);
    // result layout, least significant first.  GEMM tiles store 16 consecutive
    // columns per half-wave: columns, rows, batch.  The stream kernel runs one
    // row per lane: rows, columns, batch.
    Bits clayout;
    const bool rows_low = S.kind == KIND_STREAM && (p.flags & 8u);   // no chains
    const Bits& lo = rows_low ? M : N;
    const Bits& mid = rows_low ? N : M;
    clayout.insert(clayout.end(), lo.begin(), lo.end());
    clayout.insert(clayout.end(), mid.begin(), mid.end());
    clayout.insert(clayout.end(), batch.begin(), batch.end());
    auto ov = p.chain_in_low.find(v);
    if (ov != p.chain_in_low.end()) {
      // input of a chain (found by an earlier planning pass): the bits that
      // chain sums over lowest, so its tiles are read as contiguous blocks
      Bits want = ov->second, first, rest;
      std::sort(want.begin(), want.end());
      for (int32_t x : clayout)
        (std::binary_search(want.begin(), want.end(), x) ? first : rest).push_back(x);
      clayout = first;
      clayout.insert(clayout.end(), rest.begin(), rest.end());
    }
    for (size_t i = 0; i < clayout.size(); ++i) lay[v].s[clayout[i]] = (int8_t)i;
    p.node_layout[v] = clayout;
    p.node_ebits[v] = unite(unite(batch, M), N);
    std::sort(p.node_ebits[v].begin(), p.node_ebits[v].end());
    auto fill = [&](const Bits& cls, const Layout& L, std::vector<int8_t>& out) {
      out.clear();
      for (int x : cls) out.push_back(L.s.at(x));
    };
    fill(batch, lay[a], S.bA);
    fill(batch, lay[b], S.bB);
    fill(batch, lay[v], S.bC);
    fill(M, lay[a], S.mA);
    fill(M, lay[v], S.mC);
    fill(N, lay[b], S.nB);
    fill(N, lay[v], S.nC);
    fill(K, lay[a], S.kA);
    fill(K, lay[b], S.kB);
    S.cmac = std::ldexp(1.0, nb + nm + nnb + nk);
    S.c_bytes = (int64_t)8 << (nb + nm + nnb);
    S.tile = S.kind == KIND_GEMM ? choose_tile(p, nm, nnb, nk) : -1;
    // instance bits all-resident: sliced bits of the operands
    Bits u = unite(p.node_bits[a], p.node_bits[b]);
    int sv = 0;
    for (int x : u) sv += p.bit_sliced[x];
    S.inst_bits = sv;
    bool dep_outer = !inter(unite(p.node_bits[a], p.node_bits[b]), outer_bits_set).empty();
    p.node_phase[v] = (no_reuse || dep_outer) ? 1 : 0;
    S.phase = p.node_phase[v];
  }
  // variable leaves below each node; invariant steps (group 0) depend on
  // none of them and on no outer index
  {
    std::vector<uint8_t> var(nn_nodes, 0);
    bool any = false;
    for (int t = 0; t < n; ++t) {
      var[t] = t < (int)p.leaf_variable.size() && p.leaf_variable[t];
      any |= var[t] != 0;
    }
    for (int k = 0; k < nsteps; ++k) {
      StepDesc& S = p.steps[k];
      var[n + k] = var[S.a] | var[S.b];
      S.group = S.phase == 1 ? 2 : (any && !var[n + k] ? 0 : 1);
    }
  }
  const int root = nn_nodes - 1;

  // small steps: run as work items of persistent segments (opt-in: a GPU
  // test of the segment kernel at full size did not finish, cause not found)
  const bool persist = (p.flags & 16u) && !(p.flags & 4u);
  for (int k = 0; k < nsteps; ++k) {
    StepDesc& S = p.steps[k];
    int nb = (int)S.bA.size(), nm = (int)S.mA.size(), nnb = (int)S.nB.size(), nk = (int)S.kA.size();
    S.small = persist && (S.kind == KIND_STREAM || S.kind == KIND_SIMPLE) &&
              S.cmac <= std::ldexp(1.0, 22) && nb <= kSmallClassBits &&
              nm <= kSmallClassBits && nnb <= kSmallClassBits && nk <= kSmallClassBits;
    // tiny steps (without persistent segments): batches of them run in one
    // launch of one workgroup (TN_FLAG_NO_TINY: one launch each)
    S.tiny = !persist && !(p.flags & 512u) && S.kind != KIND_SPLITK && S.splitk_chunks <= 1 &&
             S.cmac <= std::ldexp(1.0, kTinyCmacBits) && nb + nm + nnb <= kTinyOutBits &&
             nb <= kTinyClassBits &&
             nm <= kTinyClassBits && nnb <= kTinyClassBits && nk <= kTinyClassBits;
  }
  // chains: runs of consecutive large stream steps, each consuming the
  // previous result as its large operand, grown while the tile fits
  p.chains.clear();
  if (!(p.flags & 8u)) {
    // vector-unit chain steps: 2^nk, 2^nn <= 16 (the stream kernel's
    // shapes); matrix-core chain steps also take GEMM-kind steps with a
    // small operand (chain_mfma_shape)
    const bool mfma = !(p.flags & 32u);
    auto fusable = [&](int k) {
      const StepDesc& S = p.steps[k];
      if (S.small || S.tiny) return false;
      const int nk = (int)S.kA.size(), nn = (int)S.nB.size();
      if (S.kind == KIND_STREAM && nk <= 4 && nn <= 4) return true;
      return mfma && (S.kind == KIND_STREAM || S.kind == KIND_GEMM) && chain_mfma_shape(nk, nn);
    };
    int k = 0;
    while (k < nsteps) {
      if (!fusable(k)) { ++k; continue; }
      int j = k;
      ChainGroup g, cand;
      while (j + 1 < nsteps && j + 1 - k < kChainMaxSteps && fusable(j + 1) &&
             p.steps[j + 1].a == n + j && p.steps[j + 1].group == p.steps[k].group &&
             build_chain(p, lay, sbits, k, j + 1, cand)) {
        g = cand;
        ++j;
      }
      if (j == k && !(p.flags & 128u) && build_chain(p, lay, sbits, k, k, cand)) {   // TN_FLAG_CHAIN_NO_SINGLE
        // a lone step runs on the chain kernel too: its tile walk streams
        // the large operand with the small one staged once per workgroup
        g = cand;
      }
      if (j > k || g.st.size() == 1) {
        for (int q = k; q <= j; ++q) p.steps[q].chain = (int32_t)p.chains.size();
        p.chains.push_back(g);
      }
      k = j + 1;
    }
  }

  // schedule: invariant steps, the rest of phase 0, then phase 1; inside a
  // group a topological order that takes every ready small step before the
  // next ready large one (path order among equals), so small steps form long
  // segments.  (A step depending on a later group is in that group, so the
  // order is topological.)
  std::vector<int32_t> consumer(nn_nodes, -1);
  for (int k = 0; k < nsteps; ++k) {
    consumer[p.steps[k].a] = k;
    consumer[p.steps[k].b] = k;
  }
  p.sched.clear();
  for (int ph = 0; ph < 3; ++ph) {
    std::vector<int32_t> pending(nsteps, 0);
    std::vector<int32_t> rs, rb;   // ready small / large, kept sorted descending (pop back)
    for (int k = 0; k < nsteps; ++k) {
      if (p.steps[k].group != ph) continue;
      for (int x : {p.steps[k].a, p.steps[k].b})
        if (x >= n && p.steps[x - n].group == ph) pending[k]++;
      if (pending[k] == 0) (p.steps[k].small || p.steps[k].tiny ? rs : rb).push_back(k);
    }
    auto desc = [](std::vector<int32_t>& v) { std::sort(v.begin(), v.end(), std::greater<int32_t>()); };
    desc(rs);
    desc(rb);
    while (!rs.empty() || !rb.empty()) {
      int k;
      if (!rs.empty()) { k = rs.back(); rs.pop_back(); } else { k = rb.back(); rb.pop_back(); }
      p.sched.push_back(k);
      int c = consumer[n + k];
      if (c >= 0 && p.steps[c].group == ph && --pending[c] == 0) {
        (p.steps[c].small || p.steps[c].tiny ? rs : rb).push_back(c);
        desc(rs);
        desc(rb);
      }
    }
    if (ph == 0) p.n_invariant = (int32_t)p.sched.size();
    if (ph == 1) p.n_phase0 = (int32_t)p.sched.size();
  }
  // segments: runs of >= 2 consecutive small steps of one phase
  p.segments.clear();
  p.persist_bytes = 0;
  for (size_t i = 0; i < p.sched.size();) {
    const StepDesc& S = p.steps[p.sched[i]];
    size_t j = i;
    while (j < p.sched.size() && p.steps[p.sched[j]].small &&
           p.steps[p.sched[j]].group == S.group)
      ++j;
    if (j - i >= 2) {
      Segment g{(int32_t)i, (int32_t)j, 0, S.phase};
      for (size_t q = i; q < j; ++q) {
        const StepDesc& T = p.steps[p.sched[q]];
        int ob = (int)(T.bA.size() + T.mA.size() + T.nB.size());
        g.n_items += (int32_t)(((int64_t)1 << ob) + 255) / 256;
      }
      p.segments.push_back(g);
      i = j;
    } else {
      i = std::max(j, i + 1);
    }
  }

  // batches of tiny steps: runs of >= 2 consecutive tiny steps of one group,
  // at most kTinyMaxSteps per launch (they run in order, so the arena below
  // needs no change for them)
  p.tiny_runs.clear();
  for (size_t i = 0; i < p.sched.size();) {
    const StepDesc& S = p.steps[p.sched[i]];
    size_t j = i;
    while (j < p.sched.size() && j - i < (size_t)kTinyMaxSteps && p.steps[p.sched[j]].tiny &&
           p.steps[p.sched[j]].group == S.group)
      ++j;
    if (j - i >= 2) {
      p.tiny_runs.push_back(Segment{(int32_t)i, (int32_t)j, 0, S.phase});
      i = j;
    } else {
      i = std::max(j, i + 1);
    }
  }
  // inside a batch the steps run by levels (a step's level: one above the
  // levels of the batch steps producing its operands), the steps of one
  // level at once: the batch is reordered by level (still a topological
  // order)
  p.tiny_level.assign(p.sched.size(), 0);
  for (const Segment& g : p.tiny_runs) {
    std::map<int32_t, int32_t> lvl;   // SSA node produced in the batch -> level
    std::vector<std::pair<int32_t, int32_t>> ord;   // (level, step)
    for (int q = g.begin; q < g.end; ++q) {
      const StepDesc& T = p.steps[p.sched[q]];
      int32_t L = 0;
      for (int32_t x : {T.a, T.b}) {
        auto it = lvl.find(x);
        if (it != lvl.end()) L = std::max(L, it->second + 1);
      }
      lvl[n + p.sched[q]] = L;
      ord.push_back({L, p.sched[q]});
    }
    std::stable_sort(ord.begin(), ord.end(),
                     [](const std::pair<int32_t, int32_t>& x, const std::pair<int32_t, int32_t>& y) {
                       return x.first < y.first;
                     });
    for (int q = g.begin; q < g.end; ++q) {
      p.sched[q] = ord[q - g.begin].second;
      p.tiny_level[q] = (int8_t)std::min(ord[q - g.begin].first, 127);
    }
  }

  // arena.  Steps of one persistent segment run concurrently, and so do the
  // steps of one level of a batch of tiny steps, so buffers freed by such a
  // step are returned only when the whole segment or batch is done.
  std::vector<int32_t> seg_last(p.sched.size(), -1);   // position -> end of its segment - 1
  for (const Segment& g : p.segments)
    for (int q = g.begin; q < g.end; ++q) seg_last[q] = g.end - 1;
  for (const Segment& g : p.tiny_runs)
    for (int q = g.begin; q < g.end; ++q) seg_last[q] = g.end - 1;
  Arena ar;
  p.bytes_no_deletion = 0;
  p.scratch_bytes = 0;
  std::vector<std::pair<int64_t, int64_t>> deferred;
  for (size_t pos = 0; pos < p.sched.size(); ++pos) {
    const int sk = p.sched[pos];
    StepDesc& S = p.steps[sk];
    // a chain runs at the position of its last step: one result, and the
    // inputs of all its steps released there
    const bool fused = S.chain >= 0 && !(p.flags & 64u);
    if (fused && p.chains[S.chain].last != sk) {
      S.c_off = -1;
      continue;
    }
    S.c_off = ar.alloc(S.c_bytes);
    p.bytes_no_deletion += align_up(S.c_bytes, 256);
    p.scratch_bytes = std::max(p.scratch_bytes, S.scratch_bytes);
    std::vector<int32_t> ins;
    if (fused) {
      const ChainGroup& g = p.chains[S.chain];
      ins.push_back(p.steps[g.first].a);
      for (int q = g.first; q <= g.last; ++q) ins.push_back(p.steps[q].b);
    } else {
      ins = {S.a, S.b};
    }
    for (int x : ins) {
      if (x < n) continue;
      const StepDesc& X = p.steps[x - n];
      // results consumed by a later group stay allocated: phase-0 results
      // for every outer iteration, invariant results for later calls
      if (X.group != S.group) continue;
      if (seg_last[pos] >= 0) deferred.push_back({X.c_off, X.c_bytes});
      else ar.release(X.c_off, X.c_bytes);
    }
    if (seg_last[pos] == (int32_t)pos) {
      for (auto& d : deferred) ar.release(d.first, d.second);
      deferred.clear();
    }
  }
  p.arena_bytes = ar.top;

  // root / output description
  p.root_open_log2.clear();
  p.root_res_log2.clear();
  p.res_slicebit.clear();
  p.outer_slicebit.clear();
  p.outer_bit_ids.clear();
  const Layout& RL = lay[root];
  // output bits: open indices row-major, last open index fastest
  for (int oi = (int)p.open_ids.size() - 1; oi >= 0; --oi) {
    int e = p.open_ids[oi];
    for (int j = 0; j < p.index_w[e]; ++j) p.root_open_log2.push_back(RL.s.at(p.index_bit0[e] + j));
  }
  // slice-id bits: last sliced index least significant
  int pos = 0;
  for (int si = (int)p.sliced_ids.size() - 1; si >= 0; --si) {
    int e = p.sliced_ids[si];
    for (int j = 0; j < p.index_w[e]; ++j, ++pos) {
      int bit = p.index_bit0[e] + j;
      if (p.bit_outer[bit]) {
        p.outer_slicebit.push_back(pos);
        p.outer_bit_ids.push_back(bit);
      } else {
        p.root_res_log2.push_back(RL.s.at(bit));
        p.res_slicebit.push_back(pos);
      }
    }
  }
  p.outer_bits = (int32_t)p.outer_slicebit.size();
  p.resident_bits = (int32_t)p.res_slicebit.size();
  p.open_bits = (int32_t)p.root_open_log2.size();

  // statistics
  double iters = std::ldexp(1.0, p.outer_bits);
  p.cmac_exec = 0;
  p.bytes_min_exec = 0;
  p.max_log2_res = 0;
  int launches0 = 0, launches1 = 0;
  for (int k = 0; k < nsteps; ++k) {
    const StepDesc& S = p.steps[k];
    double mult = S.phase ? iters : 1.0;
    p.cmac_exec += mult * S.cmac;
    double ea = std::ldexp(1.0, (int)p.node_ebits[S.a].size());
    double eb = std::ldexp(1.0, (int)p.node_ebits[S.b].size());
    double ec = std::ldexp(1.0, (int)p.node_ebits[S.c].size());
    p.bytes_min_exec += mult * 8.0 * (ea + eb + ec);
    p.max_log2_res = std::max(p.max_log2_res, (int32_t)p.node_ebits[S.c].size());
    (S.phase ? launches1 : launches0) += step_launches(S, p.precision);
  }
  p.n_launches = launches0 + (int32_t)iters * (launches1 + 1) + 1;
  int64_t ctrl = align_up((int64_t)4 << p.resident_bits, 256);
  p.ctrl_bytes = ctrl;
  // persistent segments: a 256-byte header (the error word every segment
  // launch reports timed-out waits into), then one copy per (segment,
  // execution) of descriptors, item tables and counters
  int64_t pb = p.segments.empty() ? 0 : 256;
  for (const Segment& g : p.segments) {
    int64_t len = g.end - g.begin;
    int64_t one = align_up(len * kSmallStepBytes, 256) + align_up((int64_t)4 * g.n_items, 256) +
                  align_up((int64_t)4 * kCtrStride * (len + 2), 256);
    pb += one * (g.phase ? (int64_t)iters : 1);
  }
  p.persist_bytes = pb;
  p.workspace_bytes = align_up(p.arena_bytes, 256) + align_up(p.scratch_bytes, 256) + ctrl + pb;
  // launches: one persistent launch replaces its segment's step launches
  for (const Segment& g : p.segments) {
    int32_t saved = 0;
    for (int q = g.begin; q < g.end; ++q) saved += step_launches(p.steps[p.sched[q]], p.precision);
    int32_t d = saved - 1;
    p.n_launches -= g.phase ? (int32_t)iters * d : d;
  }
  // batches of tiny steps: one launch each
  for (const Segment& g : p.tiny_runs) {
    int32_t saved = 0;
    for (int q = g.begin; q < g.end; ++q) saved += step_launches(p.steps[p.sched[q]], p.precision);
    int32_t d = saved - 1;
    p.n_launches -= g.phase ? (int32_t)iters * d : d;
  }
  // chains: one launch for all their steps (unless launched step by step)
  for (const ChainGroup& g : p.chains) {
    if (p.flags & 64u) break;
    int32_t d = g.last - g.first;
    p.n_launches -= g.phase ? (int32_t)iters * d : d;
  }
}

// ---------------------------------------------------------------------------
// Backward schedule (the adjoint of the contraction).  The sum over slices
// (Eq. sliced_sum) and every pairwise step are linear in each operand, so the
// adjoint runs the steps in reverse: for C = A.B, dA = dC.B^H and dB = A^H.dC
// (conjugate-Wirtinger gradients), and a result shared by many slices (S_v
// smaller than the full slice set) receives the sum of their gradients
// through the folded instance bits of the adjoint product.  With outer
// iterations, phase-1 steps run forward and backward once per iteration and
// the gradients of phase-0 results consumed there accumulate across
// iterations; phase 0 is then differentiated once.
//
// The simulated sequence of allocations below is exactly the sequence
// tn_contract_backward executes:
//   1. forward of phase 0 (fused chains where a block holds the whole chain);
//   2. if there are outer iterations: zero the gradients of the phase-0
//      results consumed by phase 1 ("frontier"), then per iteration: forward
//      of phase 1, root gradient, adjoint of the phase-1 blocks in reverse;
//      then the frontier values are dropped;
//   3. (root gradient if phase 1 is empty,) adjoint of the phase-0 blocks.
// The adjoint of a block first recomputes, step by step, the values the
// block both produces and consumes (kept until their consumer's adjoint),
// then walks the block's steps in reverse; a step's operand values and its
// result's gradient are released right after its adjoint products.
namespace {

struct BwdEval {
  int64_t peak = 0;
  double recompute = 0;
};

BwdEval simulate_backward(const Plan& p, const std::vector<int32_t>& blk, bool fuse,
                          BwdPlan* out) {
  const int n = p.n_tensors, nsteps = n - 1, nodes = n + nsteps, root = nodes - 1;
  const int N = (int)p.sched.size();
  std::vector<int32_t> pos_of(nsteps, -1), cons(nodes, -1);
  for (int q = 0; q < N; ++q) pos_of[p.sched[q]] = q;
  for (int k = 0; k < nsteps; ++k) {
    cons[p.steps[k].a] = k;
    cons[p.steps[k].b] = k;
  }
  BwdPlan B;
  B.block_of = blk;
  B.keep.assign(nodes, 0);
  B.frontier.assign(nodes, 0);
  B.fwd_off.assign(nodes, -1);
  B.rec_off.assign(nodes, -1);
  B.grad_off.assign(nodes, -1);
  B.fuse_chain.assign(p.chains.size(), 0);
  const bool chains_on = fuse && !(p.flags & 64u);
  for (size_t g = 0; g < p.chains.size(); ++g) {
    bool one = chains_on;
    for (int k = p.chains[g].first; k <= p.chains[g].last; ++k)
      one &= blk[pos_of[k]] == blk[pos_of[p.chains[g].first]];
    B.fuse_chain[g] = one;
  }
  const double iters = std::ldexp(1.0, p.outer_bits);
  BwdEval ev;
  for (int v = n; v < nodes; ++v) {
    const int k = v - n;
    if (v == root) {
      B.keep[v] = 2;
      continue;
    }
    const int kc = cons[v];
    if (p.steps[k].phase != p.steps[kc].phase) {
      B.keep[v] = 1;
      B.frontier[v] = 1;
    } else if (blk[pos_of[k]] != blk[pos_of[kc]]) {
      B.keep[v] = 1;
    } else {
      B.keep[v] = 0;
      ev.recompute += p.steps[k].cmac * (p.steps[k].phase ? iters : 1.0);
    }
  }
  auto bytes = [&](int v) { return p.steps[v - n].c_bytes; };
  Arena ar;
  auto forward = [&](int q0, int q1) {
    for (int q = q0; q < q1; ++q) {
      const int k = p.sched[q];
      const StepDesc& S = p.steps[k];
      const bool fused = S.chain >= 0 && B.fuse_chain[S.chain];
      if (fused && p.chains[S.chain].last != k) continue;
      const int v = n + k;
      B.fwd_off[v] = ar.alloc(bytes(v));
      std::vector<int> ins;
      if (fused) {
        const ChainGroup& g = p.chains[S.chain];
        ins.push_back(p.steps[g.first].a);
        for (int j = g.first; j <= g.last; ++j) ins.push_back(p.steps[j].b);
      } else {
        ins = {S.a, S.b};
      }
      for (int x : ins)
        if (x >= n && B.keep[x] == 0) ar.release(B.fwd_off[x], bytes(x));
      if (B.keep[v] == 2) ar.release(B.fwd_off[v], bytes(v));
    }
  };
  // blocks of a phase, as [begin, end) position ranges
  auto blocks_of = [&](int q0, int q1) {
    std::vector<std::pair<int, int>> r;
    for (int q = q0; q < q1;) {
      int e = q;
      while (e < q1 && blk[e] == blk[q]) ++e;
      r.push_back({q, e});
      q = e;
    }
    return r;
  };
  auto adjoint = [&](int q0, int q1, int ph) {
    auto bl = blocks_of(q0, q1);
    for (int bi = (int)bl.size() - 1; bi >= 0; --bi) {
      const int b0 = bl[bi].first, b1 = bl[bi].second;
      for (int q = b0; q < b1; ++q) {
        const int v = n + p.sched[q];
        if (B.keep[v] == 0) B.rec_off[v] = ar.alloc(bytes(v));
      }
      for (int q = b1 - 1; q >= b0; --q) {
        const StepDesc& S = p.steps[p.sched[q]];
        for (int x : {S.a, S.b})
          if (x >= n && B.grad_off[x] < 0) B.grad_off[x] = ar.alloc(bytes(x));
        ar.release(B.grad_off[S.c], bytes(S.c));
        for (int x : {S.a, S.b}) {
          if (x < n) continue;
          if (B.keep[x] == 0) ar.release(B.rec_off[x], bytes(x));
          else if (!(B.frontier[x] && ph == 1)) ar.release(B.fwd_off[x], bytes(x));
        }
      }
    }
  };
  const int n0 = p.n_phase0;
  forward(0, n0);
  if (n0 < N) {
    for (int v = n; v < nodes; ++v)
      if (B.frontier[v]) B.grad_off[v] = ar.alloc(bytes(v));
    forward(n0, N);
    B.grad_off[root] = ar.alloc(bytes(root));
    adjoint(n0, N, 1);
    for (int v = n; v < nodes; ++v)
      if (B.frontier[v]) ar.release(B.fwd_off[v], bytes(v));
  } else {
    B.grad_off[root] = ar.alloc(bytes(root));
  }
  adjoint(0, n0, 0);
  ev.peak = ar.top;
  B.arena_bytes = ar.top;
  B.cmac_recompute = ev.recompute;
  B.block_begin.clear();
  for (int q = 0; q < N; ++q)
    if (q == 0 || blk[q] != blk[q - 1]) B.block_begin.push_back(q);
  if (out) *out = std::move(B);
  return ev;
}

// Blocks grown along each phase until their results hold at least T bytes,
// never cutting inside a fused chain.
std::vector<int32_t> blocks_by_bytes(const Plan& p, int64_t T, bool fuse) {
  const int n = p.n_tensors, N = (int)p.sched.size();
  std::vector<int32_t> pos_of(n - 1, -1);
  for (int q = 0; q < N; ++q) pos_of[p.sched[q]] = q;
  std::vector<uint8_t> no_cut_after(N, 0);
  if (fuse && !(p.flags & 64u))
    for (const ChainGroup& g : p.chains) {
      int lo = N, hi = -1;
      for (int k = g.first; k <= g.last; ++k) {
        lo = std::min(lo, pos_of[k]);
        hi = std::max(hi, pos_of[k]);
      }
      for (int q = lo; q < hi; ++q) no_cut_after[q] = 1;
    }
  std::vector<int32_t> blk(N, 0);
  int id = 0;
  int64_t acc = 0;
  for (int q = 0; q < N; ++q) {
    blk[q] = id;
    acc += align_up(p.steps[p.sched[q]].c_bytes, 256);
    const bool phase_end = q + 1 == p.n_phase0;
    if (q + 1 < N && (phase_end || (acc >= T && !no_cut_after[q]))) {
      ++id;
      acc = 0;
    }
  }
  return blk;
}

}  // namespace

static void plan_backward(Plan& p, int64_t budget) {
  const int n = p.n_tensors, nsteps = n - 1;
  p.bwd = BwdPlan();
  if (nsteps == 0) {
    p.workspace_bwd_bytes = 256;
    return;
  }
  // split-k scratch: forward steps, and the adjoint products (same bit
  // counts permuted among the classes)
  int64_t bscr = p.scratch_bytes;
  for (const StepDesc& S : p.steps) {
    int nb = (int)S.bA.size(), nm = (int)S.mA.size(), nnb = (int)S.nB.size(), nk = (int)S.kA.size();
    int32_t ch;
    int64_t sc;
    choose_kind(nb, nm, nk, nnb, p.flags, &ch, &sc);  // dA: rows m, cols k, sum n
    bscr = std::max(bscr, sc);
    choose_kind(nb, nk, nnb, nm, p.flags, &ch, &sc);  // dB: rows k, cols n, sum m
    bscr = std::max(bscr, sc);
  }
  const int N = (int)p.sched.size();
  std::vector<int32_t> all(N);
  std::iota(all.begin(), all.end(), 0);
  BwdEval e_all = simulate_backward(p, all, false, nullptr);
  auto total = [&](int64_t arena) { return align_up(arena, 256) + align_up(bscr, 256) + 256; };
  const bool all_fits = budget <= 0 || total(e_all.peak) <= budget;
  if (p.ckpt_policy == CKPT_ALL || (p.ckpt_policy == CKPT_AUTO && all_fits)) {
    simulate_backward(p, all, false, &p.bwd);
    p.bwd.policy = CKPT_ALL;
  } else {
    // thresholds on the bytes a block produces, doubling; keep the one with
    // the least recomputation that fits the budget (else the smallest peak)
    int64_t lo = 256, hi = 0;
    for (const StepDesc& S : p.steps) hi += align_up(S.c_bytes, 256);
    std::vector<int32_t> best_blk;
    BwdEval best;
    bool best_fits = false;
    for (double Tf = (double)lo; Tf <= 2.0 * (double)hi; Tf *= 1.41421356) {
      const int64_t T = (int64_t)Tf;
      std::vector<int32_t> blk = blocks_by_bytes(p, T, true);
      BwdEval e = simulate_backward(p, blk, true, nullptr);
      const bool fits = budget <= 0 || total(e.peak) <= budget;
      if (best_blk.empty() || (fits && !best_fits) ||
          (fits && best_fits && e.recompute < best.recompute) ||
          (!fits && !best_fits && e.peak < best.peak)) {
        best_blk = blk;
        best = e;
        best_fits = fits;
      }
    }
    simulate_backward(p, best_blk, true, &p.bwd);
    p.bwd.policy = CKPT_RECOMPUTE;
  }
  p.bwd.scratch_bytes = bscr;
  p.workspace_bwd_bytes = total(p.bwd.arena_bytes);
}

std::string build_plan(Plan& p, int32_t n_tensors, const int32_t* ranks,
                       const int32_t* index_ids, int32_t n_index, const int32_t* index_dims,
                       int32_t n_open, const int32_t* open_ids, int32_t n_steps,
                       const int32_t* path, int32_t n_sliced, const int32_t* sliced_ids,
                       int32_t precision, int32_t max_resident_bits, int64_t ws_limit,
                       uint32_t flags, int32_t gemm_config, const int32_t* tune, int32_t n_tune,
                       int32_t ckpt_policy, const int32_t* variable_leaves, int32_t n_variable,
                       bool* unsupported) {
  *unsupported = false;
  if (n_variable < 0 || (n_variable > 0 && !variable_leaves)) return "bad variable leaf list";
  p.leaf_variable.assign(n_tensors > 0 ? n_tensors : 0, 0);
  for (int32_t i = 0; i < n_variable; ++i) {
    const int32_t t = variable_leaves[i];
    if (t < 0 || t >= n_tensors) return "variable leaf out of range";
    p.leaf_variable[t] = 1;
  }
  if (ckpt_policy < CKPT_AUTO || ckpt_policy > CKPT_RECOMPUTE) return "unknown checkpoint policy";
  p.ckpt_policy = ckpt_policy;
  if (gemm_config >= kNumGemmConfigs) return "gemm_config out of range";
  if (n_tune < 0 || (n_tune > 0 && !tune)) return "bad tune table";
  p.gemm_config = gemm_config < 0 ? -1 : gemm_config;
  p.tune.assign(tune, tune + 5 * (int64_t)n_tune);
  char buf[256];
  if (n_tensors < 1) return "n_tensors must be >= 1";
  if (n_index < 0 || n_open < 0 || n_sliced < 0) return "negative count";
  if (!ranks || (n_index > 0 && !index_dims)) return "null array";
  if (precision != PREC_C64 && precision != PREC_SPLIT_BF16) return "unknown precision";
  p.n_tensors = n_tensors;
  p.n_index = n_index;
  p.precision = precision;
  p.flags = flags;
  p.index_dims.assign(index_dims, index_dims + n_index);
  p.index_w.assign(n_index, 0);
  p.index_bit0.assign(n_index, 0);
  int nbits = 0;
  for (int i = 0; i < n_index; ++i) {
    int d = index_dims[i];
    if (d < 2) {
      snprintf(buf, sizeof buf, "index %d has dimension %d (< 2)", i, d);
      return buf;
    }
    if ((d & (d - 1)) != 0 || d > 65536) {
      *unsupported = true;
      snprintf(buf, sizeof buf, "index %d has dimension %d (not a power of two <= 65536)", i, d);
      return buf;
    }
    int w = 0;
    while ((1 << w) < d) ++w;
    p.index_w[i] = w;
    p.index_bit0[i] = nbits;
    nbits += w;
  }
  p.n_bits = nbits;
  // leaves
  p.leaf_index.assign(n_tensors, {});
  std::vector<int> count(n_index, 0);
  int64_t off = 0;
  for (int t = 0; t < n_tensors; ++t) {
    if (ranks[t] < 0) return "negative rank";
    for (int j = 0; j < ranks[t]; ++j) {
      int id = index_ids[off + j];
      if (id < 0 || id >= n_index) {
        snprintf(buf, sizeof buf, "tensor %d lists unknown index %d", t, id);
        return buf;
      }
      for (int q : p.leaf_index[t])
        if (q == id) {
          snprintf(buf, sizeof buf, "tensor %d lists index %d twice", t, id);
          return buf;
        }
      p.leaf_index[t].push_back(id);
      count[id]++;
    }
    off += ranks[t];
  }
  p.open_ids.assign(open_ids, open_ids + n_open);
  p.sliced_ids.assign(sliced_ids, sliced_ids + n_sliced);
  std::vector<uint8_t> is_open(n_index, 0), is_sl(n_index, 0);
  for (int e : p.open_ids) {
    if (e < 0 || e >= n_index || is_open[e]) return "open index unknown or repeated";
    is_open[e] = 1;
  }
  for (int e : p.sliced_ids) {
    if (e < 0 || e >= n_index || is_sl[e]) return "sliced index unknown or repeated";
    if (is_open[e]) return "an open index cannot be sliced";
    is_sl[e] = 1;
  }
  for (int i = 0; i < n_index; ++i) {
    if (is_open[i]) {
      if (count[i] < 1) {
        snprintf(buf, sizeof buf, "open index %d appears in no tensor", i);
        return buf;
      }
    } else if (count[i] != 2) {
      snprintf(buf, sizeof buf, "index %d appears in %d tensors (must be 2 unless open)", i,
               count[i]);
      return buf;
    }
  }
  // path
  if (n_steps != n_tensors - 1) return "path must have n_tensors - 1 steps";
  if (n_steps > 0 && !path) return "null path";
  p.path.assign(path, path + 2 * n_steps);
  {
    std::vector<uint8_t> used(n_tensors + n_steps, 0);
    for (int k = 0; k < n_steps; ++k) {
      int a = p.path[2 * k], b = p.path[2 * k + 1];
      if (a < 0 || b < 0 || a >= n_tensors + k || b >= n_tensors + k || a == b || used[a] ||
          used[b]) {
        snprintf(buf, sizeof buf, "path step %d (%d, %d) is not a valid SSA pair", k, a, b);
        return buf;
      }
      used[a] = used[b] = 1;
    }
  }
  // bits
  p.bit_kept.assign(nbits, 0);
  p.bit_sliced.assign(nbits, 0);
  for (int i = 0; i < n_index; ++i)
    for (int j = 0; j < p.index_w[i]; ++j) {
      p.bit_kept[p.index_bit0[i] + j] = is_open[i] || is_sl[i];
      p.bit_sliced[p.index_bit0[i] + j] = is_sl[i];
    }
  p.leaves.assign(n_tensors, LeafDesc());
  const int nn_nodes = n_tensors + n_steps;
  p.node_bits.assign(nn_nodes, {});
  for (int t = 0; t < n_tensors; ++t) {
    LeafDesc& L = p.leaves[t];
    int s = 0;
    for (int ax = (int)p.leaf_index[t].size() - 1; ax >= 0; --ax) {
      int e = p.leaf_index[t][ax];
      for (int j = 0; j < p.index_w[e]; ++j) {
        L.bits.push_back(p.index_bit0[e] + j);
        L.log2s.push_back((int8_t)(s + j));
      }
      s += p.index_w[e];
    }
    if (s > kMaxTensorBits) {
      *unsupported = true;
      return "a leaf has more than 2^40 elements";
    }
    p.node_bits[t] = L.bits;
    std::sort(p.node_bits[t].begin(), p.node_bits[t].end());
  }
  for (int k = 0; k < n_steps; ++k) {
    const Bits& A = p.node_bits[p.path[2 * k]];
    const Bits& B = p.node_bits[p.path[2 * k + 1]];
    Bits common = inter(A, B);
    Bits summed;
    for (int x : common)
      if (!p.bit_kept[x]) summed.push_back(x);
    p.node_bits[n_tensors + k] = minus(unite(A, B), summed);
  }
  for (int x : p.node_bits[nn_nodes - 1])
    if (!p.bit_kept[x]) return "the path leaves an index unsummed";

  // all-resident statistics (independent of the outer split)
  p.n_slices = 1;
  int sl_bits = 0;
  for (int e : p.sliced_ids) sl_bits += p.index_w[e];
  p.sliced_bits = sl_bits;
  if (sl_bits > 40) {
    *unsupported = true;
    return "more than 2^40 slices";
  }
  p.n_slices = (int64_t)1 << sl_bits;
  p.cmac_reuse = p.cmac_sl = 0;
  p.max_log2_sl = 0;
  p.node_sv.assign(nn_nodes, 0);
  for (int v = 0; v < nn_nodes; ++v)
    for (int x : p.node_bits[v]) p.node_sv[v] += p.bit_sliced[x];
  for (int k = 0; k < n_steps; ++k) {
    Bits u = unite(p.node_bits[p.path[2 * k]], p.node_bits[p.path[2 * k + 1]]);
    int sv = 0;
    for (int x : u) sv += p.bit_sliced[x];
    p.cmac_reuse += std::ldexp(1.0, (int)u.size());
    p.cmac_sl += std::ldexp(1.0, (int)u.size() - sv);
    int v = n_tensors + k;
    p.max_log2_sl = std::max(p.max_log2_sl, (int32_t)p.node_bits[v].size() - p.node_sv[v]);
  }
  p.cmac_noreuse = p.cmac_sl * (double)p.n_slices;
  p.f_sl = p.n_slices > 1 ? (p.cmac_noreuse - p.cmac_reuse) / ((double)(p.n_slices - 1) * p.cmac_sl)
                          : 0.0;

  // outer / resident split
  p.outer_idx.clear();
  if (flags & 1u) {
    p.outer_idx = p.sliced_ids;
  }
  schedule(p);
  // TN_FLAG_FIT_BACKWARD: the backward's workspace must fit the limit too
  const bool fit_bwd = (flags & 256u) && ws_limit > 0;
  auto too_big = [&](Plan& q) {
    if (max_resident_bits >= 0 && q.resident_bits > max_resident_bits) return true;
    if (ws_limit > 0 && q.arena_bytes > ws_limit) return true;
    if (q.max_log2_res > kMaxTensorBits) return true;
    if (fit_bwd) {
      plan_backward(q, ws_limit);
      if (q.workspace_bwd_bytes > ws_limit) return true;
    }
    return false;
  };
  while (too_big(p)) {
    // move the sliced index whose outer looping makes the plan fit, else
    // costs the least work (then the smallest peak)
    int best = -1;
    bool best_fits = false;
    double best_cost = 0;
    int64_t best_peak = 0;
    std::vector<int32_t> base = p.outer_idx;
    for (int e : p.sliced_ids) {
      if (std::find(base.begin(), base.end(), e) != base.end()) continue;
      p.outer_idx = base;
      p.outer_idx.push_back(e);
      schedule(p);
      const bool fits = !too_big(p);
      const double cost = p.cmac_exec;
      if (best < 0 || (fits && !best_fits) ||
          (fits == best_fits &&
           (cost < best_cost || (cost == best_cost && p.arena_bytes < best_peak)))) {
        best = e;
        best_fits = fits;
        best_cost = cost;
        best_peak = p.arena_bytes;
      }
    }
    if (best < 0) {
      p.outer_idx = base;
      schedule(p);
      *unsupported = true;
      return "the workspace limit cannot be met even with every sliced index looped over";
    }
    p.outer_idx = base;
    p.outer_idx.push_back(best);
    schedule(p);
  }
  p.resident_idx.clear();
  for (int e : p.sliced_ids)
    if (std::find(p.outer_idx.begin(), p.outer_idx.end(), e) == p.outer_idx.end())
      p.resident_idx.push_back(e);
  for (const StepDesc& S : p.steps) {
    if ((int)S.bA.size() > kMaxBits || (int)S.mA.size() > kMaxBits ||
        (int)S.nB.size() > kMaxBits || (int)S.kA.size() > kMaxBits) {
      *unsupported = true;
      return "a step has more than 48 bits in one class";
    }
  }
  plan_backward(p, ws_limit);
  return "";
}

}  // namespace tn
