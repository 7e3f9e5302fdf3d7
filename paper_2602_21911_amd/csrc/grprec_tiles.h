// Tile plans of the batched Euler step (host side, plain C++).
//
// A tile is a run of consecutive cells of the concatenated domains that one
// block advances: `count` owned cells in slots 1..count of the block and the
// halo cells next to them in slots 0 and count+1.  The kernels find every
// slot's cell and domain from the tile's descriptor alone.
#pragma once

#include <algorithm>
#include <cstring>
#include <vector>

namespace grp {

// Tile descriptor (80 bytes).  Bit k of first[j] marks slot 64j+k (only
// slots 2..count are marked) as the first cell of a domain; base[j] is the
// domain of the slots of word j that precede its first mark, so slot e
// (1 <= e <= count) lies in domain
//     base[e/64] + popcount(first[e/64] & ((2 << (e%64)) - 1)),
// slot 0 (a halo) in base[0], and slot count+1 (a halo) in w.
struct alignas(16) Tile {
  int start, count;
  int cl, cr;                  // halo cells of slots 0 and count+1, -1 when none
  int w, pad[3];               // domain of the last owned cell
  int base[4];
  unsigned long long first[4];
};

// Tile orders; the values are those of the GRPREC_SCHED_* constants.
enum TileOrder { kSegmentTiles = 1, kFlatTiles = 2, kPacked = 3 };

// Descriptor of the tile of `count` cells from `start`, whose first and last
// cells lie in domains z and w of the domain offsets `off` (off[s] is the
// first cell of domain s, off[S] the total).  Periodic domains wrap their
// halo cells around the domain.
inline Tile make_tile(int start, int count, int z, int w, const std::vector<int> &off, bool periodic) {
  Tile d;
  std::memset(&d, 0, sizeof(d));
  d.start = start;
  d.count = count;
  d.w = w;
  d.cl = start > off[z] ? start - 1 : (periodic ? off[z + 1] - 1 : -1);
  const int last = start + count - 1;
  d.cr = last + 1 < off[w + 1] ? last + 1 : (periodic ? off[w] : -1);
  int s = z;
  for (int e = 0; e < 256; ++e) {
    if ((e & 63) == 0) d.base[e >> 6] = s;
    if (e >= 2 && e <= count && start + e - 1 == off[s + 1]) {
      ++s;
      d.first[e >> 6] |= 1ull << (e & 63);
    }
  }
  return d;
}

// Tiles of at most block-2 owned cells over all domains, in one of the tile
// orders; dom_tile0 receives, for segment tiles, the first tile of each
// domain (and the total at [S]).  Domains hold at least one cell.
inline std::vector<Tile> plan_tiles(const std::vector<int> &off, int order, int block, bool periodic,
                                    std::vector<int> &dom_tile0) {
  struct Run {
    int start, count, z, w;
  };
  const int T = block - 2;
  const int S = (int)off.size() - 1;
  const long long tc = off[S];
  std::vector<Run> t;
  auto seg_of = [&](int c) {
    return int(std::upper_bound(off.begin(), off.end(), c) - off.begin()) - 1;
  };
  if (order == kFlatTiles) {
    for (long long st = 0; st < tc; st += T) {
      const int cnt = (int)std::min<long long>(T, tc - st);
      t.push_back({(int)st, cnt, seg_of((int)st), seg_of((int)(st + cnt - 1))});
    }
  } else if (order == kPacked) {
    int cur_start = -1, cur_cnt = 0, cur_s0 = 0;
    auto flush = [&](int last_seg) {
      if (cur_cnt > 0) t.push_back({cur_start, cur_cnt, cur_s0, last_seg});
      cur_cnt = 0;
      cur_start = -1;
    };
    for (int s = 0; s < S; ++s) {
      const int n = off[s + 1] - off[s];
      if (n > T) {
        flush(s - 1);
        const int pieces = (n + T - 1) / T;
        const int base = n / pieces, extra = n % pieces;
        int st = off[s];
        for (int k = 0; k < pieces; ++k) {
          const int cnt = base + (k < extra ? 1 : 0);
          t.push_back({st, cnt, s, s});
          st += cnt;
        }
      } else {
        if (cur_cnt + n > T) flush(s - 1);
        if (cur_cnt == 0) {
          cur_start = off[s];
          cur_s0 = s;
        }
        cur_cnt += n;
      }
    }
    flush(S - 1);
  } else {  // segment tiles (also the per-domain launches)
    dom_tile0.assign(S + 1, 0);
    for (int s = 0; s < S; ++s) {
      dom_tile0[s] = (int)t.size();
      for (int st = off[s]; st < off[s + 1]; st += T) t.push_back({st, std::min(T, off[s + 1] - st), s, s});
    }
    dom_tile0[S] = (int)t.size();
  }
  std::vector<Tile> d;
  d.reserve(t.size());
  for (const Run &r : t) d.push_back(make_tile(r.start, r.count, r.z, r.w, off, periodic));
  return d;
}

}  // namespace grp
