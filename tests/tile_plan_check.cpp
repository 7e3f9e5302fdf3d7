// Checks the batched Euler step's tile plans on the host: for random domain
// layouts, every tile order and block width, and both boundary kinds, every
// slot's index and domain as the kernel derives them from the descriptor must
// equal the brute-force answer, the owned slots must cover all slots once in
// order, and each order must keep its own rule.  Periodic plans index slots by
// cell; transmissive plans, as the library builds them, index each domain's
// ghost slot followed by its cells (domain s spans off[s] + s .. off[s+1] + s),
// and the kernel's cell and ghost derivation must hold too, with every
// domain's first cell next to its ghost in the same tile.  Prints "ok <slots>"
// or the first failures; the exit status is the number of failures (capped).
#include <cstdio>
#include <random>
#include <vector>

#include "grprec_tiles.h"

using grp::Tile;

static int domain_of(const std::vector<int> &off, int c) {
  return int(std::upper_bound(off.begin(), off.end(), c) - off.begin()) - 1;
}

int main() {
  std::mt19937 rng(20260303u);
  long long slots = 0;
  int bad = 0;
  auto fail = [&](const char *what, int trial, int order, int block, int e) {
    if (bad < 8) std::printf("FAIL %s: layout %d order %d block %d slot %d\n", what, trial, order, block, e);
    ++bad;
  };
  for (int trial = 0; trial < 300; ++trial) {
    int S = 1 + int(rng() % 80);
    if (trial % 9 == 0) S = 1;
    std::vector<int> off(S + 1, 0);
    for (int s = 0; s < S; ++s) {
      // short domains (2..6 cells) in some layouts, else up to 600 cells
      // short domains (1..6 cells) in some layouts, else up to 600 cells
      const int n = (trial % 3 == 0) ? 1 + int(rng() % 6) : 2 + int(rng() % 599);
      off[s + 1] = off[s] + n;
    }
    const bool periodic = trial % 2 == 0;
    std::vector<int> xoff(S + 1);
    for (int s = 0; s <= S; ++s) xoff[s] = off[s] + (periodic ? 0 : s);
    const std::vector<int> cell_off = off;
    for (int order : {int(grp::kSegmentTiles), int(grp::kFlatTiles), int(grp::kPacked)}) {
      for (int block : {64, 128, 256}) {
        std::vector<int> dom_tile0;
        const std::vector<int> &off = xoff;  // the slot offsets the plan is built on
        const std::vector<Tile> tiles = grp::plan_tiles(off, order, block, periodic, dom_tile0);
        std::vector<int> ghost_slot(block, 0), cell_at(block, -2);
        int next_cell = 0;
        for (size_t k = 0; k < tiles.size(); ++k) {
          const Tile &d = tiles[k];
          if (d.count < 1 || d.count > block - 2) fail("count", trial, order, block, -1);
          if (d.start != next_cell) fail("cover", trial, order, block, -1);
          next_cell = d.start + d.count;
          const int z = domain_of(off, d.start), w = domain_of(off, d.start + d.count - 1);
          if (d.w != w) fail("last domain", trial, order, block, -1);
          if (order == grp::kSegmentTiles && z != w) fail("segment tile crosses a domain", trial, order, block, -1);
          if (order == grp::kPacked && z != w && (d.start != off[z] || d.start + d.count != off[w + 1]))
            fail("packed tile splits a short domain", trial, order, block, -1);
          for (int e = 0; e < block; ++e) {
            // the kernel's derivation
            bool valid = false;
            int c = 0;
            if (e >= 1 && e <= d.count) {
              c = d.start + e - 1;
              valid = true;
            } else if (e == 0) {
              c = d.cl;
              valid = c >= 0;
            } else if (e == d.count + 1) {
              c = d.cr;
              valid = c >= 0;
            }
            const int j = block > 64 ? (e >> 6) : 0;
            const int s = (e == d.count + 1)
                              ? d.w
                              : d.base[j] + __builtin_popcountll(d.first[j] & ((2ull << (e & 63)) - 1ull));
            // brute force
            int want_c = -1, want_s = -1;
            if (e >= 1 && e <= d.count) {
              want_c = d.start + e - 1;
              want_s = domain_of(off, want_c);
            } else if (e == 0) {
              want_s = z;
              want_c = d.start > off[z] ? d.start - 1 : (periodic ? off[z + 1] - 1 : -1);
            } else if (e == d.count + 1) {
              const int last = d.start + d.count - 1;
              want_s = w;
              want_c = last + 1 < off[w + 1] ? last + 1 : (periodic ? off[w] : -1);
            }
            cell_at[e] = -2;
            ghost_slot[e] = 0;
            if (want_c < 0) {
              if (valid) fail("halo slot without a cell", trial, order, block, e);
              continue;
            }
            ++slots;
            if (!valid || c != want_c) fail("cell", trial, order, block, e);
            if (s != want_s || domain_of(off, c) != s) fail("domain", trial, order, block, e);
            // the kernel's cell and ghost derivation from slot x = c and domain s
            const int x = c;
            const int cell = periodic ? x : (x - s - 1 > 0 ? x - s - 1 : 0);
            const bool ghost = !periodic && x == cell_off[s] + s;
            ghost_slot[e] = ghost;
            cell_at[e] = ghost ? -1 : cell;
            if (periodic && ghost) fail("ghost in a periodic plan", trial, order, block, e);
            if (!ghost && (cell < cell_off[s] || cell >= cell_off[s + 1])) fail("cell outside its domain", trial, order, block, e);
            if (!periodic && !ghost && x != cell + s + 1) fail("slot of a cell", trial, order, block, e);
          }
          // a domain's first cell (owned, or the right halo) has its ghost in
          // the slot before; an owned ghost has its first cell in the slot after
          if (!periodic) {
            for (int e = 0; e < block; ++e) {
              if (cell_at[e] >= 0 && e >= 1) {
                const int s = domain_of(cell_off, cell_at[e]);
                if (cell_at[e] == cell_off[s] && !ghost_slot[e - 1]) fail("first cell without its ghost", trial, order, block, e);
              }
              if (e >= 1 && e <= d.count && ghost_slot[e] && (e + 1 >= block || cell_at[e + 1] < 0))
                fail("ghost without its first cell", trial, order, block, e);
            }
          }
        }
        if (next_cell != off[S]) fail("slots left over", trial, order, block, -1);
        if (order == grp::kSegmentTiles) {
          if ((int)dom_tile0.size() != S + 1 || dom_tile0[S] != (int)tiles.size()) {
            fail("dom_tile0 size", trial, order, block, -1);
          } else {
            for (int s = 0; s < S; ++s)
              if (tiles[dom_tile0[s]].start != off[s]) fail("dom_tile0", trial, order, block, s);
          }
        }
      }
    }
  }
  if (bad == 0) std::printf("ok %lld\n", slots);
  return bad > 100 ? 100 : bad;
}
