// Host-side tables of the Berends-Giele executor (see me_bg.h): every ordered
// sequence of distinct gluons of length 1 .. N, numbered shorter first and
// lexicographically within a length; for each, its gluon subset, its last gluon
// and the numbers of all its contiguous subsequences.
#pragma once
#include <cstdint>
#include <map>
#include <vector>

namespace me {

struct BgHostTables {
  int n = 0;
  int nslot = 0;
  int tri = 0;                  // entries per sequence in sub: n (n + 1) / 2
  std::vector<uint16_t> sub;    // [nslot][tri], entry b (b - 1) / 2 + a = number of s[a:b]
  std::vector<uint8_t> mask;    // [nslot]
  std::vector<uint8_t> last;    // [nslot]
};

inline void bg_sequences(int n, int len, std::vector<int>& cur, std::vector<bool>& used,
                         std::vector<std::vector<int>>& out) {
  if ((int)cur.size() == len) {
    out.push_back(cur);
    return;
  }
  for (int g = 0; g < n; ++g) {
    if (used[g]) continue;
    used[g] = true;
    cur.push_back(g);
    bg_sequences(n, len, cur, used, out);
    cur.pop_back();
    used[g] = false;
  }
}

// Every sequence of length 1 .. n, in slot order.
inline std::vector<std::vector<int>> bg_all_sequences(int n) {
  std::vector<std::vector<int>> seqs;
  for (int len = 1; len <= n; ++len) {
    std::vector<int> cur;
    std::vector<bool> used(n, false);
    bg_sequences(n, len, cur, used, seqs);
  }
  return seqs;
}

inline BgHostTables bg_build_tables(int n) {
  BgHostTables t;
  t.n = n;
  t.tri = n * (n + 1) / 2;
  const std::vector<std::vector<int>> seqs = bg_all_sequences(n);
  std::map<std::vector<int>, int> slot;
  for (int i = 0; i < (int)seqs.size(); ++i) slot[seqs[i]] = i;
  t.nslot = (int)seqs.size();
  t.sub.assign((size_t)t.nslot * t.tri, 0);
  t.mask.assign(t.nslot, 0);
  t.last.assign(t.nslot, 0);
  for (int i = 0; i < t.nslot; ++i) {
    const std::vector<int>& s = seqs[i];
    const int L = (int)s.size();
    int m = 0;
    for (int g : s) m |= 1 << g;
    t.mask[i] = (uint8_t)m;
    t.last[i] = (uint8_t)s.back();
    for (int b = 1; b <= L; ++b)
      for (int a = 0; a < b; ++a) {
        std::vector<int> part(s.begin() + a, s.begin() + b);
        t.sub[(size_t)i * t.tri + b * (b - 1) / 2 + a] = (uint16_t)slot.at(part);
      }
  }
  return t;
}

// Tables of the helicity-recycling kernel (me_bgh.h), n >= 4.  The full orderings
// fall into (n-1)! cycles under rotation, each represented by its ordering that
// starts with gluon 0 (cycle z = rank of that ordering among them, lexicographic).
// seg[z][start][len - 1] = slot of the segment of length len (1 .. n) starting at
// position start of the rotations of the representative (positions mod n).
// Stored currents (length L <= n-2) keep 2^L helicity variants, stored row spinors
// (length L <= n-3) 2 x 2^L (top helicity, then the gluons'): cbase / rbase =
// number of the first variant of each slot among all stored currents / rows
// (variants ordered by slot), 0 for slots not stored.
struct BgCycleHostTables {
  int ncyc = 0;
  std::vector<uint16_t> seg;
  std::vector<uint16_t> cbase;
  std::vector<uint16_t> rbase;
};

inline BgCycleHostTables bg_build_cycles(int n) {
  BgCycleHostTables c;
  const std::vector<std::vector<int>> seqs = bg_all_sequences(n);
  std::map<std::vector<int>, int> slot;
  for (int i = 0; i < (int)seqs.size(); ++i) slot[seqs[i]] = i;
  c.cbase.assign(seqs.size(), 0);
  c.rbase.assign(seqs.size(), 0);
  int nc = 0, nr = 0;
  for (int i = 0; i < (int)seqs.size(); ++i) {
    const int L = (int)seqs[i].size();
    if (L <= n - 2) {
      c.cbase[i] = (uint16_t)nc;
      nc += 1 << L;
    }
    if (L <= n - 3) {
      c.rbase[i] = (uint16_t)nr;
      nr += 2 << L;
    }
  }
  for (const std::vector<int>& s : seqs) {
    if ((int)s.size() != n || s[0] != 0) continue;
    for (int start = 0; start < n; ++start)
      for (int len = 1; len <= n; ++len) {
        std::vector<int> part;
        for (int k = 0; k < len; ++k) part.push_back(s[(start + k) % n]);
        c.seg.push_back((uint16_t)slot.at(part));
      }
    ++c.ncyc;
  }
  return c;
}

}  // namespace me
