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

inline BgHostTables bg_build_tables(int n) {
  BgHostTables t;
  t.n = n;
  t.tri = n * (n + 1) / 2;
  std::vector<std::vector<int>> seqs;
  for (int len = 1; len <= n; ++len) {
    std::vector<int> cur;
    std::vector<bool> used(n, false);
    bg_sequences(n, len, cur, used, seqs);
  }
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

}  // namespace me
