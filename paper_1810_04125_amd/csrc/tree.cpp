// Cluster tree construction on the host (Sec. 2.1: binary tree numbered
// level by level from 0 at the root, contiguous index ranges, children
// partition the parent).  Splitting rule: floor(m/2) left, rest right;
// index bisection, recursive coordinate bisection (axis of largest extent,
// ties to the lowest axis) or kd (axis = depth mod 3); points ordered by
// (coordinate, original index); indices inside a leaf ascend.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <vector>

#include "hss_internal.h"

namespace hss {

struct TreeBuild {
  std::vector<int32_t> lo, hi, left, right, parent, level;
  std::vector<std::vector<int64_t>> members;
};

static void build(int64_t n, const double* pts, int32_t leaf, int32_t method, TreeBuild& T) {
  std::deque<int32_t> q;
  T.lo.push_back(0); T.hi.push_back((int32_t)n); T.left.push_back(-1); T.right.push_back(-1);
  T.parent.push_back(-1); T.level.push_back(0);
  T.members.emplace_back(n);
  for (int64_t i = 0; i < n; ++i) T.members[0][i] = i;
  q.push_back(0);
  while (!q.empty()) {
    const int32_t t = q.front();
    q.pop_front();
    std::vector<int64_t> idx = std::move(T.members[t]);
    const int64_t m = (int64_t)idx.size();
    if (m <= leaf) {
      std::sort(idx.begin(), idx.end());
      T.members[t] = std::move(idx);
      continue;
    }
    if (method != 0) {
      int axis = 0;
      if (method == 1) {
        double best = -1.0;
        for (int a = 0; a < 3; ++a) {
          double mn = pts[3 * idx[0] + a], mx = mn;
          for (int64_t i : idx) {
            const double v = pts[3 * i + a];
            mn = std::min(mn, v);
            mx = std::max(mx, v);
          }
          const double ext = mx - mn;
          if (a == 0 || ext > best) { best = ext; axis = a; }
        }
      } else {
        axis = T.level[t] % 3;
      }
      std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
        const double vx = pts[3 * x + axis], vy = pts[3 * y + axis];
        return vx < vy || (vx == vy && x < y);
      });
    }
    const int64_t half = m / 2;
    for (int part = 0; part < 2; ++part) {
      const int64_t a = part == 0 ? 0 : half, b = part == 0 ? half : m;
      const int32_t c = (int32_t)T.lo.size();
      T.lo.push_back(T.lo[t] + (int32_t)a);
      T.hi.push_back(T.lo[t] + (int32_t)b);
      T.left.push_back(-1); T.right.push_back(-1);
      T.parent.push_back(t);
      T.level.push_back(T.level[t] + 1);
      T.members.emplace_back(idx.begin() + a, idx.begin() + b);
      if (part == 0) T.left[t] = c; else T.right[t] = c;
      q.push_back(c);
    }
  }
}

hss_tree* tree_build(int64_t n, const double* pts, int32_t leaf, int32_t method) {
  if (n < 1 || n > 0x7fffffff || leaf < 1 || method < 0 || method > 2)
    throw Error(HSS_ERR_INVALID_ARG, "tree_build: need 1 <= n < 2^31, leaf_size >= 1, method in {0,1,2}");
  if (method != 0) {
    if (!pts) throw Error(HSS_ERR_INVALID_ARG, "tree_build: RCB / kd need points");
    for (int64_t i = 0; i < 3 * n; ++i)
      if (!std::isfinite(pts[i])) throw Error(HSS_ERR_INVALID_ARG, "tree_build: non-finite point");
  }
  TreeBuild T;
  build(n, pts, leaf, method, T);
  const int32_t nn = (int32_t)T.lo.size();
  hss_tree* out = (hss_tree*)std::calloc(1, sizeof(hss_tree));
  out->n = n;
  out->num_nodes = nn;
  out->perm = (int64_t*)std::malloc(sizeof(int64_t) * n);
  int32_t** arrs[6] = {&out->lo, &out->hi, &out->left, &out->right, &out->parent, &out->level};
  const std::vector<int32_t>* src[6] = {&T.lo, &T.hi, &T.left, &T.right, &T.parent, &T.level};
  for (int k = 0; k < 6; ++k) {
    *arrs[k] = (int32_t*)std::malloc(sizeof(int32_t) * nn);
    std::memcpy(*arrs[k], src[k]->data(), sizeof(int32_t) * nn);
  }
  for (int32_t t = 0; t < nn; ++t)
    if (T.left[t] < 0)
      for (int64_t i = 0; i < (int64_t)T.members[t].size(); ++i) out->perm[T.lo[t] + i] = T.members[t][i];
  return out;
}

void tree_free(hss_tree* t) {
  if (!t) return;
  std::free(t->perm);
  std::free(t->lo); std::free(t->hi); std::free(t->left); std::free(t->right);
  std::free(t->parent); std::free(t->level);
  std::free(t);
}

}  // namespace hss
