// Host-only parts of the C ABI in include/dfb.h: the dependency-tree tracker
// for tiles that arrive one at a time (Sec. 3.1.1) and the variance-driven
// assignment of extra samples (Sec. 4.1.1).  Neither touches a GPU.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "../../include/dfb.h"
#include "dfb_tree.h"

struct dfb_tree_s {
  std::vector<dfb::TileTree> tiles;
};

namespace dfb {

dfb_status assign_samples(const float* variance, int32_t n_tiles, int64_t extra, int32_t* counts) {
  if (n_tiles <= 0 || !variance || !counts || extra < 0 || extra > INT32_MAX) return DFB_ERR_INVALID_ARG;
  std::vector<double> w(n_tiles);
  double S = 0.0;
  for (int32_t t = 0; t < n_tiles; ++t) {
    const float v = variance[t];
    w[t] = (std::isfinite(v) && v > 0.f) ? static_cast<double>(v) : 0.0;
    S += w[t];  // in tile order: the sum is part of the definition
  }
  if (!(S > 0.0)) {
    const int64_t base = extra / n_tiles, rest = extra % n_tiles;
    for (int32_t t = 0; t < n_tiles; ++t) counts[t] = static_cast<int32_t>(base + (t < rest ? 1 : 0));
    return DFB_OK;
  }
  std::vector<double> rem(n_tiles);
  int64_t given = 0;
  const double E = static_cast<double>(extra);
  for (int32_t t = 0; t < n_tiles; ++t) {
    const double q = E * w[t] / S;
    const double f = std::floor(q);
    counts[t] = static_cast<int32_t>(f);
    rem[t] = q - f;
    given += counts[t];
  }
  int64_t left = extra - given;
  if (left > 0) {
    std::vector<int32_t> order(n_tiles);
    for (int32_t t = 0; t < n_tiles; ++t) order[t] = t;
    const size_t k = static_cast<size_t>(std::min<int64_t>(left, n_tiles));
    std::partial_sort(order.begin(), order.begin() + k, order.end(), [&](int32_t a, int32_t b) {
      return rem[a] != rem[b] ? rem[a] > rem[b] : a < b;
    });
    for (size_t i = 0; i < k; ++i) counts[order[i]] += 1;
  }
  return DFB_OK;
}

}  // namespace dfb

extern "C" {

dfb_status dfb_assign_samples_host(const float* variance, int32_t n_tiles, int64_t extra, int32_t* counts) {
  return dfb::assign_samples(variance, n_tiles, extra, counts);
}

dfb_status dfb_tree_create(int32_t n_tiles, dfb_tree* out) {
  if (!out || n_tiles < 1) return DFB_ERR_INVALID_ARG;
  *out = nullptr;
  dfb_tree_s* t = new (std::nothrow) dfb_tree_s();
  if (!t) return DFB_ERR_OOM;
  try {
    t->tiles.resize(n_tiles);
  } catch (...) {
    delete t;
    return DFB_ERR_OOM;
  }
  for (auto& x : t->tiles) x.reset();
  *out = t;
  return DFB_OK;
}

dfb_status dfb_tree_destroy(dfb_tree t) {
  if (!t) return DFB_ERR_INVALID_ARG;
  delete t;
  return DFB_OK;
}

dfb_status dfb_tree_new_frame(dfb_tree t) {
  if (!t) return DFB_ERR_INVALID_ARG;
  for (auto& x : t->tiles) x.reset();
  return DFB_OK;
}

dfb_status dfb_tree_add(dfb_tree t, int32_t tile_id, int32_t generation, int32_t children, int32_t* completed) {
  if (completed) *completed = 0;
  if (!t || tile_id < 0 || tile_id >= static_cast<int32_t>(t->tiles.size()) || generation < 0 ||
      generation > dfb::kMaxGeneration || children < 0)
    return DFB_ERR_INVALID_ARG;
  bool done = false;
  bool ok;
  try {
    ok = t->tiles[tile_id].add(generation, children, done);
  } catch (...) {
    return DFB_ERR_OOM;
  }
  if (!ok) return DFB_ERR_TREE;
  if (completed) *completed = done ? 1 : 0;
  return DFB_OK;
}

dfb_status dfb_tree_query(dfb_tree t, int32_t tile_id, int32_t* state, int32_t* generation, int32_t* missing) {
  if (!t || tile_id < 0 || tile_id >= static_cast<int32_t>(t->tiles.size())) return DFB_ERR_INVALID_ARG;
  const dfb::TileTree& x = t->tiles[tile_id];
  if (state) *state = x.state();
  if (generation) *generation = x.generation();
  if (missing) *missing = static_cast<int32_t>(std::min<int64_t>(x.missing(), INT32_MAX));
  return DFB_OK;
}

}  // extern "C"
