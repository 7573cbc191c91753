// Host construction of the sparse voxel octree (SVLF section 4.1, "Scene
// volume"): only occupied leaves and their ancestors are stored, and every
// vertex of an occupied leaf owns one feature row shared by the adjacent
// leaves.
//
// Layout produced (see svlf.h): internal nodes in level order, each level in
// ascending Morton order, 8-byte records {first child, child mask}; leaves
// ranked by Morton code; vertices ranked by the Morton code of their (L+1)-bit
// lattice coordinates; leaf_corners[leaf][j] = vertex id of corner j.
#include <algorithm>
#include <cstring>
#include <thread>
#include <utility>
#include <vector>

#include "svlf_internal.hpp"

namespace svlf {
namespace {

inline uint64_t spread3(uint64_t v) {
  // insert two zero bits between the low 21 bits of v
  v &= 0x1FFFFFull;
  v = (v | (v << 32)) & 0x1F00000000FFFFull;
  v = (v | (v << 16)) & 0x1F0000FF0000FFull;
  v = (v | (v << 8)) & 0x100F00F00F00F00Full;
  v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

inline uint64_t morton(uint64_t i, uint64_t j, uint64_t k) {
  return spread3(i) | (spread3(j) << 1) | (spread3(k) << 2);
}

inline uint32_t compact3(uint64_t v) {
  v &= 0x1249249249249249ull;
  v = (v | (v >> 2)) & 0x10C30C30C30C30C3ull;
  v = (v | (v >> 4)) & 0x100F00F00F00F00Full;
  v = (v | (v >> 8)) & 0x1F0000FF0000FFull;
  v = (v | (v >> 16)) & 0x1F00000000FFFFull;
  v = (v | (v >> 32)) & 0x1FFFFFull;
  return static_cast<uint32_t>(v);
}

// Sort pairs with a few threads: sort chunks, then merge pairwise.
template <class T>
void par_sort(std::vector<T>& v) {
  const size_t n = v.size();
  unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < (1u << 20) || hw == 1) {
    std::sort(v.begin(), v.end());
    return;
  }
  size_t parts = 1;
  while (parts * 2 <= hw) parts *= 2;
  std::vector<size_t> cut(parts + 1);
  for (size_t p = 0; p <= parts; ++p) cut[p] = n * p / parts;
  {
    std::vector<std::thread> th;
    for (size_t p = 0; p < parts; ++p)
      th.emplace_back([&, p] { std::sort(v.begin() + cut[p], v.begin() + cut[p + 1]); });
    for (auto& t : th) t.join();
  }
  for (size_t w = 1; w < parts; w *= 2) {
    std::vector<std::thread> th;
    for (size_t p = 0; p + w < parts; p += 2 * w) {
      size_t a = cut[p], b = cut[p + w], c = cut[std::min(parts, p + 2 * w)];
      th.emplace_back([&, a, b, c] {
        std::inplace_merge(v.begin() + a, v.begin() + b, v.begin() + c);
      });
    }
    for (auto& t : th) t.join();
  }
}

}  // namespace

int build_octree_host(const int32_t* ijk, int64_t n, int depth, HostOctree* out,
                      bool want_arrays) {
  if (n < 0) {
    set_error("svlf_build_octree: n < 0");
    return SVLF_E_INVAL;
  }
  if (depth < 1 || depth > SVLF_MAX_DEPTH) {
    set_error("svlf_build_octree: depth must be in [1, " + std::to_string(SVLF_MAX_DEPTH) + "]");
    return SVLF_E_RANGE;
  }
  if (n > 0 && ijk == nullptr) {
    set_error("svlf_build_octree: leaf_ijk is NULL");
    return SVLF_E_INVAL;
  }
  const int64_t side = int64_t(1) << depth;
  if (n > (int64_t(1) << 31) - 1) {
    set_error("svlf_build_octree: too many leaves for int32 ids");
    return SVLF_E_RANGE;
  }
  std::vector<std::pair<uint64_t, uint32_t>> leaf(n);
  for (int64_t q = 0; q < n; ++q) {
    const int32_t i = ijk[3 * q], j = ijk[3 * q + 1], k = ijk[3 * q + 2];
    if (i < 0 || j < 0 || k < 0 || i >= side || j >= side || k >= side) {
      set_error("svlf_build_octree: leaf " + std::to_string(q) + " has a coordinate outside [0, 2^depth)");
      return SVLF_E_RANGE;
    }
    leaf[q] = {morton(i, j, k), static_cast<uint32_t>(q)};
  }
  par_sort(leaf);
  for (int64_t q = 1; q < n; ++q) {
    if (leaf[q].first == leaf[q - 1].first) {
      set_error("svlf_build_octree: duplicate leaf");
      return SVLF_E_INVAL;
    }
  }
  // node codes per level, level L = leaves
  std::vector<std::vector<uint64_t>> codes(depth + 1);
  codes[depth].resize(n);
  for (int64_t q = 0; q < n; ++q) codes[depth][q] = leaf[q].first;
  for (int l = depth - 1; l >= 0; --l) {
    auto& c = codes[l];
    const auto& f = codes[l + 1];
    c.reserve(f.size() / 2 + 1);
    for (size_t q = 0; q < f.size(); ++q) {
      const uint64_t p = f[q] >> 3;
      if (c.empty() || c.back() != p) c.push_back(p);
    }
  }
  svlf_octree_sizes& sz = out->sizes;
  std::memset(&sz, 0, sizeof(sz));
  sz.depth = depth;
  sz.n_leaves = n;
  int64_t off = 0;
  for (int l = 0; l < depth; ++l) {
    sz.level_offset[l] = off;
    off += static_cast<int64_t>(codes[l].size());
  }
  sz.level_offset[depth] = off;
  sz.n_nodes = off;
  if (off > (int64_t(1) << 31) - 1) {
    set_error("svlf_build_octree: too many nodes");
    return SVLF_E_RANGE;
  }
  // vertices: (corner code, leaf*8 + j), sorted
  std::vector<std::pair<uint64_t, uint32_t>> corner(static_cast<size_t>(n) * 8);
  for (int64_t q = 0; q < n; ++q) {
    const uint64_t code = leaf[q].first;
    const uint64_t i = compact3(code), j = compact3(code >> 1), k = compact3(code >> 2);
    for (int c = 0; c < 8; ++c)
      corner[8 * q + c] = {morton(i + (c & 1), j + ((c >> 1) & 1), k + (c >> 2)),
                           static_cast<uint32_t>(8 * q + c)};
  }
  par_sort(corner);
  int64_t nv = 0;
  if (want_arrays) out->leaf_corners.assign(static_cast<size_t>(n) * 8, -1);
  for (size_t q = 0; q < corner.size(); ++q) {
    if (q > 0 && corner[q].first != corner[q - 1].first) ++nv;
    if (want_arrays) out->leaf_corners[corner[q].second] = static_cast<int32_t>(nv);
  }
  sz.n_vertices = n > 0 ? nv + 1 : 0;
  if (!want_arrays) return SVLF_OK;

  out->nodes.assign(static_cast<size_t>(sz.n_nodes), svlf_node{0, 0});
  for (int l = 0; l < depth; ++l) {
    const auto& par = codes[l];
    const auto& kid = codes[l + 1];
    const int64_t base_here = sz.level_offset[l];
    const int64_t base_kids = (l + 1 < depth) ? sz.level_offset[l + 1] : 0;
    size_t pi = 0;
    for (size_t q = 0; q < kid.size(); ++q) {
      const uint64_t p = kid[q] >> 3;
      while (par[pi] != p) ++pi;
      svlf_node& nd = out->nodes[base_here + pi];
      if (nd.mask == 0) nd.child = static_cast<int32_t>(base_kids + static_cast<int64_t>(q));
      nd.mask |= 1u << (kid[q] & 7);
    }
  }
  out->leaf_ijk_sorted.resize(static_cast<size_t>(n) * 3);
  for (int64_t q = 0; q < n; ++q) {
    const uint64_t code = leaf[q].first;
    out->leaf_ijk_sorted[3 * q] = static_cast<int32_t>(compact3(code));
    out->leaf_ijk_sorted[3 * q + 1] = static_cast<int32_t>(compact3(code >> 1));
    out->leaf_ijk_sorted[3 * q + 2] = static_cast<int32_t>(compact3(code >> 2));
  }
  return SVLF_OK;
}

}  // namespace svlf
