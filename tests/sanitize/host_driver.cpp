// Exercises the host-only entry points of libgsw (graph validation, degree
// and graph features, tree creation, JSON loading and prediction, names and
// error strings) in a build whose host code carries AddressSanitizer and
// UndefinedBehaviorSanitizer.  Needs no GPU: entry points that need one are
// called only to check that they fail cleanly without a device.
//
//   host_driver <tree.json> [<tree.json> ...]
//
// Prints "ok" and exits 0 when every check holds; the sanitizers abort the
// process on the first memory or undefined-behaviour error.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "gsw.h"

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(1);                                                     \
    }                                                                   \
  } while (0)

namespace {

struct Csr {
  int64_t n = 0;
  std::vector<int64_t> offs;
  std::vector<int32_t> cols;
};

// Random graph of n vertices; symmetric when asked (rows sorted, no repeats).
Csr random_graph(int64_t n, int64_t m, bool symmetric, uint32_t seed) {
  std::mt19937_64 rng(seed);
  std::vector<std::vector<int32_t>> adj(n);
  for (int64_t i = 0; i < m; ++i) {
    int32_t u = (int32_t)(rng() % n), v = (int32_t)(rng() % n);
    if (u == v) continue;
    adj[u].push_back(v);
    if (symmetric) adj[v].push_back(u);
  }
  Csr g;
  g.n = n;
  g.offs.assign(n + 1, 0);
  for (int64_t v = 0; v < n; ++v) {
    auto& r = adj[v];
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
    g.offs[v + 1] = g.offs[v] + (int64_t)r.size();
    g.cols.insert(g.cols.end(), r.begin(), r.end());
  }
  return g;
}

void check_graph_entry_points() {
  for (uint32_t seed = 0; seed < 40; ++seed) {
    const bool sym = seed % 2 == 0;
    const int64_t n = 1 + seed * 7;
    Csr g = random_graph(n, 3 * n, sym, seed);
    int32_t is_sym = -1;
    CHECK(gsw_graph_validate(g.n, (int64_t)g.cols.size(), g.offs.data(), g.cols.data(), &is_sym) == GSW_OK);
    if (sym) CHECK(is_sym == 1);
    double ds[6], gf[GSW_N_GRAPH_FEATURES];
    CHECK(gsw_degree_stats(g.n, g.offs.data(), ds) == GSW_OK);
    CHECK(gsw_graph_features_host(g.n, (int64_t)g.cols.size(), g.offs.data(), g.cols.data(), gf) == GSW_OK);
    CHECK(gf[0] == (double)g.n && gf[1] == (double)g.cols.size());
    for (int i = 0; i < 6; ++i) CHECK(gf[2 + i] == ds[i]);  // out-degree statistics
    if (sym)
      for (int i = 0; i < 6; ++i) CHECK(gf[8 + i] == ds[i] && gf[14 + i] == ds[i]);
  }
  // Malformed graphs: every one is an error, none reads out of bounds.
  Csr g = random_graph(50, 200, true, 99);
  const int64_t nnz = (int64_t)g.cols.size();
  std::vector<int32_t> bad = g.cols;
  bad[nnz / 2] = 50;
  int32_t s = 0;
  CHECK(gsw_graph_validate(g.n, nnz, g.offs.data(), bad.data(), &s) != GSW_OK);
  bad[nnz / 2] = -1;
  CHECK(gsw_graph_validate(g.n, nnz, g.offs.data(), bad.data(), &s) != GSW_OK);
  std::vector<int64_t> boffs = g.offs;
  boffs[10] = boffs[11] + 1;
  CHECK(gsw_graph_validate(g.n, nnz, boffs.data(), g.cols.data(), &s) != GSW_OK);
  boffs = g.offs;
  boffs[g.n] = nnz + 1;
  CHECK(gsw_graph_validate(g.n, nnz, boffs.data(), g.cols.data(), &s) != GSW_OK);
  CHECK(gsw_graph_validate(-1, nnz, g.offs.data(), g.cols.data(), &s) != GSW_OK);
  CHECK(gsw_graph_validate(g.n, nnz, nullptr, g.cols.data(), &s) != GSW_OK);
  CHECK(std::strlen(gsw_last_error()) > 0);
  // Without a device, creating a graph is an error, not a crash.
  gsw_graph* dg = nullptr;
  CHECK(gsw_graph_create_host(g.n, nnz, g.offs.data(), g.cols.data(), 0, &dg) != GSW_OK);
  CHECK(dg == nullptr);
  gsw_graph_destroy(nullptr);
}

void check_tree_entry_points(const std::vector<std::string>& paths) {
  // A handmade tree: root splits on feature 20, left leaf tied (unknown).
  const int32_t feature[3] = {20, -2, -2};
  const double threshold[3] = {10.5, -2.0, -2.0};
  const int32_t left[3] = {1, -1, -1}, right[3] = {2, -1, -1};
  const double value[3 * 2] = {3, 3, 1, 1, 2, 2 + 1};
  const int32_t class_kernel[2] = {GSW_K_PULL_BITMAP, GSW_KERNEL_ID(GSW_K_PUSH_EDGE, GSW_COUNT_THREAD)};
  gsw_tree* t = nullptr;
  CHECK(gsw_tree_create(3, 2, feature, threshold, left, right, value, class_kernel, &t) == GSW_OK);
  double x[GSW_N_FEATURES] = {0};
  int32_t k = -1, unk = -1;
  x[20] = 5;
  CHECK(gsw_tree_predict(t, x, GSW_K_PUSH_VERTEX, 3, &k, &unk) == GSW_OK);
  CHECK(unk == 1 && k == GSW_K_PUSH_VERTEX);
  x[20] = 11;
  CHECK(gsw_tree_predict(t, x, GSW_K_PUSH_VERTEX, 3, &k, &unk) == GSW_OK);
  CHECK(unk == 0 && k == class_kernel[1]);
  gsw_tree_destroy(t);
  // A child index out of range is rejected.
  const int32_t bad_left[3] = {3, -1, -1};
  t = nullptr;
  CHECK(gsw_tree_create(3, 2, feature, threshold, bad_left, right, value, class_kernel, &t) != GSW_OK);
  CHECK(t == nullptr);
  // The shipped trees load and predict a kernel id in range.
  for (const auto& p : paths) {
    t = nullptr;
    CHECK(gsw_tree_load(p.c_str(), &t) == GSW_OK);
    std::mt19937_64 rng(7);
    for (int i = 0; i < 2000; ++i) {
      for (double& v : x) v = (double)(rng() % 100000) / 7.0;
      CHECK(gsw_tree_predict(t, x, -1, i % 5, &k, &unk) == GSW_OK);
      CHECK(k >= 0 && k < GSW_N_KERNELS);
    }
    gsw_tree_destroy(t);
  }
  // Malformed files: truncated at every length of a small valid document,
  // plus a deep nesting and wrong types.
  const std::string good =
      "{\"feature\":[0,-2,-2],\"threshold\":[1.5,-2,-2],\"left\":[1,-1,-1],\"right\":[2,-1,-1],"
      "\"value\":[[1,1],[1,0],[0,1]],\"class_kernel\":[0,6]}";
  const char* tmp = std::getenv("GSW_SAN_TMP");
  const std::string path = std::string(tmp ? tmp : "/tmp") + "/gsw_san_tree.json";
  auto load = [&](const std::string& text) {
    FILE* f = std::fopen(path.c_str(), "w");
    CHECK(f != nullptr);
    std::fwrite(text.data(), 1, text.size(), f);
    std::fclose(f);
    gsw_tree* tt = nullptr;
    gsw_status st = gsw_tree_load(path.c_str(), &tt);
    if (st == GSW_OK) gsw_tree_destroy(tt);
    else CHECK(tt == nullptr);
    return st;
  };
  CHECK(load(good) == GSW_OK);
  for (size_t len = 0; len + 1 < good.size(); ++len) CHECK(load(good.substr(0, len)) != GSW_OK);
  CHECK(load(std::string(10000, '[')) != GSW_OK);
  CHECK(load("{\"feature\":\"x\"}") != GSW_OK);
  CHECK(load("{\"feature\":[0.5,-2,-2],\"threshold\":[1,-2,-2],\"left\":[1,-1,-1],\"right\":[2,-1,-1],"
             "\"value\":[[1,1],[1,0],[0,1]],\"class_kernel\":[0,6]}") != GSW_OK);
  CHECK(load("{\"feature\":[0,-2,-2],\"threshold\":[1,-2,-2],\"left\":[1,-1,-1],\"right\":[2,-1,-1],"
             "\"value\":[[1,1],[1,0],[0,1]],\"class_kernel\":[0,99]}") != GSW_OK);
  std::remove(path.c_str());
  CHECK(gsw_tree_load("/nonexistent/tree.json", &t) != GSW_OK);
}

void check_names() {
  CHECK(gsw_abi_version() == GSW_ABI_VERSION);
  for (int i = 0; i < GSW_N_KERNELS; ++i) CHECK(gsw_kernel_name(i) && std::strlen(gsw_kernel_name(i)) > 0);
  for (int i = 0; i < GSW_N_FEATURES; ++i) CHECK(gsw_feature_name(i) && std::strlen(gsw_feature_name(i)) > 0);
  gsw_bfs_opts o;
  gsw_bfs_opts_default(&o);
  gsw_msbfs_opts mo;
  gsw_msbfs_opts_default(&mo);
}

}  // namespace

int main(int argc, char** argv) {
  std::vector<std::string> paths(argv + 1, argv + argc);
  check_names();
  check_graph_entry_points();
  check_tree_entry_points(paths);
  std::printf("ok\n");
  return 0;
}
