// CPU check of the tile assembly tables that the host set-up (paper_2506_09435_amd/csrc/setup.cpp)
// builds for the owner-computes apply and geometry: representatives, LDS exchange entries, tile
// face slots and the geometry's face layout.  Reads one mesh from a directory written by
// tests/test_face_layout.py and prints "ok" when every check holds.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <random>
#include <string>
#include <vector>

#include "fnpf_internal.h"

namespace fnpf {
std::string build_host_mesh(const fnpf_mesh_desc &m, Ctx &c, std::vector<double> &hm, std::vector<uint8_t> &flags,
                            std::vector<int32_t> &cols, std::vector<double> &mlump_w, std::vector<double> &mlump_s);
}
using namespace fnpf;

static int fails = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      if (fails < 20) std::printf("FAILED line %d: %s\n", __LINE__, #c); \
      ++fails;                                                    \
    }                                                             \
  } while (0)

template <typename T>
static std::vector<T> read_all(const std::string &path) {
  std::ifstream f(path, std::ios::binary | std::ios::ate);
  std::vector<T> v;
  if (!f) return v;
  const std::streamsize n = f.tellg();
  f.seekg(0);
  v.resize((size_t)n / sizeof(T));
  f.read(reinterpret_cast<char *>(v.data()), n);
  return v;
}

int main(int argc, char **argv) {
  if (argc != 2) return 2;
  const std::string dir = argv[1];
  std::ifstream meta(dir + "/meta.txt");
  long long dim, p, nz, n_eh, n_s;
  meta >> dim >> p >> nz >> n_eh >> n_s;
  const auto nodes = read_all<int32_t>(dir + "/nodes.bin");
  const auto corner = read_all<double>(dir + "/corner.bin");
  const auto arc = read_all<double>(dir + "/arc.bin");
  const auto tag = read_all<int32_t>(dir + "/tag.bin");
  const auto layer = read_all<double>(dir + "/layer.bin");
  fnpf_mesh_desc d{(int32_t)dim, (int32_t)p, (int32_t)nz, (int32_t)n_eh, (int64_t)n_s, nodes.data(), corner.data(),
                   arc.empty() ? nullptr : arc.data(), tag.data(), layer.empty() ? nullptr : layer.data(), 9.81};
  Ctx c;
  std::vector<double> hm, mw, ms;
  std::vector<uint8_t> flags;
  std::vector<int32_t> cols;
  const std::string err = build_host_mesh(d, c, hm, flags, cols, mw, ms);
  if (!err.empty()) {
    std::printf("set-up failed: %s\n", err.c_str());
    return 1;
  }
  if (dim != 3) {
    std::printf("ok\n");
    return 0;
  }
  const int nh = c.nh, tc = c.tile_cols;
  const int64_t ncn = n_eh * nh;
  // owner column of each node: the lowest-numbered column that has it
  std::vector<int64_t> owner(n_s, n_eh);
  for (int64_t o = 0; o < ncn; ++o) owner[nodes[o]] = std::min<int64_t>(owner[nodes[o]], o / nh);

  // (1) per tile and node: exactly one representative, the tile's first column with the node; it
  // is tile-owned exactly when the node's owner column lies in the tile
  std::vector<int64_t> rep(n_s, -1);
  for (int64_t t0 = 0; t0 < n_eh; t0 += tc) {
    const int64_t t1 = std::min<int64_t>(t0 + tc, n_eh);
    for (int64_t o = t0 * nh; o < t1 * nh; ++o) rep[nodes[o]] = -1;
    for (int64_t o = t0 * nh; o < t1 * nh; ++o) {
      const int32_t id = nodes[o];
      if (rep[id] < 0) {
        rep[id] = o;
        CHECK((flags[o] & kTRep) != 0);
        CHECK(((flags[o] & kTOwn) != 0) == (owner[id] >= t0 && owner[id] < t1));
      } else {
        CHECK((flags[o] & kTRep) == 0);
      }
    }
    // (2) exchange entries: each partner's entry is read by its representative, entries are
    // distinct within the tile and below the tile's capacity; a column node is a representative,
    // an exchange partner or the writer of a face slot of its own
    std::vector<int> used(c.tile_xmax, 0);
    for (int64_t o = t0 * nh; o < t1 * nh; ++o) {
      const int xw = c.h_xch[o * 4];
      const bool is_rep = (flags[o] & kTRep) != 0;
      CHECK((int)is_rep + (int)(xw >= 0) + (int)(!is_rep && c.h_tslot[o] >= 0) == 1);
      if (xw < 0) continue;
      CHECK(xw < c.tile_xmax);
      if (xw >= c.tile_xmax) continue;
      ++used[xw];
      const int64_t r = rep[nodes[o]];
      CHECK(c.h_xch[r * 4 + 1] == xw || c.h_xch[r * 4 + 2] == xw || c.h_xch[r * 4 + 3] == xw);
    }
    for (int e : used) CHECK(e <= 1);
    for (int64_t o = t0 * nh; o < t1 * nh; ++o)
      for (int a = 1; a < 4; ++a) {
        const int xr = c.h_xch[o * 4 + a];
        if (xr >= 0 && xr < c.tile_xmax) CHECK(used[xr] == 1);
      }
  }
  // (3) tile face slots: each written by one column node; a node's slot list holds exactly its
  // slots, in increasing order; the representatives of nodes with slots are marked shared
  std::vector<int> written(c.n_tslots, 0);
  std::vector<std::vector<int32_t>> slots_of(n_s);
  for (int64_t o = 0; o < ncn; ++o)
    if (c.h_tslot[o] >= 0) {
      CHECK(c.h_tslot[o] < c.n_tslots);
      if (c.h_tslot[o] >= c.n_tslots) continue;
      ++written[c.h_tslot[o]];
      slots_of[nodes[o]].push_back(c.h_tslot[o]);
    }
  for (int w : written) CHECK(w == 1);
  CHECK((int64_t)c.h_tps_node.size() == c.n_tps);
  int64_t with_slots = 0;
  for (int64_t n = 0; n < n_s; ++n) with_slots += !slots_of[n].empty();
  CHECK(with_slots == c.n_tps);
  for (int64_t k = 0; k < c.n_tps; ++k) {
    const int32_t n = c.h_tps_node[k];
    if (k > 0) CHECK(c.h_tps_node[k - 1] < n);
    std::vector<int32_t> mine = slots_of[n];
    std::sort(mine.begin(), mine.end());
    std::vector<int32_t> listed(c.h_tps_slot.begin() + c.h_tps_ptr[k], c.h_tps_slot.begin() + c.h_tps_ptr[k + 1]);
    CHECK(listed == mine);
  }
  for (int64_t o = 0; o < ncn; ++o)
    if ((flags[o] & kTOwn) != 0) CHECK(((flags[o] & kTShared) != 0) == !slots_of[nodes[o]].empty());
  // (4) the geometry's face layout: every place of a level row written by one column node; the
  // sum over a node's places, in the order the face pass takes them, equals the owner tile's value
  // plus its slots in increasing slot order, bit for bit
  std::vector<int> gw(c.n_gslots, 0);
  for (int64_t o = 0; o < ncn; ++o)
    if (c.h_gslot[o] >= 0) {
      CHECK(c.h_gslot[o] < c.n_gslots);
      if (c.h_gslot[o] < c.n_gslots) ++gw[c.h_gslot[o]];
    }
  for (int w : gw) CHECK(w == 1);
  std::mt19937_64 rng(11);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  std::vector<double> val(ncn), F(c.n_tslots, 0.0), G(c.n_gslots, 0.0), own(n_s, 0.0);
  for (auto &v : val) v = U(rng);
  for (int64_t o = 0; o < ncn; ++o) {
    if (c.h_tslot[o] >= 0 && c.h_tslot[o] < c.n_tslots) F[c.h_tslot[o]] = val[o];
    if ((flags[o] & kTOwn) && (flags[o] & kTShared)) own[nodes[o]] = val[o];
    if (c.h_gslot[o] >= 0 && c.h_gslot[o] < c.n_gslots) G[c.h_gslot[o]] = val[o];
  }
  for (int64_t k = 0; k < c.n_tps; ++k) {
    double a = own[c.h_tps_node[k]];
    for (int q = c.h_tps_ptr[k]; q < c.h_tps_ptr[k + 1]; ++q) a += F[c.h_tps_slot[q]];
    double b = G[k];
    b += G[c.n_tps + k];
    for (int q = c.h_gx_ptr[k]; q < c.h_gx_ptr[k + 1]; ++q) b += G[c.h_gx_slot[q]];
    CHECK(a == b);
  }
  if (fails) {
    std::printf("%d checks failed\n", fails);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
