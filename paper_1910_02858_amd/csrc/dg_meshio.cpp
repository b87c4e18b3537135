// Element-package mesh files and exact connectivity from global node indices.
//
// Sec. 2.1.1 (mesh format): the mesh file stores, per element, one package with the element's
// side connectivity (conforming and non-conforming) and its node information (global node index
// and position), so that any contiguous range of elements is one contiguous part of the file and
// can be read on its own; the coordinates of a physical node are stored with every element that
// has it and are tied together by the global index.  The layout here is this project's own
// (little-endian binary, no HDF5 in this environment):
//   header (64 bytes): magic "DGSEMMSH", int32 version = 1, int32 n_geo, int64 K, int32 flags
//                      (bit 0: side records carry mortar kinds), zero padding;
//   package of element e at offset 64 + e * P, P = n^3 * 32 + 6 * 8 bytes (n = n_geo + 1):
//     int64 node index [n^3], float64 coordinates [3][n^3] (node i + n (j + n k)),
//     6 side records {int32 neighbour element (-1: none), int8 neighbour side or boundary kind,
//                     int8 orientation code, int8 mortar kind, int8 0}.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <vector>

#include "../../include/dgsem.h"

namespace {

constexpr char kMagic[8] = {'D', 'G', 'S', 'E', 'M', 'M', 'S', 'H'};
constexpr int kHeader = 64;

size_t package_bytes(int ngeo) {
  const size_t n = (size_t)ngeo + 1;
  return n * n * n * 32 + 6 * 8;
}

struct File {
  std::FILE *f = nullptr;
  explicit File(const char *path, const char *mode) { f = std::fopen(path, mode); }
  ~File() {
    if (f) std::fclose(f);
  }
};

int read_header(std::FILE *f, int *ngeo, int64_t *K, int *flags) {
  unsigned char h[kHeader];
  if (std::fread(h, 1, kHeader, f) != (size_t)kHeader) return DG_ERR_ARG;
  if (std::memcmp(h, kMagic, 8) != 0) return DG_ERR_ARG;
  int32_t version, ng, fl;
  int64_t k;
  std::memcpy(&version, h + 8, 4);
  std::memcpy(&ng, h + 12, 4);
  std::memcpy(&k, h + 16, 8);
  std::memcpy(&fl, h + 24, 4);
  if (version != 1 || ng < 1 || ng > 16 || k < 1) return DG_ERR_ARG;
  *ngeo = ng;
  *K = k;
  *flags = fl;
  return DG_OK;
}

// the face point (a,b) of side s of a tensor element with n nodes per direction: node index
inline int face_node(int n, int s, int a, int b) {
  const int d = s >> 1, m = (s & 1) ? n - 1 : 0;
  return d == 0 ? m + n * (a + n * b) : (d == 1 ? a + n * (m + n * b) : a + n * (b + n * m));
}

}  // namespace

extern "C" {

int dg_mesh_file_write(const char *path, int n_elems, int n_geo, const double *xgeo, const int64_t *node_id,
                       const int32_t *nbr_elem, const int8_t *nbr_side, const int8_t *flip, const int8_t *mortar) {
  if (!path || n_elems < 1 || n_geo < 1 || n_geo > 16 || !xgeo || !node_id || !nbr_elem || !nbr_side)
    return DG_ERR_ARG;
  File fh(path, "wb");
  if (!fh.f) return DG_ERR_ARG;
  unsigned char h[kHeader] = {};
  std::memcpy(h, kMagic, 8);
  const int32_t version = 1, ng = n_geo, fl = mortar ? 1 : 0;
  const int64_t K = n_elems;
  std::memcpy(h + 8, &version, 4);
  std::memcpy(h + 12, &ng, 4);
  std::memcpy(h + 16, &K, 8);
  std::memcpy(h + 24, &fl, 4);
  if (std::fwrite(h, 1, kHeader, fh.f) != (size_t)kHeader) return DG_ERR_ARG;
  const size_t n3 = (size_t)(n_geo + 1) * (n_geo + 1) * (n_geo + 1);
  std::vector<unsigned char> pkg(package_bytes(n_geo));
  for (int64_t e = 0; e < K; ++e) {
    unsigned char *p = pkg.data();
    std::memcpy(p, node_id + e * n3, n3 * 8);
    p += n3 * 8;
    std::memcpy(p, xgeo + e * 3 * n3, 3 * n3 * 8);
    p += 3 * n3 * 8;
    for (int s = 0; s < 6; ++s) {
      const int32_t nb = nbr_elem[e * 6 + s];
      std::memcpy(p, &nb, 4);
      p[4] = (unsigned char)nbr_side[e * 6 + s];
      p[5] = (unsigned char)(flip ? flip[e * 6 + s] : 0);
      p[6] = (unsigned char)(mortar ? mortar[e * 6 + s] : 0);
      p[7] = 0;
      p += 8;
    }
    if (std::fwrite(pkg.data(), 1, pkg.size(), fh.f) != pkg.size()) return DG_ERR_ARG;
  }
  return DG_OK;
}

int dg_mesh_file_info(const char *path, int64_t out[3]) {
  if (!path || !out) return DG_ERR_ARG;
  File fh(path, "rb");
  if (!fh.f) return DG_ERR_ARG;
  int ngeo, flags;
  int64_t K;
  if (int rc = read_header(fh.f, &ngeo, &K, &flags)) return rc;
  out[0] = K;
  out[1] = ngeo;
  out[2] = flags;
  return DG_OK;
}

int dg_mesh_file_read(const char *path, int64_t first, int count, double *xgeo, int64_t *node_id, int32_t *nbr_elem,
                      int8_t *nbr_side, int8_t *flip, int8_t *mortar) {
  if (!path || first < 0 || count < 1) return DG_ERR_ARG;
  File fh(path, "rb");
  if (!fh.f) return DG_ERR_ARG;
  int ngeo, flags;
  int64_t K;
  if (int rc = read_header(fh.f, &ngeo, &K, &flags)) return rc;
  if (first + count > K) return DG_ERR_ARG;
  const size_t P = package_bytes(ngeo), n3 = (size_t)(ngeo + 1) * (ngeo + 1) * (ngeo + 1);
  if (std::fseek(fh.f, (long)(kHeader + first * (int64_t)P), SEEK_SET) != 0) return DG_ERR_ARG;
  // the range is one contiguous part of the file
  std::vector<unsigned char> buf(P * (size_t)count);
  if (std::fread(buf.data(), 1, buf.size(), fh.f) != buf.size()) return DG_ERR_ARG;
  for (int i = 0; i < count; ++i) {
    const unsigned char *p = buf.data() + P * i;
    if (node_id) std::memcpy(node_id + (size_t)i * n3, p, n3 * 8);
    p += n3 * 8;
    if (xgeo) std::memcpy(xgeo + (size_t)i * 3 * n3, p, 3 * n3 * 8);
    p += 3 * n3 * 8;
    for (int s = 0; s < 6; ++s) {
      int32_t nb;
      std::memcpy(&nb, p, 4);
      if (nbr_elem) nbr_elem[i * 6 + s] = nb;
      if (nbr_side) nbr_side[i * 6 + s] = (int8_t)p[4];
      if (flip) flip[i * 6 + s] = (int8_t)p[5];
      if (mortar) mortar[i * 6 + s] = (flags & 1) ? (int8_t)p[6] : 0;
      p += 8;
    }
  }
  return DG_OK;
}

int dg_mesh_connect_nodes(int n_elems, int n_geo, const int64_t *node_id, int bc_kind, int32_t *nbr_elem,
                          int8_t *nbr_side, int8_t *flip) {
  if (n_elems < 1 || n_geo < 1 || n_geo > 16 || !node_id || !nbr_elem || !nbr_side || !flip) return DG_ERR_ARG;
  if (bc_kind < DG_BC_SYMMETRY || bc_kind > DG_BC_OUTFLOW) return DG_ERR_ARG;
  const int n = n_geo + 1, N = n_geo, n3 = n * n * n;
  const int K = n_elems;
  // face corners in face-point order (0,0), (N,0), (0,N), (N,N); a face is keyed by its sorted
  // corner indices
  auto corners = [&](int e, int s, int64_t c[4]) {
    const int ab[4][2] = {{0, 0}, {N, 0}, {0, N}, {N, N}};
    for (int q = 0; q < 4; ++q) c[q] = node_id[(size_t)e * n3 + face_node(n, s, ab[q][0], ab[q][1])];
  };
  std::map<std::vector<int64_t>, std::vector<int>> faces;
  for (int e = 0; e < K; ++e)
    for (int s = 0; s < 6; ++s) {
      int64_t c[4];
      corners(e, s, c);
      std::vector<int64_t> key(c, c + 4);
      std::sort(key.begin(), key.end());
      faces[key].push_back(e * 6 + s);
    }
  for (int q = 0; q < 6 * K; ++q) { nbr_elem[q] = -1; nbr_side[q] = (int8_t)bc_kind; flip[q] = 0; }
  for (auto &kv : faces) {
    const std::vector<int> &sides = kv.second;
    if (sides.size() == 1) continue;
    if (sides.size() != 2) return DG_ERR_MESH;  // a face shared by more than two sides
    for (int t = 0; t < 2; ++t) {
      const int q = sides[t], r = sides[1 - t];
      const int e = q / 6, s = q % 6, e2 = r / 6, s2 = r % 6;
      int64_t c[4], c2[4];
      corners(e, s, c);
      corners(e2, s2, c2);
      // orientation code: swap if o & 4, then reverse the first index if o & 1, the second if o & 2
      int found = -1;
      for (int o = 0; o < 8 && found < 0; ++o) {
        bool ok = true;
        const int ab[4][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};
        for (int k = 0; k < 4 && ok; ++k) {
          const int a = ab[k][0], b = ab[k][1];
          const int p = (o & 4) ? b : a, qq = (o & 4) ? a : b;
          const int a2 = (o & 1) ? 1 - p : p, b2 = (o & 2) ? 1 - qq : qq;
          ok = c[k] == c2[a2 + 2 * b2];
        }
        if (ok) found = o;
      }
      if (found < 0) return DG_ERR_MESH;
      nbr_elem[q] = e2;
      nbr_side[q] = (int8_t)s2;
      flip[q] = (int8_t)found;
    }
  }
  return DG_OK;
}

}  // extern "C"
