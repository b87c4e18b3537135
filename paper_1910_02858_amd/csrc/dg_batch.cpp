// Host side of batched ensembles: many independent meshes (different element counts, degrees
// and viscosities, one shared scheme) advanced together.  A stage launches, per degree present,
// one lifting kernel and one split-form operator kernel over the concatenated element lists
// of all members of that degree; members are looked up on the device from a table of
// descriptors.  Full RK steps can be captured once into a HIP graph and replayed.  The
// number of elements per workgroup of each kernel and degree is chosen by timing the
// candidates on the caller's data (dg_batch_tune).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dg_internal.h"

namespace {

constexpr int kMaxTables = 64;  // cached descriptor tables (distinct stage configurations)
constexpr int kMaxGraphs = 16;  // cached step graphs

struct Group {
  int N = 0;
  std::vector<int> idx;  // member indices (caller order) of this degree
  int total = 0;         // elements
  int offset = 0;        // first descriptor of the group in every table
  int *d_first = nullptr;
  int epb_lift = 1, epb_main = 1;
};

struct Table {
  uint64_t key = 0;
  std::vector<dg::Member> host;
  dg::Member *dev = nullptr;
};

struct Graph {
  uint64_t key = 0;
  hipGraphExec_t exec = nullptr;
};

uint64_t fnv1a(const void *p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char *c = (const unsigned char *)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

}  // namespace

struct dg_batch {
  std::vector<dg_handle *> mem;
  std::vector<Group> groups;
  std::vector<Table> tables;  // most recently used last
  std::vector<Graph> graphs;
  hipStream_t cap = nullptr;  // private stream for graph capture and replay
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // one branch per degree group inside the step graph (the groups share no data), forked from
  // and joined to the capture stream with events
  std::vector<hipStream_t> br;
  std::vector<hipEvent_t> br_ev;
  hipEvent_t fork_ev = nullptr;
  bool ns = false;
  int vf = 0;
  int fused = 0;  // 1: one lifting and one operator launch per stage for all degrees
  std::string err;

  hipStream_t stream() const { return mem[0]->stream; }
};

namespace {

int bfail(dg_batch *b, int code, const std::string &msg) {
  if (b) b->err = msg;
  return code;
}

int batch_lift(int N, const dg::BatchView &v, int epb, hipStream_t st) {
  switch (N) {
#define DG_CASE(NN) \
  case NN: return dg::launch_batch_lift<NN>(v, epb, st);
    DG_CASE(1) DG_CASE(2) DG_CASE(3) DG_CASE(4) DG_CASE(5) DG_CASE(6) DG_CASE(7) DG_CASE(8)
#undef DG_CASE
    default: return DG_ERR_UNSUPPORTED;
  }
}

int batch_split(int N, const dg::BatchView &v, bool ns, int vf, int epb, hipStream_t st) {
  switch (N) {
#define DG_CASE(NN) \
  case NN: return dg::launch_batch_split<NN>(v, ns, vf, epb, st);
    DG_CASE(1) DG_CASE(2) DG_CASE(3) DG_CASE(4) DG_CASE(5) DG_CASE(6) DG_CASE(7) DG_CASE(8)
#undef DG_CASE
    default: return DG_ERR_UNSUPPORTED;
  }
}

dg::BatchView view(const dg_batch *b, const Group &g, const dg::Member *table) {
  dg::BatchView v;
  v.m = table + g.offset;
  v.first = g.d_first;
  v.count = (int)g.idx.size();
  v.total = g.total;
  v.tab = b->mem[g.idx[0]]->d_tab;
  v.general = 0;
  for (int i : g.idx)
    if (b->mem[i]->d_fc) v.general = 1;
  return v;
}

// descriptors of one stage, in group order
std::vector<dg::Member> describe(const dg_batch *b, const double *const *U_in, double *const *U_out,
                                 double *const *R, const double *a, const double *bc, const double *dt) {
  std::vector<dg::Member> m;
  m.reserve(b->mem.size());
  for (const Group &g : b->groups)
    for (int i : g.idx) {
      const dg_handle *h = b->mem[i];
      // field by field into zeroed storage, so padding bytes are defined for the content hash
      dg::Member d;
      std::memset(&d, 0, sizeof(d));
      d.g.Ja = h->d_Ja; d.g.sJ = h->d_sJ; d.g.fn = h->d_fn; d.g.nbr = h->d_nbr; d.g.fc = h->d_fc; d.g.tab = h->d_tab; d.g.K = h->K;
      d.g.Gd = h->d_Gd; d.g.Gf = h->d_Gf;
      d.ph.gamma = h->ph.gamma; d.ph.R = h->ph.R; d.ph.mu = h->ph.mu; d.ph.Pr = h->ph.Pr;
      d.ph.kappa = h->ph.kappa; d.ph.vf = h->ph.vf; d.ph.rs = h->ph.rs;
      for (int v = 0; v < 5; ++v) d.ph.ub[v] = h->ph.ub[v];
      d.ph.tw = h->ph.tw;
      d.ph.pout = h->ph.pout;
      d.U = U_in[i];
      d.G = h->d_G;
      d.out = U_out[i];
      d.R = R[i];
      d.a = a[i];
      d.b = bc[i];
      d.dt = dt[i];
      m.push_back(d);
    }
  return m;
}

// device copy of a descriptor table, created on first use and cached by content
int table_for(dg_batch *b, const std::vector<dg::Member> &m, const dg::Member **dev) {
  const uint64_t key = fnv1a(m.data(), m.size() * sizeof(dg::Member));
  for (size_t i = 0; i < b->tables.size(); ++i) {
    Table &t = b->tables[i];
    if (t.key == key && t.host.size() == m.size() &&
        std::memcmp(t.host.data(), m.data(), m.size() * sizeof(dg::Member)) == 0) {
      *dev = t.dev;
      if (i + 1 != b->tables.size()) std::rotate(b->tables.begin() + i, b->tables.begin() + i + 1, b->tables.end());
      return DG_OK;
    }
  }
  if ((int)b->tables.size() >= kMaxTables) {
    // the oldest table may still be read by queued kernels
    if (hipStreamSynchronize(b->stream()) != hipSuccess) return bfail(b, DG_ERR_HIP, "stream synchronisation failed");
    (void)hipFree(b->tables.front().dev);
    b->tables.erase(b->tables.begin());
  }
  Table t;
  t.key = key;
  t.host = m;
  if (hipMalloc((void **)&t.dev, m.size() * sizeof(dg::Member)) != hipSuccess) {
    (void)hipGetLastError();
    return bfail(b, DG_ERR_OOM, "allocation of a member table failed");
  }
  if (hipMemcpy(t.dev, m.data(), m.size() * sizeof(dg::Member), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(t.dev);
    return bfail(b, DG_ERR_HIP, "upload of a member table failed");
  }
  *dev = t.dev;
  b->tables.push_back(std::move(t));
  return DG_OK;
}

// whether one launch can cover every degree: degrees up to 7, structured meshes, few degrees
bool fusable(const dg_batch *b) {
  if ((int)b->groups.size() > dg::FUSED_MAXG) return false;
  for (const Group &g : b->groups) {
    if (dg::fused_epb(g.N, false) < 1) return false;
    for (int i : g.idx)
      if (b->mem[i]->d_fc) return false;
  }
  return true;
}

int launch_stage_fused(dg_batch *b, const dg::Member *table, hipStream_t st) {
  dg::FusedView fl, fs;
  std::memset(&fl, 0, sizeof(fl));
  std::memset(&fs, 0, sizeof(fs));
  fl.ng = fs.ng = (int)b->groups.size();
  for (int gi = 0; gi < fl.ng; ++gi) {
    const Group &g = b->groups[gi];
    fl.v[gi] = fs.v[gi] = view(b, g, table);
    fl.N[gi] = fs.N[gi] = g.N;
    const int el = dg::fused_epb(g.N, true), es = dg::fused_epb(g.N, false);
    fl.start[gi + 1] = fl.start[gi] + (g.total + el - 1) / el;
    fs.start[gi + 1] = fs.start[gi] + (g.total + es - 1) / es;
  }
  if (b->ns) {
    const int rc = dg::launch_fused_lift(fl, st);
    if (rc) return bfail(b, rc, "launch of the fused lifting kernel failed");
  }
  const int rc = dg::launch_fused_split(fs, b->ns, b->vf, st);
  if (rc) return bfail(b, rc, "launch of the fused operator kernel failed");
  return DG_OK;
}

int launch_group_stage(dg_batch *b, const Group &g, const dg::Member *table, hipStream_t st) {
  const dg::BatchView v = view(b, g, table);
  if (b->ns) {
    int rc = batch_lift(g.N, v, g.epb_lift, st);
    if (rc) return bfail(b, rc, "launch of a batched lifting kernel failed");
  }
  int rc = batch_split(g.N, v, b->ns, b->vf, g.epb_main, st);
  if (rc) return bfail(b, rc, "launch of a batched operator kernel failed");
  return DG_OK;
}

int launch_stage(dg_batch *b, const dg::Member *table, hipStream_t st) {
  if (b->fused) return launch_stage_fused(b, table, st);
  for (const Group &g : b->groups) {
    const int rc = launch_group_stage(b, g, table, st);
    if (rc) return rc;
  }
  return DG_OK;
}

#ifndef DG_BATCH_BRANCHES
#define DG_BATCH_BRANCHES 1
#endif
// the five stages of a step into the capture stream: with several degree groups, each group's
// ten launches on its own branch (fork and join through events), so that the graph lets the
// groups' kernels overlap
int capture_step(dg_batch *b, const dg::Member *const *tabs) {
  if (b->fused || b->groups.size() < 2 || !DG_BATCH_BRANCHES) {
    for (int s = 0; s < 5; ++s)
      if (int rc = launch_stage(b, tabs[s], b->cap)) return rc;
    return DG_OK;
  }
  if (hipEventRecord(b->fork_ev, b->cap) != hipSuccess) return bfail(b, DG_ERR_HIP, "graph fork failed");
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    if (hipStreamWaitEvent(b->br[gi], b->fork_ev, 0) != hipSuccess) return bfail(b, DG_ERR_HIP, "graph fork failed");
    for (int s = 0; s < 5; ++s)
      if (int rc = launch_group_stage(b, b->groups[gi], tabs[s], b->br[gi])) return rc;
    if (hipEventRecord(b->br_ev[gi], b->br[gi]) != hipSuccess || hipStreamWaitEvent(b->cap, b->br_ev[gi], 0) != hipSuccess)
      return bfail(b, DG_ERR_HIP, "graph join failed");
  }
  return DG_OK;
}

int check_arrays(dg_batch *b, const double *const *U_in, double *const *U_out, double *const *R) {
  if (!U_in || !U_out || !R) return bfail(b, DG_ERR_ARG, "NULL pointer array");
  for (size_t i = 0; i < b->mem.size(); ++i) {
    const void *p[3] = {U_in[i], U_out[i], R[i]};
    for (const void *q : p)
      if (!q || !aligned8(q)) return bfail(b, DG_ERR_ARG, "member " + std::to_string(i) + ": NULL or misaligned buffer");
    if (p[0] == p[1] || p[0] == p[2] || p[1] == p[2])
      return bfail(b, DG_ERR_ARG, "member " + std::to_string(i) + ": U_in, U_out and R must be distinct");
  }
  return DG_OK;
}

}  // namespace

extern "C" {

int dg_batch_create(dg_handle *const *members, int n_members, dg_batch **out) {
  if (!out) return DG_ERR_ARG;
  *out = nullptr;
  if (!members || n_members < 1) return DG_ERR_ARG;
  for (int i = 0; i < n_members; ++i)
    if (!members[i]) return DG_ERR_ARG;
  const dg_handle *h0 = members[0];
  for (int i = 0; i < n_members; ++i) {
    const dg_handle *h = members[i];
    if (h->node_type != DG_NODES_LGL || h->sc.form != DG_FORM_SPLIT || h->nm || h->fv_on) return DG_ERR_UNSUPPORTED;
    if (h->needs_state && !h->state_set) return DG_ERR_ARG;  // its boundary state is not set
    if (h->needs_tw && !h->tw_set) return DG_ERR_ARG;        // its wall temperature is not set
    if (h->needs_pout && !h->pout_set) return DG_ERR_ARG;    // its outflow pressure is not set
    if (h->sc.eqn != h0->sc.eqn || h->sc.volflux != h0->sc.volflux || h->sc.riemann != h0->sc.riemann)
      return DG_ERR_UNSUPPORTED;
    for (int j = 0; j < i; ++j)
      if (members[j] == h) return DG_ERR_ARG;  // a member's gradient scratch cannot serve twice
  }
  dg_batch *b = new (std::nothrow) dg_batch();
  if (!b) return DG_ERR_OOM;
  b->mem.assign(members, members + n_members);
  b->ns = h0->sc.eqn == DG_NAVIER_STOKES;
  b->vf = h0->sc.volflux;
  int offset = 0;
  for (int N = 1; N <= dg::NMAX; ++N) {
    Group g;
    g.N = N;
    for (int i = 0; i < n_members; ++i)
      if (members[i]->N == N) g.idx.push_back(i);
    if (g.idx.empty()) continue;
    std::vector<int> first(g.idx.size() + 1, 0);
    for (size_t j = 0; j < g.idx.size(); ++j) first[j + 1] = first[j] + members[g.idx[j]]->K;
    g.total = first.back();
    g.offset = offset;
    offset += (int)g.idx.size();
    if (hipMalloc((void **)&g.d_first, first.size() * sizeof(int)) != hipSuccess ||
        hipMemcpy(g.d_first, first.data(), first.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      b->groups.push_back(g);
      dg_batch_destroy(b);
      return DG_ERR_OOM;
    }
    b->groups.push_back(g);
  }
  bool ok = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) == hipSuccess;
  for (size_t gi = 0; ok && gi < b->groups.size(); ++gi) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    if (ok) b->br.push_back(st);
    ok = ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
    if (ok) b->br_ev.push_back(ev);
  }
  if (!ok) {
    (void)hipGetLastError();
    dg_batch_destroy(b);
    return DG_ERR_HIP;
  }
  *out = b;
  return DG_OK;
}

int dg_batch_rk_stage(dg_batch *b, const double *const *U_in, double *const *U_out, double *const *R, const double *a,
                      const double *b_coef, const double *dt) {
  if (!b) return DG_ERR_ARG;
  int rc = check_arrays(b, U_in, U_out, R);
  if (rc) return rc;
  if (!a || !b_coef || !dt) return bfail(b, DG_ERR_ARG, "NULL coefficient array");
  for (size_t i = 0; i < b->mem.size(); ++i)
    if (!std::isfinite(a[i]) || !std::isfinite(b_coef[i]) || !std::isfinite(dt[i]))
      return bfail(b, DG_ERR_ARG, "non-finite coefficient for member " + std::to_string(i));
  const dg::Member *table = nullptr;
  rc = table_for(b, describe(b, U_in, U_out, R, a, b_coef, dt), &table);
  if (rc) return rc;
  return launch_stage(b, table, b->stream());
}

int dg_batch_step(dg_batch *b, double *const *U, double *const *U_out, double *const *R, const double *dt,
                  int use_graph) {
  if (!b) return DG_ERR_ARG;
  int rc = check_arrays(b, U, U_out, R);
  if (rc) return rc;
  if (!dt) return bfail(b, DG_ERR_ARG, "NULL time-step array");
  const size_t n = b->mem.size();
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(dt[i]) || dt[i] <= 0.0) return bfail(b, DG_ERR_ARG, "invalid time step for member " + std::to_string(i));
  double A[5], B[5], C[5];
  dg_rk_coefficients(A, B, C);
  // stage s reads the buffer written by stage s-1: U -> U_out -> U -> U_out -> U -> U_out
  const dg::Member *tabs[5];
  std::vector<double> av(n), bv(n);
  std::vector<const double *> in(n);
  std::vector<double *> outp(n);
  for (int s = 0; s < 5; ++s) {
    for (size_t i = 0; i < n; ++i) {
      av[i] = A[s];
      bv[i] = B[s];
      in[i] = (s % 2 == 0) ? U[i] : U_out[i];
      outp[i] = (s % 2 == 0) ? U_out[i] : U[i];
    }
    rc = table_for(b, describe(b, in.data(), outp.data(), R, av.data(), bv.data(), dt), &tabs[s]);
    if (rc) return rc;
  }
  // five stages leave the result in U_out (stages 1, 3, 5 write it)
  if (!use_graph) {
    for (int s = 0; s < 5; ++s) {
      rc = launch_stage(b, tabs[s], b->stream());
      if (rc) return rc;
    }
    return DG_OK;
  }
  uint64_t key = fnv1a(U, n * sizeof(double *));
  key = fnv1a(U_out, n * sizeof(double *), key);
  key = fnv1a(R, n * sizeof(double *), key);
  key = fnv1a(dt, n * sizeof(double), key);
  key = fnv1a(tabs, sizeof(tabs), key);
  for (const Group &g : b->groups) {
    key = fnv1a(&g.epb_lift, sizeof(int), key);
    key = fnv1a(&g.epb_main, sizeof(int), key);
  }
  key = fnv1a(&b->fused, sizeof(int), key);
  hipGraphExec_t exec = nullptr;
  for (const Graph &gr : b->graphs)
    if (gr.key == key) exec = gr.exec;
  if (!exec) {
    if ((int)b->graphs.size() >= kMaxGraphs) {
      if (hipStreamSynchronize(b->cap) != hipSuccess) return bfail(b, DG_ERR_HIP, "stream synchronisation failed");
      (void)hipGraphExecDestroy(b->graphs.front().exec);
      b->graphs.erase(b->graphs.begin());
    }
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return bfail(b, DG_ERR_HIP, "stream capture could not start");
    const int lrc = capture_step(b, tabs);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->cap, &graph);
    if (lrc) {
      if (graph) (void)hipGraphDestroy(graph);
      return lrc;
    }
    if (ec != hipSuccess || !graph) return bfail(b, DG_ERR_HIP, "stream capture failed");
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return bfail(b, DG_ERR_HIP, "graph instantiation failed");
    b->graphs.push_back({key, exec});
  }
  // order the replay after the caller's queued work and the caller's later work after it
  if (hipEventRecord(b->ev_in, b->stream()) != hipSuccess || hipStreamWaitEvent(b->cap, b->ev_in, 0) != hipSuccess ||
      hipGraphLaunch(exec, b->cap) != hipSuccess || hipEventRecord(b->ev_out, b->cap) != hipSuccess ||
      hipStreamWaitEvent(b->stream(), b->ev_out, 0) != hipSuccess)
    return bfail(b, DG_ERR_HIP, "graph launch failed");
  return DG_OK;
}

int dg_batch_set_tile(dg_batch *b, int N, int epb_lift, int epb_main) {
  if (!b) return DG_ERR_ARG;
  for (Group &g : b->groups)
    if (g.N == N) {
      const int mx = dg::batch_max_epb(N);
      auto ok = [mx](int e) { return (e == 1 || e == 2 || e == 4) && e <= mx; };
      if (!ok(epb_lift) || !ok(epb_main)) return bfail(b, DG_ERR_ARG, "elements per workgroup out of range");
      g.epb_lift = epb_lift;
      g.epb_main = epb_main;
      return DG_OK;
    }
  return bfail(b, DG_ERR_ARG, "no member of this degree");
}

int dg_batch_tune(dg_batch *b, const double *const *U, int repeats) {
  if (!b || !U || repeats < 1) return DG_ERR_ARG;
  const size_t n = b->mem.size();
  for (size_t i = 0; i < n; ++i)
    if (!U[i] || !aligned8(U[i])) return bfail(b, DG_ERR_ARG, "NULL or misaligned state");
  hipStream_t st = b->stream();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    return bfail(b, DG_ERR_HIP, "event creation failed");
  }
  double A[5], B[5], C[5];
  dg_rk_coefficients(A, B, C);
  int rc = DG_OK;
  for (Group &g : b->groups) {
    // scratch stage outputs (the members' states are only read)
    std::vector<double *> outs(n, nullptr), Rs(n, nullptr);
    for (int i : g.idx) {
      const size_t bytes = (size_t)b->mem[i]->K * 5 * b->mem[i]->n3 * sizeof(double);
      if (hipMalloc((void **)&outs[i], bytes) != hipSuccess || hipMalloc((void **)&Rs[i], bytes) != hipSuccess ||
          hipMemsetAsync(Rs[i], 0, bytes, st) != hipSuccess) {
        (void)hipGetLastError();
        rc = bfail(b, DG_ERR_OOM, "allocation of tuning scratch failed");
        break;
      }
    }
    std::vector<dg::Member> m;
    if (!rc) {
      std::vector<double> av(n, A[1]), bv(n, B[1]), dtv(n, 1e-9);
      std::vector<double *> o2(n), r2(n);
      for (size_t i = 0; i < n; ++i) {
        o2[i] = outs[i] ? outs[i] : const_cast<double *>(U[i]);  // other groups are not launched
        r2[i] = Rs[i] ? Rs[i] : const_cast<double *>(U[i]);
      }
      m = describe(b, U, o2.data(), r2.data(), av.data(), bv.data(), dtv.data());
    }
    const dg::Member *table = nullptr;
    if (!rc) rc = table_for(b, m, &table);
    for (int kind = 0; kind < 2 && !rc; ++kind) {
      if (kind == 0 && !b->ns) continue;
      float best = 1e30f;
      int best_epb = 1;
      for (int epb : {1, 2, 4}) {
        if (epb > dg::batch_max_epb(g.N)) continue;
        const dg::BatchView v = view(b, g, table);
        auto go = [&]() {
          return kind == 0 ? batch_lift(g.N, v, epb, st) : batch_split(g.N, v, b->ns, b->vf, epb, st);
        };
        rc = go();  // warm-up
        if (rc) break;
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < repeats && !rc; ++r) rc = go();
        (void)hipEventRecord(e1, st);
        if (rc || hipEventSynchronize(e1) != hipSuccess) {
          rc = rc ? rc : DG_ERR_HIP;
          break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) { best = ms; best_epb = epb; }
      }
      if (!rc) (kind == 0 ? g.epb_lift : g.epb_main) = best_epb;
    }
    if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = bfail(b, DG_ERR_HIP, "stream synchronisation failed");
    for (size_t i = 0; i < n; ++i) {
      if (outs[i]) (void)hipFree(outs[i]);
      if (Rs[i]) (void)hipFree(Rs[i]);
    }
    if (rc) break;
  }
  if (!rc && fusable(b)) {
    // one stage of every member, per-degree launches against the fused pair, the faster kept
    std::vector<double *> outs(n, nullptr), Rs(n, nullptr);
    for (size_t i = 0; i < n && !rc; ++i) {
      const size_t bytes = (size_t)b->mem[i]->K * 5 * b->mem[i]->n3 * sizeof(double);
      if (hipMalloc((void **)&outs[i], bytes) != hipSuccess || hipMalloc((void **)&Rs[i], bytes) != hipSuccess ||
          hipMemsetAsync(Rs[i], 0, bytes, st) != hipSuccess) {
        (void)hipGetLastError();
        rc = bfail(b, DG_ERR_OOM, "allocation of tuning scratch failed");
      }
    }
    const dg::Member *table = nullptr;
    if (!rc) {
      std::vector<double> av(n, A[1]), bv(n, B[1]), dtv(n, 1e-9);
      rc = table_for(b, describe(b, U, outs.data(), Rs.data(), av.data(), bv.data(), dtv.data()), &table);
    }
    float t_mode[2] = {1e30f, 1e30f};
    for (int mode = 0; mode < 2 && !rc; ++mode) {
      b->fused = mode;
      rc = launch_stage(b, table, st);  // warm-up
      (void)hipEventRecord(e0, st);
      for (int r = 0; r < repeats && !rc; ++r) rc = launch_stage(b, table, st);
      (void)hipEventRecord(e1, st);
      if (rc || hipEventSynchronize(e1) != hipSuccess) {
        rc = rc ? rc : DG_ERR_HIP;
        break;
      }
      (void)hipEventElapsedTime(&t_mode[mode], e0, e1);
    }
    b->fused = (!rc && t_mode[1] < t_mode[0]) ? 1 : 0;
    if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = bfail(b, DG_ERR_HIP, "stream synchronisation failed");
    for (size_t i = 0; i < n; ++i) {
      if (outs[i]) (void)hipFree(outs[i]);
      if (Rs[i]) (void)hipFree(Rs[i]);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc && b->err.empty()) b->err = "tuning launch failed";
  return rc;
}

int dg_batch_set_fused(dg_batch *b, int fused) {
  if (!b || (fused != 0 && fused != 1)) return DG_ERR_ARG;
  if (fused && !fusable(b)) return bfail(b, DG_ERR_UNSUPPORTED, "a degree above 7 or a member with face codes");
  b->fused = fused;
  return DG_OK;
}

int dg_batch_fused(const dg_batch *b) { return b ? b->fused : DG_ERR_ARG; }

int dg_batch_info(const dg_batch *b, int *out, int cap) {
  if (!b) return DG_ERR_ARG;
  const int ng = (int)b->groups.size();
  if (out) {
    for (int i = 0; i < ng && 5 * i + 4 < cap; ++i) {
      const Group &g = b->groups[i];
      out[5 * i] = g.N;
      out[5 * i + 1] = (int)g.idx.size();
      out[5 * i + 2] = g.total;
      out[5 * i + 3] = g.epb_lift;
      out[5 * i + 4] = g.epb_main;
    }
  }
  return ng;
}

const char *dg_batch_last_error(const dg_batch *b) { return b ? b->err.c_str() : "no batch"; }

void dg_batch_destroy(dg_batch *b) {
  if (!b) return;
  if (!b->mem.empty()) (void)hipStreamSynchronize(b->stream());
  if (b->cap) (void)hipStreamSynchronize(b->cap);
  for (Graph &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
  for (Table &t : b->tables) (void)hipFree(t.dev);
  for (Group &g : b->groups)
    if (g.d_first) (void)hipFree(g.d_first);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
  for (hipEvent_t ev : b->br_ev) (void)hipEventDestroy(ev);
  for (hipStream_t st : b->br) (void)hipStreamDestroy(st);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

}  // extern "C"
