// C-ABI entry points, planner and workspace management of the ladder library.
//
// A plan is built once per (kind, precision, options, list of symmetry
// shapes) and cached per device.  It holds every device table the kernels
// need (pair maps, K tables, column groups, tile lists) and the launch
// sequence: the (ac|bd) assembly is split into column groups, and groups are
// packed into batches whose intermediate buffer stays under a byte cap, so the
// v^4 tensor is never formed.  Per call only the per-system pointer table is
// uploaded (from pinned host memory, guarded by an event) and the launches are
// enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <dlfcn.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/cdcc.h"
#include "ladder_types.hpp"

namespace cdcc {
hipError_t launch_fill_int(int *p, int n, int v, hipStream_t s);
hipError_t launch_pack(const PackJob *jobs, const int2 *rows, int nrows, const SysPtrs *sp, const int4 *ijtab,
                       const int4 *vvtab, hipStream_t s);
hipError_t launch_dress(const DressJob *jobs, const int2 *rows, int nrows, const SysPtrs *sp, hipStream_t s);
hipError_t launch_assemble_f64(int cls, int grid, const P1Desc *descs, const Tile *tiles, const Queues &Q,
                               int *cnt, const SysPtrs *sp, double *xbuf, hipStream_t s);
hipError_t launch_contract_f64(int grid, const P2Group *groups, const Tile *tiles, const Queues &Q, int *cnt,
                               const SysPtrs *sp, const double *xbuf, const int4 *ktab, const int4 *ijtab,
                               const int4 *vvtab, double *part, hipStream_t s);
hipError_t launch_reduce_unpack(int njobs, const P2Group *groups, const Tile *jobs, const SysPtrs *sp,
                                const double *part, const int4 *ijtab, const int4 *vvtab, hipStream_t s);
int occupancy_f64(int which, int cls);
hipError_t launch_energy(const EnergyJob *jobs, int njobs, const SysPtrs *sp, const int *vvfull, hipStream_t s);
// split paths (kernels_mixed.hip); fmt 0 = BF16 slices, 1 = 8-bit digits
hipError_t launch_slice(int fmt, const SliceJob *jobs, const int2 *rows, int nrows, const SysPtrs *sp,
                        int stage_bytes, hipStream_t s);
hipError_t launch_assemble_mixed(int fmt, int cls, int longk, int neg, int grid, const P1Desc *descs,
                                 const Tile *tiles, const Queues &Q, int *cnt, const SysPtrs *sp, double *xbuf,
                                 hipStream_t s);
int occupancy_mixed(int fmt, int cls);
// vvvv density (kernels_f64.hip, kernels_density.hip)
hipError_t launch_assemble_density(int grid, const P1Desc *descs, const Tile *tiles, const Queues &Q, int *cnt,
                                   const SysPtrs *sp, double *xbuf, hipStream_t s);
int occupancy_density_w();
hipError_t launch_density_pack(const DensPackJob *jobs, const int2 *tiles, int ntiles, const int *swap,
                               const DensPtrs *dp, hipStream_t s);
hipError_t launch_density_gemm(int grid, const GemmDesc *descs, const Tile *tiles, const Queues &Q, int *cnt,
                               const DensPtrs *dp, const double *xbuf, double *part, hipStream_t s);
hipError_t launch_density_reduce(int njobs, const GemmDesc *descs, const Tile *jobs, const DensPtrs *dp,
                                 const double *part, hipStream_t s);
// partial symmetric-antisymmetric contraction (kernels_partial.hip)
hipError_t launch_pm_pack(const PmDesc *descs, const PmChunk *lch, int nl, const PmChunk *tch, int nt,
                          const int2 *kp, const PmSquare *sqs, const PmPtrs *pp, hipStream_t s);
hipError_t launch_pm_gemm(const PmDesc *descs, const int4 *tiles, int ntiles, const PmSquare *sqs,
                          const PmPtrs *pp, hipStream_t s);
// two-step Cholesky decomposition (kernels_cd.hip)
hipError_t launch_cd_diag(const double *V, int64_t n, double *D, hipStream_t s);
hipError_t launch_cd_gather_cols(const double *V, int64_t n, const int32_t *qrows, int nq, double *M, int ldm,
                                 hipStream_t s);
hipError_t launch_cd_micro(const int32_t *qr, const CdQList &QL, const CdPtrs &P, int64_t nmax, int nirrep,
                           CdState *st, double *dq,
                           int qcap, int t0, int steps, hipStream_t s);
hipError_t launch_cd_gemm_nt(const CdGemmBatch &B, hipStream_t s);
hipError_t launch_cd_gather_metric(const double *V, int64_t n, const int32_t *piv, int np, double *K, double *Y,
                                   hipStream_t s);
hipError_t launch_cd_potrf_diag(const CdDiagBatch &D, int *bad, hipStream_t s);

int occupancy_density_gemm();
}  // namespace cdcc

using namespace cdcc;

namespace {

constexpr int64_t kAlign = 256;
inline int64_t align_up(int64_t x, int64_t a = kAlign) { return (x + a - 1) / a * a; }

// P1 (assembly) tile classes.
constexpr int kP1BM[3] = {64, 128, 128};
constexpr int kP1BN[3] = {64, 64, 128};
constexpr int kMixBM[4] = {64, 128, 128, 64};   // mixed path assembly tiles
constexpr int kMixBN[4] = {128, 64, 128, 64};

// Split precisions: slice format (0 BF16, 1 8-bit digits), K block width and
// bytes per sliced element.
inline bool is_split(int precision) { return precision == CDCC_MIXED || precision == CDCC_MIXED_I8; }
inline int split_fmt(int precision) { return precision == CDCC_MIXED_I8 ? 1 : 0; }
inline int split_kblock(int precision) { return precision == CDCC_MIXED_I8 ? 32 : 16; }
inline int split_elem_bytes(int precision) { return precision == CDCC_MIXED_I8 ? 4 : 8; }
// Longest K that the 8-bit kernels accumulate exactly in one pass (1023
// blocks of 32); longer rows go to the kernel with K segments.
constexpr int kI8MaxK = 1023 * 32;
// Contraction tiles: 16 * fm packed (ij) rows x 32 group columns, fm = 1..4
// per group (the kernel switches on it per tile).
constexpr int kP2BN = 32;
inline int contract_fm(int n_ij) {
  if (n_ij <= 64) return std::max(1, (n_ij + 15) / 16);
  // least row padding over 48- and 64-row tiles, ties to 64
  const int p3 = (n_ij + 47) / 48 * 48, p4 = (n_ij + 63) / 64 * 64;
  return p3 < p4 ? 3 : 4;
}

struct Launch {
  int cls = 0, start = 0, count = 0, grid = 0;
  int longk = 0;  // 8-bit split path: some tile has K > kI8MaxK (the K-segment kernel)
  Queues q{};
};
struct BatchPlan {
  std::vector<Launch> p1, p2;
  Launch red;  // split-K reduce + unpack jobs (count 0: none)
};

// Split-K segment of the contraction (default; the tile table or the
// options can set another per shape): fixed per group shape, never per
// batch, so a system's result is the same alone and in any batch.  4096
// entries: at o=40/v=400 the contraction took 8.6 ms per call with 1024,
// 8.1 with 2048 and 8.0 with 4096 to 65536 (the tiles of one launch fill the
// chip without splitting, and the partials cost traffic); at o=20/v=200 the
// lengths measured the same.
constexpr int kKSeg = 4096;

struct SysPlan {
  cdcc_layout_t lay{};
  int64_t th_elems = 0;      // packed +/- amplitudes
  int64_t u_elems = 0;       // Lambda operand stack
  int64_t slice_bytes = 0;   // split paths: sliced operand
  int64_t scale_rows = 0;    // split paths: row scales
  int p1cls = 0;
  int kseg = 0;              // contraction K-segment length (0: the rule)
};

// Completion marker of a plan's last enqueued work: recorded after every
// call that uses the plan, waited for before the plan's device tables and
// graphs are freed, so that evicting a plan never frees memory a queued
// launch still reads.
struct PlanFence {
  hipEvent_t ev = nullptr;
  bool recorded = false;
  void mark(hipStream_t s) {
    if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      ev = nullptr;
      (void)hipStreamSynchronize(s);  // no event: make the work complete now instead
      return;
    }
    recorded = hipEventRecord(ev, s) == hipSuccess;
  }
  void wait() {
    if (ev && recorded) (void)hipEventSynchronize(ev);
    recorded = false;
  }
  ~PlanFence() {
    wait();
    if (ev) (void)hipEventDestroy(ev);
  }
};

// Plans by key, evicting the least recently used one beyond `cap` entries.
template <class P>
struct PlanCache {
  explicit PlanCache(size_t c) : cap(c) {}
  size_t cap;
  uint64_t tick = 0;
  std::map<std::string, std::pair<std::shared_ptr<P>, uint64_t>> m;
  std::shared_ptr<P> find(const std::string &k) {
    auto it = m.find(k);
    if (it == m.end()) return nullptr;
    it->second.second = ++tick;
    return it->second.first;
  }
  void put(const std::string &k, std::shared_ptr<P> p) {
    while (m.size() >= cap) {
      auto lru = m.begin();
      for (auto it = m.begin(); it != m.end(); ++it)
        if (it->second.second < lru->second.second) lru = it;
      m.erase(lru);  // the plan's destructor waits for its fence
    }
    m[k] = {std::move(p), ++tick};
  }
  void clear() { m.clear(); }
  size_t size() const { return m.size(); }
};

struct Plan {
  int nsys = 0;
  int lambda = 0, dressed = 0, precision = 0;
  std::vector<SysPlan> sys;
  // device tables (single allocation)
  void *dtab = nullptr;
  PackJob *packjobs = nullptr;
  int2 *packrows = nullptr;
  int npackrows = 0;
  DressJob *dressjobs = nullptr;
  int2 *dressrows = nullptr;
  int ndressrows = 0;
  P1Desc *p1 = nullptr;
  int np1 = 0;
  Tile *p1tiles = nullptr;
  P2Group *p2 = nullptr;
  Tile *p2tiles = nullptr;
  Tile *redjobs = nullptr;
  int64_t part_elems = 0;
  int4 *ktab = nullptr, *ijtab = nullptr, *vvtab = nullptr;
  int *vvfull = nullptr;
  EnergyJob *ejobs = nullptr;
  int nejobs = 0;
  SliceJob *slicejobs = nullptr;
  int2 *slicerows = nullptr;
  int nslicerows = 0;
  int slice_stage = 0;   // dynamic LDS bytes of the slice launch (0: rows read twice)
  bool fuse_dress = false;  // mixed Lambda: the slice launch builds the stack, no dress launch
  std::vector<BatchPlan> batches;
  int ncounters = 0;
  int64_t xbuf_elems = 0;
  // captured launch sequences, keyed by the workspace base they were built for
  std::map<void *, hipGraphExec_t> graphs;
  // plans for a caller-provided table region (allocation-free entry point):
  // the tables are kept on the host and copied to that region on every call
  std::vector<char> host_tables;
  PlanFence fence;
  ~Plan() {
    fence.wait();
    for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
    if (dtab) (void)hipFree(dtab);
  }
};

struct Workspace {
  void *dev = nullptr;
  int64_t bytes = 0;
  void *staging = nullptr;  // pinned host
  int64_t staging_bytes = 0;
  hipEvent_t ev = nullptr;
  bool ev_recorded = false;
  ~Workspace() {
    if (ev) {
      (void)hipEventSynchronize(ev);
      (void)hipEventDestroy(ev);
    }
    if (dev) (void)hipFree(dev);
    if (staging) (void)hipHostFree(staging);
  }
};

std::mutex g_mu;
int g_num_cu = 256;

// Optional event timing of kernel classes (see cdcc_timing_enable).
struct TimedSpan {
  int cls;
  int launches;
  hipEvent_t a, b;
};
bool g_timing = false;
std::vector<TimedSpan> g_spans;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t take_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// RAII bracket around the launches of one kernel class.
struct Span {
  int cls, n;
  hipStream_t s;
  hipEvent_t a = nullptr;
  Span(int c, int launches, hipStream_t st) : cls(c), n(launches), s(st) {
    if (g_timing && n > 0) {
      a = take_event();
      if (a) (void)hipEventRecord(a, s);
    }
  }
  ~Span() {
    if (!a) return;
    hipEvent_t b = take_event();
    if (!b) return;
    (void)hipEventRecord(b, s);
    g_spans.push_back({cls, n, a, b});
  }
};
PlanCache<Plan> g_plans(256);  // key includes device
std::map<std::pair<int, void *>, std::unique_ptr<Workspace>> g_ws;  // (device, stream)

int64_t env_i64(const char *name, int64_t dflt) {
  const char *v = std::getenv(name);
  if (!v || !*v) return dflt;
  return std::strtoll(v, nullptr, 10);
}

struct TableBuilder {
  std::vector<char> bytes;
  template <class T>
  int64_t add(const std::vector<T> &v) {
    const int64_t off = align_up(int64_t(bytes.size()));
    bytes.resize(off + int64_t(v.size() * sizeof(T)) + 1);
    if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
};

bool valid_sym(const cdcc_sym_t &s) {
  if (!(s.nirrep == 1 || s.nirrep == 2 || s.nirrep == 4 || s.nirrep == 8)) return false;
  for (int g = 0; g < s.nirrep; ++g)
    if (s.nocc[g] < 0 || s.nvir[g] < 0 || s.ncd[g] < 0) return false;
  return true;
}

std::string plan_key(int dev, int nsys, const cdcc_problem_t *p, int lambda, int dressed, const cdcc_opts_t &o,
                     int64_t cap) {
  std::string k;
  k.reserve(64 + nsys * 100);
  auto put = [&](int64_t x) {
    k += std::to_string(x);
    k += ',';
  };
  put(dev);
  put(lambda);
  put(dressed);
  put(o.precision);
  put(o.tile_policy);
  put(o.contract_kseg);
  put(cap);
  put(nsys);
  for (int s = 0; s < nsys; ++s) {
    const cdcc_sym_t &y = p[s].lay->sym;
    put(p[s].pair_energy != nullptr);  // the plan holds the pair-energy jobs only when asked for
    put(y.nirrep);
    for (int g = 0; g < y.nirrep; ++g) {
      put(y.nocc[g]);
      put(y.nvir[g]);
      put(y.ncd[g]);
    }
    k += '|';
  }
  return k;
}

// Tile table written by the autotuner (paper_2512_21909_amd/autotune.py):
// lines "<key> <class>[:<kseg>]" with <class> the assembly tile class and
// <kseg> the contraction's K-segment length (0 or absent: the rule below).
// Keys are either the exact shape, "<fp64|mixed|mixed_i8> <t2|lambda> h
// nocc[h] nvir[h] ncd[h]", or a shape bucket (shape_bucket), so that shapes
// never tuned themselves take the choice of tuned shapes of the same size
// class.  Read from $CDCC_TILE_TABLE or from tile_table.txt next to this
// library, once (and again after cdcc_tile_table_reload).
struct TileChoice {
  int cls = -1;
  int kseg = 0;
};
std::map<std::string, TileChoice> *g_tile_table = nullptr;
std::string g_tile_table_path;  // set by cdcc_tile_table_reload ("" = default)

const char *prec_name(int precision) {
  return precision == CDCC_MIXED_I8 ? "mixed_i8" : precision == CDCC_MIXED ? "mixed" : "fp64";
}

std::string shape_key(const cdcc_sym_t &y, int precision, int lambda) {
  std::ostringstream k;
  k << prec_name(precision) << ' ' << (lambda ? "lambda" : "t2") << ' ' << y.nirrep;
  for (const int32_t *a : {y.nocc, y.nvir, y.ncd})
    for (int g = 0; g < y.nirrep; ++g) k << ' ' << a[g];
  return k.str();
}

// Size class of a shape: "<prec> <kind> b<h> <T> <K> <M>" with T the number of
// 64 x 64 assembly tiles, K their mean Cholesky length (x2 for the Lambda
// stack) and M the largest packed occupied pair count (contraction rows), each
// as round(2 log2(x)) (half-octave buckets; -1 for zero).
std::string shape_bucket(const cdcc_sym_t &y, int precision, int lambda) {
  const int h = y.nirrep;
  const int32_t *no = y.nocc, *nv = y.nvir, *nc = y.ncd;
  const int kmul = lambda ? 2 : 1;
  double tiles = 0, kw = 0, mrows = 0;
  for (int ga = 0; ga < h; ++ga)
    for (int gb = 0; gb <= ga; ++gb) {
      const int G = ga ^ gb;
      for (int gc = 0; gc < h; ++gc) {
        const int gP = ga ^ gc, gd = gb ^ gP;
        if (nc[gP] == 0) continue;
        const double M = double(nv[ga]) * nv[gc], N = double(nv[gb]) * nv[gd] * (ga == gb ? 0.5 : 1.0);
        const double t = std::ceil(M / 64) * std::ceil(N / 64);
        tiles += t;
        kw += t * double(kmul) * nc[gP];
      }
      double pk = 0;
      for (int gi = 0; gi < h; ++gi) {
        const int gj = gi ^ G;
        if (gi > gj) pk += double(no[gi]) * no[gj];
        if (gi == gj) pk += double(no[gi]) * (no[gi] + 1) / 2;
      }
      mrows = std::max(mrows, pk);
    }
  auto b = [](double x) { return x > 0 ? long(std::lround(2.0 * std::log2(x))) : -1L; };
  std::ostringstream k;
  k << prec_name(precision) << ' ' << (lambda ? "lambda" : "t2") << " b" << h << ' ' << b(tiles) << ' '
    << b(tiles > 0 ? kw / tiles : 0) << ' ' << b(mrows);
  return k.str();
}

const std::map<std::string, TileChoice> &tile_table() {
  if (g_tile_table) return *g_tile_table;
  g_tile_table = new std::map<std::string, TileChoice>();
  std::string path = g_tile_table_path;
  if (path.empty()) {
    if (const char *e = std::getenv("CDCC_TILE_TABLE")) {
      path = e;
    } else {
      Dl_info info;
      if (dladdr(reinterpret_cast<void *>(&cdcc_irrep_layout), &info) && info.dli_fname) {
        path = info.dli_fname;
        const size_t cut = path.find_last_of('/');
        path = (cut == std::string::npos ? std::string(".") : path.substr(0, cut)) + "/tile_table.txt";
      }
    }
  }
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    if (line.empty() || line[0] == '#') continue;
    const size_t cut = line.find_last_of(' ');
    if (cut == std::string::npos) continue;
    TileChoice c;
    const char *v = line.c_str() + cut + 1;
    c.cls = std::atoi(v);
    if (const char *colon = std::strchr(v, ':')) c.kseg = std::atoi(colon + 1);
    (*g_tile_table)[line.substr(0, cut)] = c;
  }
  return *g_tile_table;
}

// The table's choice for a shape: its exact entry, else its size class's.
TileChoice table_choice(const cdcc_sym_t &y, int precision, int lambda) {
  const auto &T = tile_table();
  auto it = T.find(shape_key(y, precision, lambda));
  if (it == T.end()) it = T.find(shape_bucket(y, precision, lambda));
  return it == T.end() ? TileChoice{} : it->second;
}

int choose_p1_class(const cdcc_layout_t &L, int policy, int precision, int lambda) {
  const bool mixed = is_split(precision);
  if (policy >= 1 && policy <= (mixed ? 4 : 3)) return policy - 1;
  const TileChoice c = table_choice(L.sym, precision, lambda);
  if (c.cls >= 0 && c.cls <= (mixed ? 3 : 2)) return c.cls;
  // untuned shapes: 128 x 64 for split-BF16; 64 x 64 for the 8-bit digits
  // (thirteen accumulators per 32 x 32 block: the 64-wide waves of the other
  // classes run at one wave per SIMD)
  if (mixed) return precision == CDCC_MIXED_I8 ? 3 : 1;
  // Tile-table heuristic: the largest tile that still gives >= 2 tiles per CU.
  const int h = L.sym.nirrep;
  const int32_t *nv = L.sym.nvir, *nc = L.sym.ncd;
  double tiles[3] = {0, 0, 0};
  for (int ga = 0; ga < h; ++ga)
    for (int gb = 0; gb <= ga; ++gb)
      for (int gc = 0; gc < h; ++gc) {
        const int gP = ga ^ gc, gd = gb ^ gP;
        if (nc[gP] == 0) continue;
        const double M = double(nv[ga]) * nv[gc], N = double(nv[gb]) * nv[gd] * (ga == gb ? 0.5 : 1.0);
        for (int c = 0; c < 3; ++c) tiles[c] += std::ceil(M / kP1BM[c]) * std::ceil(N / kP1BN[c]);
      }
  // measured on the 8-irrep o=20/v=200 workload: the 64x64 class (4 waves per
  // SIMD) beats the larger ones unless there are many more tiles than slots
  if (tiles[1] >= 8192) return 1;
  return 0;
}

// Packed i>=j (or a>=b) list of pair irrep G: (x_global_row_xy, row_yx, X, Y)
void pair_table(const int32_t *n, int h, int G, const int64_t off[CDCC_MAX_IRREP], const int64_t goff[CDCC_MAX_IRREP],
                std::vector<int4> &out, int64_t sb_start[CDCC_MAX_IRREP]) {
  const int64_t first = int64_t(out.size());
  for (int g1 = 0; g1 < h; ++g1) {
    const int g2 = g1 ^ G;
    sb_start[g1] = int64_t(out.size()) - first;  // relative to this pair irrep's list
    if (g1 < g2) continue;
    for (int x = 0; x < n[g1]; ++x)
      for (int y = 0; y < (g1 == g2 ? x + 1 : n[g2]); ++y) {
        int4 e;
        e.x = int(off[g1] + int64_t(x) * n[g2] + y);
        e.y = int(off[g2] + int64_t(y) * n[g1] + x);
        e.z = int(goff[g1] + x);
        e.w = int(goff[g2] + y);
        out.push_back(e);
      }
  }
}

// table_base: NULL = the plan allocates and fills its device tables; else the
// tables are laid out for that device address and kept on the host
// (P.host_tables), and the caller copies them there before every use.
// largest (ac|bd) region of one column group (the a range is split above it)
constexpr int64_t kGroupRegionMaxBytes = int64_t(4) << 30;

int build_plan(int nsys, const cdcc_problem_t *probs, int lambda, int dressed, const cdcc_opts_t &opts, int64_t cap,
               Plan &P, void *table_base = nullptr) {
  P.nsys = nsys;
  P.lambda = lambda;
  P.dressed = dressed;
  P.precision = opts.precision;
  P.sys.resize(nsys);
  std::vector<PackJob> packjobs;
  std::vector<int2> packrows;
  std::vector<DressJob> dressjobs;
  std::vector<int2> dressrows;
  std::vector<int4> ktab, ijtab, vvtab;
  std::vector<int> vvfull;
  std::vector<EnergyJob> ejobs;
  std::vector<SliceJob> slicejobs;
  std::vector<int2> slicerows;

  struct GroupRec {
    P2Group g;
    std::vector<P1Desc> descs;
    int64_t region = 0;
    int sys = 0;
  };
  std::vector<GroupRec> groups;
  // cap_elems bounds a batch; a column group's own region is further held to
  // kGroupRegionMaxBytes
  const int64_t cap_elems = std::max<int64_t>(cap / 8, 1);
  const int64_t group_cap_elems = std::max<int64_t>(std::min(cap, kGroupRegionMaxBytes) / 8, 1);

  // rows of up to kSliceStageMax bytes are staged in LDS by the slice launch;
  // the mixed Lambda stack is then built there and never stored
  constexpr int kSliceStageMax = 48 * 1024;
  {
    int64_t mxrow = 0;
    const int km = (lambda && dressed) ? 2 : 1;
    for (int s = 0; s < nsys; ++s)
      for (int g = 0; g < probs[s].lay->sym.nirrep; ++g) mxrow = std::max<int64_t>(mxrow, int64_t(km) * probs[s].lay->sym.ncd[g] * 8);
    const bool fits = mxrow <= kSliceStageMax;
    P.slice_stage = fits ? int(std::max<int64_t>(mxrow, 8)) : 0;
    P.fuse_dress = fits && lambda && dressed != 2 && is_split(opts.precision);
  }
  for (int s = 0; s < nsys; ++s) {
    SysPlan &SP = P.sys[s];
    SP.lay = *probs[s].lay;
    const cdcc_layout_t &L = SP.lay;
    const int h = L.sym.nirrep;
    const int32_t *no = L.sym.nocc, *nv = L.sym.nvir, *nc = L.sym.ncd;
    const int kmul = (lambda && dressed) ? 2 : 1;
    const bool mixed = is_split(opts.precision);
    const int kblk = split_kblock(opts.precision), ebytes = split_elem_bytes(opts.precision);
    SP.p1cls = choose_p1_class(L, opts.tile_policy, opts.precision, lambda);
    // contraction K segment: forced, else tuned, else the rule (0)
    SP.kseg = opts.contract_kseg > 0 ? opts.contract_kseg : std::max(0, table_choice(L.sym, opts.precision, lambda).kseg);
    if (lambda && !P.fuse_dress && dressed != 2) SP.u_elems = kmul * L.b_size;
    // mixed path: slice every operand block once per call
    int64_t blk_s[CDCC_MAX_IRREP][CDCC_MAX_IRREP], blk_sc[CDCC_MAX_IRREP][CDCC_MAX_IRREP];
    int blk_kp[CDCC_MAX_IRREP];
    for (int gP = 0; gP < h; ++gP) blk_kp[gP] = kmul * ((nc[gP] + kblk - 1) / kblk * kblk);
    for (int gP = 0; gP < h; ++gP)
      for (int ga = 0; ga < h; ++ga) {
        blk_s[gP][ga] = SP.slice_bytes;
        blk_sc[gP][ga] = SP.scale_rows;
        const int64_t r = int64_t(nv[ga]) * nv[ga ^ gP];
        if (!mixed || nc[gP] == 0 || r == 0) continue;
        SliceJob J{};
        J.sys = s;
        J.rows = int(r);
        J.np = nc[gP];
        J.halves = kmul;
        J.Kp = blk_kp[gP];
        J.src_off = kmul * L.b_off[gP][ga];
        J.dst_off = SP.slice_bytes;
        J.scale_off = SP.scale_rows;
        if (P.fuse_dress) {
          const int ge = ga ^ gP;
          J.dress = 1;
          J.ve = nv[ge];
          J.om = no[ge];
          J.b_off = L.b_off[gP][ge];
          J.bvo_off = L.bvo_off[gP][ga];
          J.t1_off = L.t1_off[ge];
        }
        const int jid = int(slicejobs.size());
        slicejobs.push_back(J);
        for (int q = 0; q < r; ++q) slicerows.push_back(int2{jid, q});
        SP.slice_bytes += r * J.Kp * ebytes;
        SP.scale_rows += r;
      }

    int ij_off[CDCC_MAX_IRREP], vv_off[CDCC_MAX_IRREP], vvf_off[CDCC_MAX_IRREP];
    int64_t vv_sb[CDCC_MAX_IRREP][CDCC_MAX_IRREP], oo_sb[CDCC_MAX_IRREP];
    int64_t th_off[CDCC_MAX_IRREP];
    for (int G = 0; G < h; ++G) {
      ij_off[G] = int(ijtab.size());
      pair_table(no, h, G, L.oo_off[G], L.occ_off, ijtab, oo_sb);
      vv_off[G] = int(vvtab.size());
      pair_table(nv, h, G, L.vv_off[G], L.vir_off, vvtab, vv_sb[G]);
      vvf_off[G] = int(vvfull.size());
      for (int ga = 0; ga < h; ++ga) {
        const int gb = ga ^ G;
        for (int a = 0; a < nv[ga]; ++a)
          for (int b = 0; b < nv[gb]; ++b) vvfull.push_back(int(L.vv_off[G][gb] + int64_t(b) * nv[ga] + a));
      }
      th_off[G] = SP.th_elems;
      const int64_t nr = L.n_oo_pk[G], ncl = L.n_vv_pk[G];
      if (nr > 0 && ncl > 0) {
        PackJob J{};
        J.sys = s;
        J.nrow = int(nr);
        J.ncol = int(ncl);
        J.ldx = int(L.n_vv[G]);
        J.ij_off = ij_off[G];
        J.vv_off = vv_off[G];
        J.x_off = L.amp_off[G];
        J.th_off = SP.th_elems;
        J.ldt = int(align_up(nr, 16));  // k-major tauhat: 128-byte columns
        const int jid = int(packjobs.size());
        packjobs.push_back(J);
        // 64 x 64 (row, column) tiles, numbered rb * column_tiles + kb
        const int nrb = int((nr + 63) / 64), nkb = int((ncl + 63) / 64);
        for (int t = 0; t < nrb * nkb; ++t) packrows.push_back(int2{jid, t});
        SP.th_elems += 2 * int64_t(J.ldt) * ncl;
      }
      if (probs[s].pair_energy)
        for (int gi = 0; gi < h; ++gi) {
          const int gj = gi ^ G;
          for (int i = 0; i < no[gi]; ++i)
            for (int j = 0; j < no[gj]; ++j) {
              EnergyJob E{};
              E.sys = s;
              E.ncol = int(L.n_vv[G]);
              E.ldr = int(L.n_vv[G]);
              E.vvfull_off = vvf_off[G];
              E.row = int(L.oo_off[G][gi] + int64_t(i) * no[gj] + j);
              E.I = int(L.occ_off[gi] + i);
              E.J = int(L.occ_off[gj] + j);
              E.nocc_tot = int(L.nocc_tot);
              E.r_off = L.amp_off[G];
              if (E.ncol > 0) ejobs.push_back(E);
            }
        }
    }
    // Lambda operand stack (in the mixed path the slice launch builds it;
    // with a caller's stack there is nothing to build)
    if (lambda && !P.fuse_dress && dressed != 2)
      for (int gP = 0; gP < h; ++gP)
        for (int ga = 0; ga < h; ++ga) {
          const int ge = ga ^ gP;
          if (nc[gP] == 0 || nv[ga] == 0 || nv[ge] == 0) continue;
          DressJob D{};
          D.sys = s;
          D.va = nv[ga];
          D.ve = nv[ge];
          D.np = nc[gP];
          D.om = no[ge];
          D.u_off = kmul * L.b_off[gP][ga];
          D.b_off = L.b_off[gP][ge];
          D.bvo_off = L.bvo_off[gP][ga];
          D.t1_off = L.t1_off[ge];
          const int jid = int(dressjobs.size());
          dressjobs.push_back(D);
          for (int ae = 0; ae < nv[ga] * nv[ge]; ++ae) dressrows.push_back(int2{jid, ae});
        }

    // column groups
    for (int G = 0; G < h; ++G) {
      const int64_t n_ij = L.n_oo_pk[G];
      for (int ga = 0; ga < h; ++ga) {
        const int gb = ga ^ G;
        if (ga < gb || nv[ga] == 0 || nv[gb] == 0) continue;
        const bool tri = ga == gb;
        // region rows: (c,d) for Gc with N_{Ga^Gc} > 0
        int64_t xrow0[CDCC_MAX_IRREP];
        bool valid[CDCC_MAX_IRREP];
        int64_t nrows = 0;
        for (int gc = 0; gc < h; ++gc) {
          const int gd = gc ^ G;
          valid[gc] = nc[ga ^ gc] > 0 && nv[gc] > 0 && nv[gd] > 0;
          xrow0[gc] = nrows;
          if (valid[gc]) nrows += int64_t(nv[gc]) * nv[gd];
        }
        // K table of (G, Ga)
        const int kt_off = int(ktab.size());
        {
          const int64_t base = vv_off[G];
          for (int gc = 0; gc < h; ++gc) {
            const int gd = gc ^ G;
            if (gc < gd) continue;
            for (int c = 0; c < nv[gc]; ++c)
              for (int d = 0; d < (gc == gd ? c + 1 : nv[gd]); ++d) {
                const int64_t kcol = vv_sb[G][gc] + (gc == gd ? int64_t(c) * (c + 1) / 2 + d : int64_t(c) * nv[gd] + d);
                const int r1 = valid[gc] ? int(xrow0[gc] + int64_t(c) * nv[gd] + d) : -1;
                const int r2 = valid[gd] ? int(xrow0[gd] + int64_t(d) * nv[gc] + c) : -1;
                if (r1 < 0 && r2 < 0) continue;
                ktab.push_back(int4{int(kcol), r1, r2, 0});
              }
          }
          (void)base;
          while ((ktab.size() - kt_off) % 16) ktab.push_back(int4{-1, -1, -1, 0});
        }
        const int kt_len = int(ktab.size()) - kt_off;
        // split the a range so that one group's region fits the cap
        auto ncols_of = [&](int a0, int a1) -> int64_t {
          return tri ? (int64_t(a1) * (a1 + 1) / 2 - int64_t(a0) * (a0 + 1) / 2) : int64_t(a1 - a0) * nv[gb];
        };
        int a0 = 0;
        while (a0 < nv[ga]) {
          int a1 = a0 + 1;
          while (a1 < nv[ga] && std::max<int64_t>(nrows, 1) * ncols_of(a0, a1 + 1) <= group_cap_elems) ++a1;
          GroupRec R;
          R.sys = s;
          P2Group &g = R.g;
          g.sys = s;
          g.G = G;
          g.n_ij = int(n_ij);
          g.ncols = int(ncols_of(a0, a1));
          g.ldx = int(align_up(g.ncols, 16));  // 128-byte rows: whole cache lines per MFMA fragment
          g.ktab_len = kt_len;
          g.ktab_off = kt_off;
          g.ij_off = ij_off[G];
          g.col_off = int(vv_off[G] + vv_sb[G][ga] + (tri ? int64_t(a0) * (a0 + 1) / 2 : int64_t(a0) * nv[gb]));
          g.ldr = int(L.n_vv[G]);
          g.th_ld = int(L.n_vv_pk[G]);
          g.th_off = th_off[G];
          g.th_rs = int(align_up(n_ij, 16));
          g.r_off = L.amp_off[G];
          g.fm = contract_fm(int(n_ij));
          const int kseg_len = SP.kseg > 0 ? (SP.kseg + 15) / 16 * 16 : kKSeg;
          g.nsplit = std::max(1, (kt_len + kseg_len / 2) / kseg_len);
          g.kseg = ((kt_len + g.nsplit - 1) / g.nsplit + 15) / 16 * 16;
          if (g.nsplit > 1) g.nsplit = (kt_len + g.kseg - 1) / g.kseg;
          R.region = nrows * g.ldx;
          // assembly GEMMs
          const int bm = mixed ? kMixBM[SP.p1cls] : kP1BM[SP.p1cls];
          for (int gc = 0; gc < h; ++gc) {
            if (!valid[gc]) continue;
            const int gd = gc ^ G, gP = ga ^ gc;
            const int vc = nv[gc], vd = nv[gd];
            const int K = kmul * nc[gP];
            const int step = tri ? std::max(1, bm / std::max(vc, 1)) : (a1 - a0);
            for (int as = a0; as < a1; as += step) {
              const int ae = std::min(a1, as + step);
              P1Desc d{};
              d.sys = s;
              d.M = (ae - as) * vc;
              d.nb = tri ? ae : nv[gb];
              d.N = d.nb * vd;
              d.K = K;
              d.kneg = (lambda && dressed) ? nc[gP] : K;
              d.vc = vc;
              d.vd = vd;
              d.vb = nv[gb];
              d.a_first = as;
              d.ga0 = a0;
              d.tri = tri ? 1 : 0;
              d.ldx = g.ldx;
              d.xrow0 = int(xrow0[gc]);
              d.aoff = kmul * L.b_off[gP][ga] + int64_t(as) * vc * K;
              d.boff = kmul * L.b_off[gP][gb];
              d.Kp = blk_kp[gP];
              d.kneg_blk = (lambda && dressed) ? blk_kp[gP] / 2 / kblk : blk_kp[gP] / kblk;
              d.a_soff = blk_s[gP][ga] + int64_t(as) * vc * d.Kp * ebytes;
              d.b_soff = blk_s[gP][gb];
              d.a_scoff = blk_sc[gP][ga] + int64_t(as) * vc;
              d.b_scoff = blk_sc[gP][gb];
              R.descs.push_back(d);
            }
          }
          groups.push_back(std::move(R));
          a0 = a1;
        }
      }
    }
  }

  // batches: consecutive groups whose regions fit the cap.  Under the
  // library's default cap the call runs as one batch when all of its regions
  // fit (no launch tails between batches), else in batches of at most
  // kGroupRegionMaxBytes (larger ones measured slower at the o=135/v=543
  // size).  A cap set by the caller or by CDCC_BATCH_MB is used as given.
  int64_t batch_elems = cap_elems;
  if (opts.batch_bytes <= 0 && std::getenv("CDCC_BATCH_MB") == nullptr) {
    int64_t total = 0;
    for (const GroupRec &R : groups) total += align_up(R.region, 32);
    if (total > cap_elems) batch_elems = std::min(cap_elems, group_cap_elems);
  }
  std::vector<P1Desc> p1;
  std::vector<Tile> p1tiles;
  std::vector<P2Group> p2;
  std::vector<Tile> p2tiles;
  std::vector<Tile> redjobs;
  size_t gi = 0;
  while (gi < groups.size()) {
    int64_t used = 0;
    size_t gj = gi;
    while (gj < groups.size() && (gj == gi || used + groups[gj].region <= batch_elems)) {
      used += align_up(groups[gj].region, 32);
      ++gj;
    }
    BatchPlan B;
    // gather tiles by class
    std::vector<std::vector<std::pair<int64_t, Tile>>> t1(4), t2(1);
    // supertile shape per assembly class: as many tiles as one XCD runs at
    // once, with balanced A and B row counts
    int st_m[4], st_n[4], st_chunk[4];
    for (int c = 0; c < 4; ++c) {
      const bool mx = is_split(P.precision);
      if (!mx && c == 3) {
        st_m[c] = st_n[c] = st_chunk[c] = 1;
        continue;
      }
      const int bm = mx ? kMixBM[c] : kP1BM[c], bn = mx ? kMixBN[c] : kP1BN[c];
      const int occ = mx ? occupancy_mixed(split_fmt(P.precision), c) : occupancy_f64(0, c);
      const int conc = std::max(1, g_num_cu / 8 * occ);
      st_m[c] = std::max(1, int(std::lround(std::sqrt(double(conc) * bn / bm))));
      st_n[c] = std::max(1, conc / st_m[c]);
      st_chunk[c] = st_m[c] * st_n[c];
    }
    // deal chunks of consecutive tiles round-robin to the 8 XCD queues
    auto emit = [&](std::vector<std::pair<int64_t, Tile>> &v, int chunk, int cls, int occ,
                    std::vector<Tile> &out, std::vector<Launch> &launches) {
      if (v.empty()) return;
      std::stable_sort(v.begin(), v.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
      std::vector<std::vector<Tile>> qs(8);
      for (size_t i = 0; i < v.size(); ++i) qs[(i / chunk) % 8].push_back(v[i].second);
      Launch l;
      l.cls = cls;
      l.start = int(out.size());
      l.count = int(v.size());
      int acc = 0;
      for (int x = 0; x < 8; ++x) {
        l.q.qb[x] = acc;
        for (const Tile &t : qs[x]) out.push_back(t);
        acc += int(qs[x].size());
      }
      l.q.qb[8] = acc;
      const int cap = std::max(8, g_num_cu * std::max(occ, 1));
      l.grid = std::min(cap, (l.count + 7) / 8 * 8);
      launches.push_back(l);
    };
    int64_t xo = 0;
    int64_t po = 0;
    Launch red;
    red.start = int(redjobs.size());
    int max_tm = 1;  // most row tiles of one contraction column block in the batch
    for (size_t k = gi; k < gj; ++k) {
      GroupRec &R = groups[k];
      R.g.xoff = xo;
      xo += align_up(R.region, 32);
      const int gid = int(p2.size());
      const int bm2 = 16 * R.g.fm;
      const int tm = (R.g.n_ij + bm2 - 1) / bm2, tn = (R.g.ncols + kP2BN - 1) / kP2BN;
      max_tm = std::max(max_tm, tm);
      R.g.tiles_n = tn;
      R.g.part_off = po;
      if (R.g.n_ij > 0 && R.g.ncols > 0) {
        // the row tiles of one column block and K segment read the same X
        // columns: listed next to each other they land in one chunk of one
        // XCD's queue and run together, so X comes from that XCD's L2 once
        // instead of from HBM once per row tile
        auto push = [&](int a, int b, int ks) {
          const int len = std::min(R.g.kseg, R.g.ktab_len - ks * R.g.kseg);
          t2[0].push_back({int64_t(len) * R.g.fm + 1, Tile{gid, a, b, ks}});
        };
        if (tm > 4) {
          // many row tiles: a tile also reads 2x as many tauhat bytes (16 fm
          // rows x 2 halves) as X bytes (32 columns x 2 rows), and tauhat is
          // shared along a row of tiles, X along a column; a chunk of 3 row
          // tiles x 4 column blocks of one K segment reads each once
          constexpr int SA = 3, SB = 4;
          for (int ks = 0; ks < R.g.nsplit; ++ks)
            for (int a0 = 0; a0 < tm; a0 += SA)
              for (int b0 = 0; b0 < tn; b0 += SB)
                for (int b = b0; b < std::min(tn, b0 + SB); ++b)
                  for (int a = a0; a < std::min(tm, a0 + SA); ++a) push(a, b, ks);
        } else {
          for (int b = 0; b < tn; ++b)
            for (int ks = 0; ks < R.g.nsplit; ++ks)
              for (int a = 0; a < tm; ++a) push(a, b, ks);
        }
        if (R.g.nsplit > 1)
          for (int a = 0; a < tm; ++a)
            for (int b = 0; b < tn; ++b) redjobs.push_back(Tile{gid, a, b, 0});
        if (R.g.nsplit > 1) po += int64_t(tm) * tn * R.g.nsplit * 2 * bm2 * kP2BN;
      }
      p2.push_back(R.g);
      const int c1 = P.sys[R.sys].p1cls;
      const bool mixed = is_split(P.precision);
      const int bm = mixed ? kMixBM[c1] : kP1BM[c1], bn = mixed ? kMixBN[c1] : kP1BN[c1];
      const int stm = st_m[c1], stn = st_n[c1];
      for (P1Desc d : R.descs) {
        d.xoff = R.g.xoff;
        const int did = int(p1.size());
        p1.push_back(d);
        const int tm = (d.M + bm - 1) / bm, tn = (d.N + bn - 1) / bn;
        // stm x stn supertiles, one XCD's worth of concurrent tiles: they
        // share stm*bm A rows and stn*bn B rows in that XCD's L2
        for (int sa = 0; sa < tm; sa += stm)
          for (int sb = 0; sb < tn; sb += stn)
            for (int a = sa; a < std::min(tm, sa + stm); ++a)
              for (int b = sb; b < std::min(tn, sb + stn); ++b) {
                if (d.tri) {  // skip tiles that lie entirely above the a>=b triangle
                  const int n0 = b * bn, n1 = std::min(d.N, n0 + bn) - 1;
                  const int minb = (n0 / d.nb == n1 / d.nb) ? n0 % d.nb : 0;
                  const int maxa = d.a_first + std::min(d.M - 1, a * bm + bm - 1) / d.vc;
                  if (minb > maxa) continue;
                }
                t1[c1].push_back({int64_t(d.K), Tile{did, a, b, c1}});
              }
      }
    }
    P.xbuf_elems = std::max(P.xbuf_elems, xo);
    P.part_elems = std::max(P.part_elems, po);
    red.count = int(redjobs.size()) - red.start;
    B.red = red;
    const bool mixedp = is_split(P.precision);
    for (int c = 0; c < 4; ++c)
      emit(t1[c], st_chunk[c], c, mixedp ? occupancy_mixed(split_fmt(P.precision), c) : occupancy_f64(0, c), p1tiles,
           B.p1);
    // chunks of whole column blocks (12 holds 1-4 or 6 row tiles); 8 where
    // blocks have one or two (finer dealing balances the queues better)
    emit(t2[0], max_tm > 2 ? 12 : 8, 0, occupancy_f64(1, 0), p2tiles, B.p2);
    if (P.precision == CDCC_MIXED_I8)
      for (Launch &l : B.p1)
        for (int i = l.start; i < l.start + l.count; ++i)
          if (p1[p1tiles[i].desc].Kp > kI8MaxK) l.longk = 1;
    P.batches.push_back(std::move(B));
    gi = gj;
  }
  P.np1 = int(p1.size());
  int nl = 0;
  for (auto &b : P.batches) nl += int(b.p1.size() + b.p2.size());
  P.ncounters = 8 * nl * kQueueStride;

  // upload all tables in one allocation
  TableBuilder T;
  const int64_t o_pj = T.add(packjobs), o_pr = T.add(packrows), o_dj = T.add(dressjobs), o_dr = T.add(dressrows);
  const int64_t o_p1 = T.add(p1), o_t1 = T.add(p1tiles), o_p2 = T.add(p2), o_t2 = T.add(p2tiles);
  const int64_t o_kt = T.add(ktab), o_ij = T.add(ijtab), o_vv = T.add(vvtab), o_vf = T.add(vvfull);
  const int64_t o_ej = T.add(ejobs), o_sj = T.add(slicejobs), o_sr = T.add(slicerows);
  const int64_t o_rj = T.add(redjobs);
  char *b = nullptr;
  if (table_base) {
    P.host_tables = std::move(T.bytes);
    b = static_cast<char *>(table_base);
  } else {
    if (hipMalloc(&P.dtab, std::max<size_t>(T.bytes.size(), 256)) != hipSuccess) return CDCC_ENOMEM;
    if (hipMemcpy(P.dtab, T.bytes.data(), T.bytes.size(), hipMemcpyHostToDevice) != hipSuccess) return CDCC_EDEVICE;
    b = static_cast<char *>(P.dtab);
  }
  P.packjobs = reinterpret_cast<PackJob *>(b + o_pj);
  P.packrows = reinterpret_cast<int2 *>(b + o_pr);
  P.npackrows = int(packrows.size());
  P.dressjobs = reinterpret_cast<DressJob *>(b + o_dj);
  P.dressrows = reinterpret_cast<int2 *>(b + o_dr);
  P.ndressrows = int(dressrows.size());
  P.p1 = reinterpret_cast<P1Desc *>(b + o_p1);
  P.p1tiles = reinterpret_cast<Tile *>(b + o_t1);
  P.p2 = reinterpret_cast<P2Group *>(b + o_p2);
  P.p2tiles = reinterpret_cast<Tile *>(b + o_t2);
  P.redjobs = reinterpret_cast<Tile *>(b + o_rj);
  P.ktab = reinterpret_cast<int4 *>(b + o_kt);
  P.ijtab = reinterpret_cast<int4 *>(b + o_ij);
  P.vvtab = reinterpret_cast<int4 *>(b + o_vv);
  P.vvfull = reinterpret_cast<int *>(b + o_vf);
  P.ejobs = reinterpret_cast<EnergyJob *>(b + o_ej);
  P.nejobs = int(ejobs.size());
  P.slicejobs = reinterpret_cast<SliceJob *>(b + o_sj);
  P.slicerows = reinterpret_cast<int2 *>(b + o_sr);
  P.nslicerows = int(slicerows.size());
  return CDCC_OK;
}

// Workspace layout of one call.
constexpr int64_t kEpilogueSinkBytes = 64 * 64 * 8;

struct WsLayout {
  int64_t counters = 0, sysptrs = 0, xbuf = 0, part = 0, total = 0;
  std::vector<int64_t> th, u, sl, sc;
};

WsLayout ws_layout(const Plan &P) {
  WsLayout W;
  int64_t o = 0;
  W.counters = o;
  o = align_up(o + int64_t(std::max(P.ncounters, 1)) * 4);
  W.sysptrs = o;
  o = align_up(o + int64_t(P.nsys) * int64_t(sizeof(SysPtrs)));
  // 64 x 64 doubles just below the batch buffer take the split-BF16
  // epilogue's stores of elements it does not keep (it issues a fixed number
  // per tile)
  W.xbuf = o + kEpilogueSinkBytes;
  o = align_up(W.xbuf + P.xbuf_elems * 8);
  W.part = o;
  o = align_up(o + P.part_elems * 8);
  W.th.resize(P.nsys);
  W.u.resize(P.nsys);
  W.sl.resize(P.nsys);
  W.sc.resize(P.nsys);
  for (int s = 0; s < P.nsys; ++s) {
    W.th[s] = o;
    o = align_up(o + P.sys[s].th_elems * 8);
    W.u[s] = o;
    o = align_up(o + P.sys[s].u_elems * 8);
    W.sl[s] = o;
    o = align_up(o + P.sys[s].slice_bytes);
    W.sc[s] = o;
    o = align_up(o + P.sys[s].scale_rows * 8);
  }
  W.total = o;
  return W;
}

int validate(int32_t nsys, const cdcc_problem_t *probs, int lambda, int *dressed) {
  if (nsys < 1 || !probs) return CDCC_EINVAL;
  int dr = -1;
  for (int s = 0; s < nsys; ++s) {
    const cdcc_problem_t &p = probs[s];
    if (!p.lay || !p.B || !p.X || !p.R) return CDCC_EINVAL;
    if (!valid_sym(p.lay->sym)) return p.lay->sym.nirrep >= 1 && p.lay->sym.nirrep <= 8 ? CDCC_EUNSUPPORTED : CDCC_EINVAL;
    cdcc_layout_t chk;
    if (cdcc_irrep_layout(&p.lay->sym, &chk) != CDCC_OK) return CDCC_EINVAL;
    if (chk.amp_size != p.lay->amp_size || chk.b_size != p.lay->b_size) return CDCC_EINVAL;
    if (p.delta && (!p.eps_occ || !p.eps_vir)) return CDCC_EINVAL;
    if (lambda) {
      if ((p.Bvo == nullptr) != (p.t1 == nullptr)) return CDCC_EINVAL;
      // 0 undressed, 1 dressed here from B, L and t1, 2 dressed stack given (U)
      const int d = p.U ? 2 : (p.t1 ? 1 : 0);
      if (dr >= 0 && dr != d) return CDCC_EINVAL;  // one batch: one kind of dressing
      dr = d;
    } else if (p.U) {
      return CDCC_EINVAL;  // the stack is a Lambda operand
    }
    // the amplitude tables use 32-bit indices
    for (int G = 0; G < p.lay->sym.nirrep; ++G)
      if (p.lay->n_vv[G] >= (int64_t(1) << 31) || p.lay->n_oo[G] >= (int64_t(1) << 31)) return CDCC_EUNSUPPORTED;
  }
  *dressed = dr > 0 ? dr : 0;
  return CDCC_OK;
}

// Default cap of the (ac|bd) batch buffer: 16 GiB, a small share of the 288 GB
// of one MI355X; fewer, larger batches fill the chip better (each launch ends
// in a tail where CUs idle).  The vvvv density keeps 4 GiB batches.
constexpr int64_t kDefaultBatchMB = 16384;
constexpr int64_t kDefaultDensityBatchMB = 4096;

int64_t batch_cap(const cdcc_opts_t &o) {
  int64_t cap = o.batch_bytes > 0 ? o.batch_bytes : env_i64("CDCC_BATCH_MB", kDefaultBatchMB) * (int64_t(1) << 20);
  return std::max<int64_t>(cap, 1 << 16);
}

int get_plan(int dev, int32_t nsys, const cdcc_problem_t *probs, int lambda, int dressed, const cdcc_opts_t &opts,
             std::shared_ptr<Plan> &out) {
  const int64_t cap = batch_cap(opts);
  const std::string key = plan_key(dev, nsys, probs, lambda, dressed, opts, cap);
  if (auto hit = g_plans.find(key)) {
    out = hit;
    return CDCC_OK;
  }
  auto P = std::make_shared<Plan>();
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0) g_num_cu = ncu;
  const int rc = build_plan(nsys, probs, lambda, dressed, opts, cap, *P);
  if (rc != CDCC_OK) return rc;
  g_plans.put(key, P);
  out = P;
  return CDCC_OK;
}

int get_workspace(int dev, hipStream_t stream, int64_t bytes, int64_t staging, Workspace *&out) {
  auto &slot = g_ws[{dev, (void *)stream}];
  if (!slot) slot.reset(new Workspace());
  Workspace &W = *slot;
  const int64_t fail_above = env_i64("CDCC_FAIL_ALLOC_ABOVE", -1);
  if (W.bytes < bytes) {
    if (fail_above >= 0 && bytes > fail_above) return CDCC_ENOMEM;
    if (W.dev) {
      if (hipStreamSynchronize(stream) != hipSuccess) return CDCC_EDEVICE;
      (void)hipFree(W.dev);
      W.dev = nullptr;
      W.bytes = 0;
    }
    if (hipMalloc(&W.dev, bytes) != hipSuccess) {
      (void)hipGetLastError();
      W.dev = nullptr;
      return CDCC_ENOMEM;
    }
    W.bytes = bytes;
  }
  if (!W.ev) {
    if (hipEventCreateWithFlags(&W.ev, hipEventDisableTiming) != hipSuccess) return CDCC_EDEVICE;
  }
  if (W.staging_bytes < staging) {
    if (W.ev_recorded && hipEventSynchronize(W.ev) != hipSuccess) return CDCC_EDEVICE;
    if (W.staging) (void)hipHostFree(W.staging);
    W.staging = nullptr;
    if (hipHostMalloc(&W.staging, staging, hipHostMallocDefault) != hipSuccess) return CDCC_ENOMEM;
    W.staging_bytes = staging;
  }
  out = &W;
  return CDCC_OK;
}

#define HIPCHK(x)                               \
  do {                                          \
    if ((x) != hipSuccess) return CDCC_EDEVICE; \
  } while (0)

// Every kernel of one evaluation, in order, on stream s.
int enqueue_sequence(const Plan &Pl, SysPtrs *dsp, int *counters, double *xbuf, double *part, hipStream_t stream) {
  const Plan *P = &Pl;
  HIPCHK(launch_fill_int(counters, P->ncounters, 0, stream));
  if (P->lambda && !P->fuse_dress && P->ndressrows > 0) {
    Span sp(0, P->ndressrows > 0, stream);
    HIPCHK(launch_dress(P->dressjobs, P->dressrows, P->ndressrows, dsp, stream));
  }
  if (is_split(P->precision)) {
    Span sp(5, P->nslicerows > 0, stream);
    HIPCHK(launch_slice(split_fmt(P->precision), P->slicejobs, P->slicerows, P->nslicerows, dsp, P->slice_stage, stream));
  }
  {
    Span sp(1, P->npackrows > 0, stream);
    HIPCHK(launch_pack(P->packjobs, P->packrows, P->npackrows, dsp, P->ijtab, P->vvtab, stream));
  }
  int ci = 0;
  for (const BatchPlan &B : P->batches) {
    {
      Span sp(2, int(B.p1.size()), stream);
      for (const Launch &l : B.p1) {
        int *cnt = counters + 8 * kQueueStride * ci++;
        if (is_split(P->precision))
          HIPCHK(launch_assemble_mixed(split_fmt(P->precision), l.cls, l.longk, P->lambda && P->dressed, l.grid,
                                       P->p1, P->p1tiles + l.start, l.q, cnt, dsp, xbuf, stream));
        else
          HIPCHK(launch_assemble_f64(l.cls, l.grid, P->p1, P->p1tiles + l.start, l.q, cnt, dsp, xbuf, stream));
      }
    }
    {
      Span sp(3, int(B.p2.size()), stream);
      for (const Launch &l : B.p2)
        HIPCHK(launch_contract_f64(l.grid, P->p2, P->p2tiles + l.start, l.q, counters + 8 * kQueueStride * ci++, dsp, xbuf,
                                   P->ktab, P->ijtab, P->vvtab, part, stream));
      HIPCHK(launch_reduce_unpack(B.red.count, P->p2, P->redjobs + B.red.start, dsp, part, P->ijtab,
                                  P->vvtab, stream));
    }
  }
  {
    Span sp(4, P->nejobs > 0, stream);
    HIPCHK(launch_energy(P->ejobs, P->nejobs, dsp, P->vvfull, stream));
  }
  return CDCC_OK;
}

std::map<int, hipStream_t> g_capture_streams;

hipStream_t capture_stream(int dev) {
  auto it = g_capture_streams.find(dev);
  if (it != g_capture_streams.end()) return it->second;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
  g_capture_streams[dev] = s;
  return s;
}

int run_ladder(int32_t nsys, const cdcc_problem_t *probs, const cdcc_opts_t *popts, void *vstream, int lambda) {
  cdcc_opts_t opts{};
  if (popts) opts = *popts;
  if (opts.precision != CDCC_FP64 && !is_split(opts.precision)) return CDCC_EINVAL;
  if (opts.tile_policy < 0 || opts.tile_policy > 4) return CDCC_EINVAL;
  if (opts.tile_policy == 4 && !is_split(opts.precision)) return CDCC_EINVAL;
  if (opts.contract_kseg < 0 || opts.contract_kseg > (1 << 20)) return CDCC_EINVAL;
  int dressed = 0;
  int rc = validate(nsys, probs, lambda, &dressed);
  if (rc != CDCC_OK) return rc;
  hipStream_t stream = static_cast<hipStream_t>(vstream);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));

  std::lock_guard<std::mutex> lock(g_mu);
  std::shared_ptr<Plan> P;
  rc = get_plan(dev, nsys, probs, lambda, dressed, opts, P);
  if (rc != CDCC_OK) return rc;
  const WsLayout W = ws_layout(*P);
  Workspace *ws = nullptr;
  rc = get_workspace(dev, stream, W.total, int64_t(nsys) * sizeof(SysPtrs), ws);
  if (rc != CDCC_OK) return rc;
  char *base = static_cast<char *>(ws->dev);

  // per-call pointer table
  if (ws->ev_recorded) HIPCHK(hipEventSynchronize(ws->ev));
  SysPtrs *hs = static_cast<SysPtrs *>(ws->staging);
  for (int s = 0; s < nsys; ++s) {
    const cdcc_problem_t &p = probs[s];
    SysPtrs q{};
    q.opnd = !lambda ? p.B : (dressed == 2 ? p.U : reinterpret_cast<const double *>(base + W.u[s]));
    q.X = p.X;
    q.R = p.R;
    q.delta = p.delta;
    q.eps_occ = p.eps_occ;
    q.eps_vir = p.eps_vir;
    q.epair = p.pair_energy;
    q.eamp = p.energy_amps ? p.energy_amps : p.X;
    q.tauhat = reinterpret_cast<double *>(base + W.th[s]);
    q.B = p.B;
    q.Bvo = p.Bvo;
    q.t1 = p.t1;
    q.slices = reinterpret_cast<unsigned char *>(base + W.sl[s]);
    q.rowscale = reinterpret_cast<double *>(base + W.sc[s]);
    hs[s] = q;
  }
  SysPtrs *dsp = reinterpret_cast<SysPtrs *>(base + W.sysptrs);
  HIPCHK(hipMemcpyAsync(dsp, hs, size_t(nsys) * sizeof(SysPtrs), hipMemcpyHostToDevice, stream));
  HIPCHK(hipEventRecord(ws->ev, stream));
  ws->ev_recorded = true;

  int *counters = reinterpret_cast<int *>(base + W.counters);
  double *xbuf = reinterpret_cast<double *>(base + W.xbuf);
  double *part = reinterpret_cast<double *>(base + W.part);
  const bool use_graph = !g_timing && env_i64("CDCC_GRAPH", 1) != 0;
  if (!use_graph) {
    rc = enqueue_sequence(*P, dsp, counters, xbuf, part, stream);
    P->fence.mark(stream);
    return rc;
  }
  auto it = P->graphs.find(ws->dev);
  if (it == P->graphs.end()) {
    // capture the kernel sequence once per (plan, workspace) on a private stream
    hipStream_t cap = capture_stream(dev);
    if (!cap) return CDCC_EDEVICE;
    HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    const int rc2 = enqueue_sequence(*P, dsp, counters, xbuf, part, cap);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cap, &graph);
    if (rc2 != CDCC_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc2 != CDCC_OK ? rc2 : CDCC_EDEVICE;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return CDCC_EDEVICE;
    it = P->graphs.emplace(ws->dev, exec).first;
  }
  HIPCHK(hipGraphLaunch(it->second, stream));
  P->fence.mark(stream);
  return CDCC_OK;
}

// ===========================================================================
// vvvv spin-adapted two-body density (Appendix two-body densities; density
// section, Gamma~ = 2 Gamma_PqRs - Gamma_PqSr; gradient section):
//   W_(ab),(cd) = sum_mn [Y_mn^ab X'_mn^cd + X_mn^ab Y'_mn^cd]  = 2 Gamma~_abcd
//   X'^cd = 2 X^cd - X^dc,  Y'^cd = 2 Y^cd - Y^dc
//   G^P_ac      = 1/2 sum_bd W_(ab),(cd) L^P_bd
// Regions: for each (system, Cholesky irrep GP, Ga) and range of a, the W
// rows (a, c) (c in Ga^GP) times all (b, d) pairs of GP go to the batch
// buffer (first stage: one T T'^T GEMM per Gb, K = 2 n_oo(Ga^Gb)); the second
// stage multiplies the region by the GP block of L and writes the result rows
// (a, c) of block (GP, Ga): directly when K = n_vv(GP) fits one segment, else
// through partial tiles and the reduction.  Every result element is written
// once.
// ===========================================================================
struct DensBatch {
  Launch w, g;
  int rstart = 0, rcount = 0;  // reduction jobs
};

struct DensPlan {
  int nsys = 0;
  void *dtab = nullptr;
  DensPackJob *packjobs = nullptr;
  int2 *packtiles = nullptr;
  int *swap = nullptr;  // per (system, pair irrep): column of (d,c) for each column (c,d)
  int npacktiles = 0;
  P1Desc *wdesc = nullptr;
  Tile *wtiles = nullptr;
  GemmDesc *gdesc = nullptr;
  Tile *gtiles = nullptr;
  Tile *rjobs = nullptr;
  std::vector<DensBatch> batches;
  int ncounters = 0;
  int64_t xbuf_elems = 0, part_elems = 0;
  std::vector<int64_t> t_elems;
  PlanFence fence;
  ~DensPlan() {
    fence.wait();
    if (dtab) (void)hipFree(dtab);
  }
};
PlanCache<DensPlan> g_dplans(64);

int64_t vv_count(const cdcc_layout_t &L, int G) { return L.n_vv[G]; }

// Deal a tile list to the eight XCD queues in chunks (longest first).
Launch deal_tiles(std::vector<std::pair<int64_t, Tile>> &v, int chunk, int occ, std::vector<Tile> &out) {
  Launch l;
  std::stable_sort(v.begin(), v.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
  std::vector<std::vector<Tile>> qs(8);
  for (size_t i = 0; i < v.size(); ++i) qs[(i / chunk) % 8].push_back(v[i].second);
  l.start = int(out.size());
  int acc = 0;
  for (int x = 0; x < 8; ++x) {
    l.q.qb[x] = acc;
    for (const Tile &t : qs[x]) out.push_back(t);
    acc += int(qs[x].size());
  }
  l.q.qb[8] = acc;
  l.count = acc;
  const int cap = std::max(8, g_num_cu * std::max(occ, 1));
  l.grid = acc > 0 ? std::min(cap, (acc + 7) / 8 * 8) : 0;
  return l;
}

int build_density_plan(int nsys, const cdcc_density_problem_t *probs, int64_t cap, DensPlan &P) {
  constexpr int WBM = 128, WBN = 64, GBM = kGemmBM, GBN = kGemmBN;
  P.nsys = nsys;
  P.t_elems.assign(nsys, 0);
  const int64_t cap_elems = std::max<int64_t>(cap / 8, 1);
  std::vector<DensPackJob> packjobs;
  std::vector<int2> packtiles;
  std::vector<int> swap;
  struct Region {
    int sys;
    int64_t elems;
    std::vector<P1Desc> w;
    GemmDesc g;
  };
  std::vector<Region> regions;
  for (int s = 0; s < nsys; ++s) {
    const cdcc_layout_t &L = *probs[s].lay;
    const int h = L.sym.nirrep;
    const int32_t *no = L.sym.nocc, *nv = L.sym.nvir, *nc = L.sym.ncd;
    // T tables: per pair irrep G, [Y | X] rows then [X' | Y'] rows (K = 2 n_oo)
    int64_t tw_off[CDCC_MAX_IRREP], tv_off[CDCC_MAX_IRREP];
    int64_t t = 0;
    for (int G = 0; G < h; ++G) {
      const int64_t K2 = 2 * L.n_oo[G], nr = L.n_vv[G];
      tw_off[G] = t;
      tv_off[G] = t + nr * K2;
      if (K2 > 0 && nr > 0) {
        DensPackJob J{};
        J.sys = s;
        J.nrow = int(L.n_oo[G]);
        J.ncol = int(nr);
        J.x_off = L.amp_off[G];
        J.tw_off = t;
        J.sw_off = int(swap.size());
        swap.resize(swap.size() + size_t(nr), -1);
        for (int gc = 0; gc < h; ++gc) {
          const int gd = gc ^ G;
          for (int c = 0; c < nv[gc]; ++c)
            for (int d = 0; d < nv[gd]; ++d)
              swap[size_t(J.sw_off) + size_t(L.vv_off[G][gc] + int64_t(c) * nv[gd] + d)] =
                  int(L.vv_off[G][gd] + int64_t(d) * nv[gc] + c);
        }
        const int jid = int(packjobs.size());
        packjobs.push_back(J);
        const int nt = int((L.n_oo[G] + 63) / 64 * ((nr + 63) / 64));
        for (int q = 0; q < nt; ++q) packtiles.push_back(int2{jid, q});
      }
      t += 2 * nr * K2;
    }
    P.t_elems[s] = t + 64;  // padding: a K = 0 block reads (masked) at offset 0
    for (int gP = 0; gP < h; ++gP) {
      const int64_t kvv = L.n_vv[gP];
      if (nc[gP] == 0 || kvv == 0) continue;
      const int64_t ldw = align_up(kvv, 4);  // W row stride: 32-byte aligned rows for the GEMM's A loads
      for (int ga = 0; ga < h; ++ga) {
        const int gc = ga ^ gP;
        if (nv[ga] == 0 || nv[gc] == 0) continue;
        const int64_t per_a = int64_t(nv[gc]) * ldw;
        const int step = int(std::max<int64_t>(1, std::min<int64_t>(nv[ga], cap_elems / std::max<int64_t>(per_a, 1))));
        for (int a0 = 0; a0 < nv[ga]; a0 += step) {
          const int a1 = std::min(nv[ga], a0 + step);
          Region R;
          R.sys = s;
          R.elems = int64_t(a1 - a0) * per_a;
          for (int gb = 0; gb < h; ++gb) {
            const int gd = gb ^ gP, G = ga ^ gb;
            if (nv[gb] == 0 || nv[gd] == 0) continue;
            const int K = int(2 * L.n_oo[G]);
            P1Desc d{};
            d.sys = s;
            d.M = (a1 - a0) * nv[gb];
            d.N = nv[gc] * nv[gd];
            d.K = K;
            d.kneg = K;
            d.vc = nv[gb];
            d.vd = nv[gd];
            d.vb = nv[gb];
            d.nb = nv[gc];
            d.a_first = a0;
            d.ga0 = a0;
            d.tri = 0;
            d.ldx = int(ldw);
            d.xrow0 = int(L.vv_off[gP][gb]);
            d.aoff = K > 0 ? tw_off[G] + (L.vv_off[G][ga] + int64_t(a0) * nv[gb]) * K : 0;
            d.boff = K > 0 ? tv_off[G] + L.vv_off[G][gc] * K : 0;
            R.w.push_back(d);
          }
          GemmDesc g{};
          g.sys = s;
          g.M = (a1 - a0) * nv[gc];
          g.N = nc[gP];
          g.K = int(kvv);
          g.lda = int(ldw);
          g.ldb = nc[gP];
          g.ldc = nc[gP];
          g.boff = L.b_off[gP][0];
          g.coff = L.b_off[gP][ga] + int64_t(a0) * nv[gc] * nc[gP];
          g.alpha = 0.5;
          R.g = g;
          regions.push_back(std::move(R));
        }
      }
    }
  }
  // batches of regions under the cap
  std::vector<P1Desc> wd;
  std::vector<GemmDesc> gd;
  std::vector<Tile> wt, gt, rjobs;
  const int occw = occupancy_density_w(), occg = occupancy_density_gemm();
  size_t ri = 0;
  int nl = 0;
  while (ri < regions.size()) {
    size_t rj = ri;
    int64_t used = 0;
    while (rj < regions.size() && (rj == ri || used + align_up(regions[rj].elems, 32) <= cap_elems)) {
      used += align_up(regions[rj].elems, 32);
      ++rj;
    }
    std::vector<std::pair<int64_t, Tile>> tw, tg;
    int64_t xo = 0, po = 0;
    const int rstart = int(rjobs.size());
    for (size_t k = ri; k < rj; ++k) {
      Region &R = regions[k];
      for (P1Desc d : R.w) {
        d.xoff = xo;
        const int did = int(wd.size());
        wd.push_back(d);
        const int tm = (d.M + WBM - 1) / WBM, tn = (d.N + WBN - 1) / WBN;
        for (int a = 0; a < tm; ++a)
          for (int b = 0; b < tn; ++b) tw.push_back({int64_t(d.K) + 1, Tile{did, a, b, 0}});
      }
      GemmDesc g = R.g;
      g.aoff = xo;
      const int tm = (g.M + GBM - 1) / GBM, tn = (g.N + GBN - 1) / GBN;
      g.nseg = (g.K + kGemmKSeg - 1) / kGemmKSeg;
      g.tiles_n = tn;
      g.poff = po;
      if (g.nseg > 1) po += int64_t(tm) * tn * g.nseg * GBM * GBN;
      const int gid = int(gd.size());
      gd.push_back(g);
      for (int a = 0; a < tm; ++a)
        for (int b = 0; b < tn; ++b) {
          for (int sg = 0; sg < g.nseg; ++sg)
            tg.push_back({int64_t(std::min(g.K - sg * kGemmKSeg, kGemmKSeg)) + 1, Tile{gid, a, b, sg}});
          if (g.nseg > 1) rjobs.push_back(Tile{gid, a, b, 0});
        }
      xo += align_up(R.elems, 32);
    }
    P.xbuf_elems = std::max(P.xbuf_elems, xo);
    P.part_elems = std::max(P.part_elems, po);
    DensBatch B;
    B.w = deal_tiles(tw, 16, occw, wt);
    B.g = deal_tiles(tg, 16, occg, gt);
    B.rstart = rstart;
    B.rcount = int(rjobs.size()) - rstart;
    P.batches.push_back(B);
    nl += 2;
    ri = rj;
  }
  P.ncounters = 8 * std::max(nl, 1) * kQueueStride;
  TableBuilder T;
  const int64_t o_pj = T.add(packjobs), o_pt = T.add(packtiles), o_wd = T.add(wd), o_wt = T.add(wt);
  const int64_t o_gd = T.add(gd), o_gt = T.add(gt), o_rj = T.add(rjobs), o_sw = T.add(swap);
  if (hipMalloc(&P.dtab, std::max<size_t>(T.bytes.size(), 256)) != hipSuccess) return CDCC_ENOMEM;
  if (hipMemcpy(P.dtab, T.bytes.data(), T.bytes.size(), hipMemcpyHostToDevice) != hipSuccess) return CDCC_EDEVICE;
  char *b = static_cast<char *>(P.dtab);
  P.packjobs = reinterpret_cast<DensPackJob *>(b + o_pj);
  P.packtiles = reinterpret_cast<int2 *>(b + o_pt);
  P.npacktiles = int(packtiles.size());
  P.wdesc = reinterpret_cast<P1Desc *>(b + o_wd);
  P.wtiles = reinterpret_cast<Tile *>(b + o_wt);
  P.gdesc = reinterpret_cast<GemmDesc *>(b + o_gd);
  P.gtiles = reinterpret_cast<Tile *>(b + o_gt);
  P.rjobs = reinterpret_cast<Tile *>(b + o_rj);
  P.swap = reinterpret_cast<int *>(b + o_sw);
  return CDCC_OK;
}

int validate_density(int32_t nsys, const cdcc_density_problem_t *probs) {
  if (nsys < 0 || (nsys > 0 && !probs)) return CDCC_EINVAL;
  for (int s = 0; s < nsys; ++s) {
    const cdcc_density_problem_t &p = probs[s];
    if (!p.lay) return CDCC_EINVAL;
    if (!valid_sym(p.lay->sym)) return p.lay->sym.nirrep > 0 ? CDCC_EUNSUPPORTED : CDCC_EINVAL;
    if (p.lay->amp_size > 0 && (!p.X || !p.Y)) return CDCC_EINVAL;
    if (p.lay->b_size > 0 && (!p.L || !p.G)) return CDCC_EINVAL;
  }
  return CDCC_OK;
}

struct DensWs {
  int64_t counters = 0, dptrs = 0, sptrs = 0, xbuf = 0, part = 0, total = 0;
  std::vector<int64_t> t;
};
DensWs dens_ws_layout(const DensPlan &P) {
  DensWs W;
  int64_t o = 0;
  W.counters = o;
  o = align_up(o + int64_t(std::max(P.ncounters, 1)) * 4);
  W.dptrs = o;
  o = align_up(o + int64_t(P.nsys) * int64_t(sizeof(DensPtrs)));
  W.sptrs = o;
  o = align_up(o + int64_t(P.nsys) * int64_t(sizeof(SysPtrs)));
  W.xbuf = o;
  o = align_up(o + P.xbuf_elems * 8);
  W.part = o;
  o = align_up(o + P.part_elems * 8);
  W.t.resize(P.nsys);
  for (int s = 0; s < P.nsys; ++s) {
    W.t[s] = o;
    o = align_up(o + P.t_elems[s] * 8);
  }
  W.total = o;
  return W;
}

int run_density(int32_t nsys, const cdcc_density_problem_t *probs, const cdcc_opts_t *popts, void *vstream) {
  cdcc_opts_t opts{};
  if (popts) opts = *popts;
  if (opts.precision != CDCC_FP64) return is_split(opts.precision) ? CDCC_EUNSUPPORTED : CDCC_EINVAL;
  int rc = validate_density(nsys, probs);
  if (rc != CDCC_OK) return rc;
  if (nsys == 0) return CDCC_OK;
  hipStream_t stream = static_cast<hipStream_t>(vstream);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_mu);
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0) g_num_cu = ncu;
  }
  const int64_t cap =
      opts.batch_bytes > 0 ? opts.batch_bytes : env_i64("CDCC_BATCH_MB", kDefaultDensityBatchMB) * (int64_t(1) << 20);
  std::string key = "density|" + std::to_string(dev) + "|" + std::to_string(cap) + "|" + std::to_string(nsys);
  for (int s = 0; s < nsys; ++s) {
    const cdcc_sym_t &y = probs[s].lay->sym;
    key += "|" + std::to_string(y.nirrep);
    for (int g = 0; g < y.nirrep; ++g)
      key += "," + std::to_string(y.nocc[g]) + "," + std::to_string(y.nvir[g]) + "," + std::to_string(y.ncd[g]);
  }
  std::shared_ptr<DensPlan> P = g_dplans.find(key);
  if (!P) {
    P = std::make_shared<DensPlan>();
    rc = build_density_plan(nsys, probs, cap, *P);
    if (rc != CDCC_OK) return rc;
    g_dplans.put(key, P);
  }
  const DensWs W = dens_ws_layout(*P);
  Workspace *ws = nullptr;
  rc = get_workspace(dev, stream, W.total, int64_t(nsys) * int64_t(sizeof(DensPtrs) + sizeof(SysPtrs)), ws);
  if (rc != CDCC_OK) return rc;
  char *base = static_cast<char *>(ws->dev);
  if (ws->ev_recorded) HIPCHK(hipEventSynchronize(ws->ev));
  DensPtrs *hd = static_cast<DensPtrs *>(ws->staging);
  SysPtrs *hs = reinterpret_cast<SysPtrs *>(hd + nsys);
  for (int s = 0; s < nsys; ++s) {
    DensPtrs d{};
    d.X = probs[s].X;
    d.Y = probs[s].Y;
    d.L = probs[s].L;
    d.G = probs[s].G;
    d.T = reinterpret_cast<double *>(base + W.t[s]);
    hd[s] = d;
    SysPtrs q{};
    q.opnd = d.T;
    hs[s] = q;
  }
  DensPtrs *ddp = reinterpret_cast<DensPtrs *>(base + W.dptrs);
  SysPtrs *dsp = reinterpret_cast<SysPtrs *>(base + W.sptrs);
  HIPCHK(hipMemcpyAsync(ddp, hd, size_t(nsys) * sizeof(DensPtrs), hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemcpyAsync(dsp, hs, size_t(nsys) * sizeof(SysPtrs), hipMemcpyHostToDevice, stream));
  HIPCHK(hipEventRecord(ws->ev, stream));
  ws->ev_recorded = true;

  int *counters = reinterpret_cast<int *>(base + W.counters);
  double *xbuf = reinterpret_cast<double *>(base + W.xbuf);
  double *part = reinterpret_cast<double *>(base + W.part);
  HIPCHK(launch_fill_int(counters, P->ncounters, 0, stream));
  {
    Span sp(1, P->npacktiles > 0, stream);
    HIPCHK(launch_density_pack(P->packjobs, P->packtiles, P->npacktiles, P->swap, ddp, stream));
  }
  int ci = 0;
  for (const DensBatch &B : P->batches) {
    {
      Span sp(6, B.w.count > 0, stream);
      HIPCHK(launch_assemble_density(B.w.grid, P->wdesc, P->wtiles + B.w.start, B.w.q,
                                     counters + 8 * kQueueStride * ci++, dsp, xbuf, stream));
    }
    {
      Span sp(7, B.g.count > 0, stream);
      HIPCHK(launch_density_gemm(B.g.grid, P->gdesc, P->gtiles + B.g.start, B.g.q,
                                 counters + 8 * kQueueStride * ci++, ddp, xbuf, part, stream));
    }
    if (B.rcount > 0) {
      Span sp(8, true, stream);
      HIPCHK(launch_density_reduce(B.rcount, P->gdesc, P->rjobs + B.rstart, ddp, part, stream));
    }
  }
  P->fence.mark(stream);
  return CDCC_OK;
}

// ===========================================================================
// O(O^3 V^3) contraction, partial symmetric-antisymmetric algorithm (the
// paragraph closing the I_pq section): M_bi^dc = sum_mn lam_bi^mn tau_mn^dc.
// One block per (system, pair irrep G) with rows (b,i); K = the m >= n pairs
// of G; columns = squares of 8 d x 8 c over the d >= c pairs.  Each launch
// covers every block of every system; every element of M is written once.
// ===========================================================================
struct PmPlan {
  int nsys = 0;
  void *dtab = nullptr;
  PmDesc *descs = nullptr;
  int4 *tiles = nullptr;
  int ntiles = 0;
  PmSquare *sqs = nullptr;
  int2 *kp = nullptr;
  PmChunk *lchunks = nullptr, *tchunks = nullptr;
  int nlchunks = 0, ntchunks = 0;
  std::vector<int64_t> ws_elems;
  PlanFence fence;
  ~PmPlan() {
    fence.wait();
    if (dtab) (void)hipFree(dtab);
  }
};
PlanCache<PmPlan> g_pmplans(64);

int build_pm_plan(int nsys, const cdcc_partial_problem_t *probs, PmPlan &P) {
  constexpr int BM = 64;
  P.nsys = nsys;
  P.ws_elems.assign(nsys, 0);
  std::vector<PmDesc> descs;
  std::vector<int4> tiles;
  std::vector<PmSquare> sqs;
  std::vector<int2> kp;
  std::vector<PmChunk> lch, tch;
  for (int s = 0; s < nsys; ++s) {
    const cdcc_layout_t &L = *probs[s].lay;
    cdcc_vo_layout_t V;
    if (cdcc_vo_layout(&L, &V) != CDCC_OK) return CDCC_EINVAL;
    const int h = L.sym.nirrep;
    const int32_t *no = L.sym.nocc, *nv = L.sym.nvir;
    int64_t wo = 0;
    for (int G = 0; G < h; ++G) {
      if (V.n_vo[G] == 0 || L.n_vv[G] == 0) continue;
      PmDesc D{};
      D.sys = s;
      D.nrow = int(V.n_vo[G]);
      D.kp_off = int(kp.size());
      for (int gm = 0; gm < h; ++gm) {
        const int gn = gm ^ G;
        if (gm < gn) continue;
        for (int m = 0; m < no[gm]; ++m)
          for (int n = 0; n < (gm == gn ? m + 1 : no[gn]); ++n)
            kp.push_back(int2{int(L.oo_off[G][gm] + int64_t(m) * no[gn] + n),
                              int(L.oo_off[G][gn] + int64_t(n) * no[gm] + m)});
      }
      D.nk = int(kp.size()) - D.kp_off;
      D.ldk = int(align_up(int64_t(D.nk), 16));
      D.sq_off = int(sqs.size());
      for (int gd = 0; gd < h; ++gd) {
        const int gc = gd ^ G;
        if (gd < gc || nv[gd] == 0 || nv[gc] == 0) continue;
        const int nbd = (nv[gd] + 7) / 8, nbc = (nv[gc] + 7) / 8;
        for (int dB = 0; dB < nbd; ++dB)
          for (int cB = 0; cB < nbc; ++cB) {
            if (gd == gc && cB > dB) continue;
            PmSquare Q{};
            Q.base_dc = int(L.vv_off[G][gd] + int64_t(dB) * 8 * nv[gc] + cB * 8);
            Q.base_cd = int(L.vv_off[G][gc] + int64_t(cB) * 8 * nv[gd] + dB * 8);
            Q.ld_dc = nv[gc];
            Q.ld_cd = nv[gd];
            Q.nd = std::min(8, nv[gd] - dB * 8);
            Q.nc = std::min(8, nv[gc] - cB * 8);
            Q.diag = (gd == gc && dB == cB) ? 1 : 0;
            sqs.push_back(Q);
          }
      }
      D.nsq = int(sqs.size()) - D.sq_off;
      D.lam_off = V.lam_off[G];
      D.tau_off = L.amp_off[G];
      D.m_off = V.m_off[G];
      D.n_oo = L.n_oo[G];
      D.n_vv = L.n_vv[G];
      D.lp_off = wo;
      wo += align_up(2 * int64_t(D.nrow) * D.ldk, 32);
      D.tp_off = wo;
      wo += align_up(2 * int64_t(D.ldk) * D.nsq * 64, 32);
      const int did = int(descs.size());
      descs.push_back(D);
      const int tm = (D.nrow + BM - 1) / BM;
      for (int a = 0; a < tm; ++a)
        for (int q = 0; q < D.nsq; ++q) tiles.push_back(int4{did, a, q, 0});
      const int64_t nl = (int64_t(D.nrow) * D.ldk + 255) / 256, nt = (int64_t(D.ldk) * D.nsq * 64 + 255) / 256;
      for (int64_t c = 0; c < nl; ++c) lch.push_back(PmChunk{did, int(c)});
      for (int64_t c = 0; c < nt; ++c) tch.push_back(PmChunk{did, int(c)});
    }
    P.ws_elems[s] = wo;
  }
  TableBuilder T;
  const int64_t o_d = T.add(descs), o_t = T.add(tiles), o_s = T.add(sqs), o_k = T.add(kp);
  const int64_t o_l = T.add(lch), o_c = T.add(tch);
  if (hipMalloc(&P.dtab, std::max<size_t>(T.bytes.size(), 256)) != hipSuccess) return CDCC_ENOMEM;
  if (hipMemcpy(P.dtab, T.bytes.data(), T.bytes.size(), hipMemcpyHostToDevice) != hipSuccess) return CDCC_EDEVICE;
  char *b = static_cast<char *>(P.dtab);
  P.descs = reinterpret_cast<PmDesc *>(b + o_d);
  P.tiles = reinterpret_cast<int4 *>(b + o_t);
  P.ntiles = int(tiles.size());
  P.sqs = reinterpret_cast<PmSquare *>(b + o_s);
  P.kp = reinterpret_cast<int2 *>(b + o_k);
  P.lchunks = reinterpret_cast<PmChunk *>(b + o_l);
  P.nlchunks = int(lch.size());
  P.tchunks = reinterpret_cast<PmChunk *>(b + o_c);
  P.ntchunks = int(tch.size());
  return CDCC_OK;
}

int validate_partial(int32_t nsys, const cdcc_partial_problem_t *probs) {
  if (nsys < 0 || (nsys > 0 && !probs)) return CDCC_EINVAL;
  for (int s = 0; s < nsys; ++s) {
    const cdcc_partial_problem_t &p = probs[s];
    if (!p.lay) return CDCC_EINVAL;
    if (!valid_sym(p.lay->sym)) return p.lay->sym.nirrep > 0 ? CDCC_EUNSUPPORTED : CDCC_EINVAL;
    cdcc_vo_layout_t V;
    if (cdcc_vo_layout(p.lay, &V) != CDCC_OK) return CDCC_EINVAL;
    if (V.m_size > 0 && (!p.lam || !p.tau || !p.M)) return CDCC_EINVAL;
  }
  return CDCC_OK;
}

int run_partial(int32_t nsys, const cdcc_partial_problem_t *probs, const cdcc_opts_t *popts, void *vstream) {
  cdcc_opts_t opts{};
  if (popts) opts = *popts;
  if (opts.precision != CDCC_FP64) return is_split(opts.precision) ? CDCC_EUNSUPPORTED : CDCC_EINVAL;
  int rc = validate_partial(nsys, probs);
  if (rc != CDCC_OK) return rc;
  if (nsys == 0) return CDCC_OK;
  hipStream_t stream = static_cast<hipStream_t>(vstream);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_mu);
  std::string key = "partial|" + std::to_string(dev) + "|" + std::to_string(nsys);
  for (int s = 0; s < nsys; ++s) {
    const cdcc_sym_t &y = probs[s].lay->sym;
    key += "|" + std::to_string(y.nirrep);
    for (int g = 0; g < y.nirrep; ++g) key += "," + std::to_string(y.nocc[g]) + "," + std::to_string(y.nvir[g]);
  }
  std::shared_ptr<PmPlan> P = g_pmplans.find(key);
  if (!P) {
    P = std::make_shared<PmPlan>();
    rc = build_pm_plan(nsys, probs, *P);
    if (rc != CDCC_OK) return rc;
    g_pmplans.put(key, P);
  }
  int64_t total = align_up(int64_t(nsys) * int64_t(sizeof(PmPtrs)));
  std::vector<int64_t> wofs(nsys);
  for (int s = 0; s < nsys; ++s) {
    wofs[s] = total;
    total = align_up(total + P->ws_elems[s] * 8);
  }
  Workspace *ws = nullptr;
  rc = get_workspace(dev, stream, std::max<int64_t>(total, 256), int64_t(nsys) * int64_t(sizeof(PmPtrs)), ws);
  if (rc != CDCC_OK) return rc;
  char *base = static_cast<char *>(ws->dev);
  if (ws->ev_recorded) HIPCHK(hipEventSynchronize(ws->ev));
  PmPtrs *hp = static_cast<PmPtrs *>(ws->staging);
  for (int s = 0; s < nsys; ++s) {
    PmPtrs q{};
    q.lam = probs[s].lam;
    q.tau = probs[s].tau;
    q.M = probs[s].M;
    q.ws = reinterpret_cast<double *>(base + wofs[s]);
    hp[s] = q;
  }
  PmPtrs *dpp = reinterpret_cast<PmPtrs *>(base);
  HIPCHK(hipMemcpyAsync(dpp, hp, size_t(nsys) * sizeof(PmPtrs), hipMemcpyHostToDevice, stream));
  HIPCHK(hipEventRecord(ws->ev, stream));
  ws->ev_recorded = true;
  {
    Span sp(9, P->nlchunks + P->ntchunks > 0, stream);
    HIPCHK(launch_pm_pack(P->descs, P->lchunks, P->nlchunks, P->tchunks, P->ntchunks, P->kp, P->sqs, dpp, stream));
  }
  {
    Span sp(10, P->ntiles > 0, stream);
    HIPCHK(launch_pm_gemm(P->descs, P->tiles, P->ntiles, P->sqs, dpp, stream));
  }
  P->fence.mark(stream);
  return CDCC_OK;
}

// ===========================================================================
// Two-step Cholesky decomposition (section on the symmetry-adapted two-step
// CD algorithm, Algorithm 1; the second-step equation of the CD/DF section).
// The host drives the macro iterations (qualification from a copy of the
// diagonals, pruning); the device runs the residual columns, the micro
// iterations and the second-step factorisation and solves.
// ===========================================================================
struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  int alloc(size_t bytes) {
    if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return CDCC_ENOMEM;
    }
    return CDCC_OK;
  }
};
struct HostBuf {
  void *p = nullptr;
  ~HostBuf() {
    if (p) (void)hipHostFree(p);
  }
  int alloc(size_t bytes) {
    if (hipHostMalloc(&p, std::max<size_t>(bytes, 256), hipHostMallocDefault) != hipSuccess) {
      p = nullptr;
      return CDCC_ENOMEM;
    }
    return CDCC_OK;
  }
};

int validate_cd_matrix(const cdcc_cd_matrix_t *m) {
  if (!m) return CDCC_EINVAL;
  if (!(m->nirrep == 1 || m->nirrep == 2 || m->nirrep == 4 || m->nirrep == 8))
    return m->nirrep > 0 ? CDCC_EUNSUPPORTED : CDCC_EINVAL;
  for (int g = 0; g < m->nirrep; ++g) {
    if (m->n[g] < 0 || m->n[g] > (int64_t(1) << 30)) return CDCC_EINVAL;
    if (m->n[g] > 0 && !m->V[g]) return CDCC_EINVAL;
  }
  return CDCC_OK;
}

constexpr int kCdChunk = 64;  // micro-iteration launches between host checks

int run_cd_basis(const cdcc_cd_matrix_t *mat, const cdcc_cd_params_t *prm, int64_t *const piv_out[CDCC_MAX_IRREP],
                 int64_t npiv[CDCC_MAX_IRREP], hipStream_t stream) {
  int rc = validate_cd_matrix(mat);
  if (rc != CDCC_OK) return rc;
  if (!prm || !npiv || !piv_out) return CDCC_EINVAL;
  const double tau = prm->tau, sigma = prm->sigma;
  const int qmax = prm->qmax;
  if (!(tau > 0.0) || !(sigma > 0.0 && sigma <= 1.0) || qmax < 1 || qmax > kCdQmaxCap) return CDCC_EINVAL;
  const int h = mat->nirrep;
  for (int g = 0; g < h; ++g)
    if (mat->n[g] > 0 && !piv_out[g]) return CDCC_EINVAL;
  // device buffers: per irrep D, inP, L1 (n x n), M (n x qcap), piv; shared qrows, states, diagonals
  int64_t off[8][6], tot = 0, ntot = 0, nmax = 0;
  CdPtrs P{};
  for (int g = 0; g < h; ++g) {
    const int64_t n = mat->n[g];
    P.n[g] = n;
    P.qcap[g] = int(std::min<int64_t>(qmax, std::max<int64_t>(n, 1)));
    ntot += n;
    nmax = std::max(nmax, n);
    off[g][0] = tot;
    tot = align_up(tot + n * 8);
    off[g][1] = tot;
    tot = align_up(tot + n);
    off[g][2] = tot;
    tot = align_up(tot + n * n * 8);
    off[g][3] = tot;
    tot = align_up(tot + n * P.qcap[g] * 8);
    off[g][4] = tot;
    tot = align_up(tot + n * 4);
    off[g][5] = tot;
    tot = align_up(tot + n * 4);
  }
  const int64_t o_qr = tot;
  tot = align_up(tot + int64_t(qmax) * 4);
  const int64_t o_st = tot;
  tot = align_up(tot + 2 * int64_t(sizeof(CdState)));
  const int64_t o_dq = tot;
  tot = align_up(tot + 2 * int64_t(qmax) * 8);
  DevBuf dev;
  if ((rc = dev.alloc(size_t(tot))) != CDCC_OK) return rc;
  char *base = static_cast<char *>(dev.p);
  for (int g = 0; g < h; ++g) {
    P.D[g] = reinterpret_cast<double *>(base + off[g][0]);
    P.inP[g] = reinterpret_cast<uint8_t *>(base + off[g][1]);
    P.L1[g] = reinterpret_cast<double *>(base + off[g][2]);
    P.M[g] = reinterpret_cast<double *>(base + off[g][3]);
    P.piv[g] = reinterpret_cast<int32_t *>(base + off[g][4]);
    P.qpos[g] = reinterpret_cast<int32_t *>(base + off[g][5]);
  }
  int32_t *dqr = reinterpret_cast<int32_t *>(base + o_qr);
  CdState *dst = reinterpret_cast<CdState *>(base + o_st);  // two states, alternating per step
  double *ddq = reinterpret_cast<double *>(base + o_dq);     // two copies of the qualified diagonals
  // pinned host mirrors
  HostBuf hD, hP, hQ, hQr, hSt, hPos, hDq;
  if ((rc = hD.alloc(size_t(ntot) * 8)) != CDCC_OK) return rc;
  if ((rc = hP.alloc(size_t(ntot))) != CDCC_OK) return rc;
  if ((rc = hQ.alloc(size_t(qmax) * sizeof(CdQ))) != CDCC_OK) return rc;
  if ((rc = hQr.alloc(size_t(qmax) * 4)) != CDCC_OK) return rc;
  if ((rc = hSt.alloc(2 * sizeof(CdState))) != CDCC_OK) return rc;
  if ((rc = hPos.alloc(size_t(ntot) * 4)) != CDCC_OK) return rc;
  if ((rc = hDq.alloc(size_t(qmax) * 8)) != CDCC_OK) return rc;
  double *Dh = static_cast<double *>(hD.p);
  uint8_t *Ph = static_cast<uint8_t *>(hP.p);
  CdQ *Qh = static_cast<CdQ *>(hQ.p);
  int32_t *Qrh = static_cast<int32_t *>(hQr.p);
  CdState *Sh = static_cast<CdState *>(hSt.p);
  int32_t *Posh = static_cast<int32_t *>(hPos.p);
  double *Dqh = static_cast<double *>(hDq.p);
  for (int64_t i = 0; i < ntot; ++i) Posh[i] = -1;
  int64_t goff[9] = {0};
  for (int g = 0; g < h; ++g) goff[g + 1] = goff[g] + mat->n[g];

  auto pull_D = [&]() -> int {
    for (int g = 0; g < h; ++g)
      if (mat->n[g] > 0)
        HIPCHK(hipMemcpyAsync(Dh + goff[g], P.D[g], size_t(mat->n[g]) * 8, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    return CDCC_OK;
  };
  auto push_P = [&]() -> int {
    for (int g = 0; g < h; ++g)
      if (mat->n[g] > 0)
        HIPCHK(hipMemcpyAsync(P.inP[g], Ph + goff[g], size_t(mat->n[g]), hipMemcpyHostToDevice, stream));
    return CDCC_OK;
  };

  int k[8] = {0};
  {
    Span sp(11, ntot > 0, stream);
    for (int g = 0; g < h; ++g) HIPCHK(launch_cd_diag(mat->V[g], mat->n[g], P.D[g], stream));
  }
  if ((rc = pull_D()) != CDCC_OK) return rc;
  for (int64_t i = 0; i < ntot; ++i) Ph[i] = Dh[i] >= tau ? 1 : 0;
  if ((rc = push_P()) != CDCC_OK) return rc;

  std::vector<std::tuple<double, int, int>> cand;
  for (;;) {
    double dmax = -1.0;
    bool any = false;
    for (int g = 0; g < h; ++g)
      for (int64_t r = 0; r < mat->n[g]; ++r)
        if (Ph[goff[g] + r]) {
          any = true;
          dmax = std::max(dmax, Dh[goff[g] + r]);
        }
    if (!any) break;
    // qualified list: the qmax largest diagonals of P that are >= sigma * D_max
    cand.clear();
    for (int g = 0; g < h; ++g)
      for (int64_t r = 0; r < mat->n[g]; ++r)
        if (Ph[goff[g] + r] && Dh[goff[g] + r] >= sigma * dmax) cand.emplace_back(-Dh[goff[g] + r], g, int(r));
    // only the first qmax in (-D, irrep, index) order are kept, in order
    const int nq = int(std::min<size_t>(cand.size(), size_t(qmax)));
    if (cand.size() > size_t(nq)) std::nth_element(cand.begin(), cand.begin() + nq, cand.end());
    std::sort(cand.begin(), cand.begin() + nq);
    int nqg[8] = {0}, qbeg[8] = {0};
    for (int e = 0; e < nq; ++e) ++nqg[std::get<1>(cand[e])];
    for (int g = 1; g < h; ++g) qbeg[g] = qbeg[g - 1] + nqg[g - 1];
    int fill[8] = {0};
    for (int e = 0; e < nq; ++e) {
      const int g = std::get<1>(cand[e]), r = std::get<2>(cand[e]);
      const int slot = fill[g]++;
      Qh[e] = CdQ{g, r, slot, 0};
      Qrh[qbeg[g] + slot] = r;
      Posh[goff[g] + r] = slot;
      Dqh[qbeg[g] + slot] = Dh[goff[g] + r];
    }
    CdQList QL{};
    int maxq = 0;
    for (int g = 0; g < h; ++g) {
      QL.beg[g] = qbeg[g];
      QL.cnt[g] = nqg[g];
      maxq = std::max(maxq, nqg[g]);
    }
    // both state records start equal (k0 and tau_mic stay fixed in both)
    Sh[0] = CdState{};
    for (int g = 0; g < h; ++g) {
      Sh[0].k[g] = k[g];
      Sh[0].k0[g] = k[g];
    }
    Sh[0].tau_mic = std::max(tau, sigma * dmax);
    Sh[1] = Sh[0];
    HIPCHK(hipMemcpyAsync(dqr, Qrh, size_t(nq) * 4, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(dst, Sh, 2 * sizeof(CdState), hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(ddq, Dqh, size_t(nq) * 8, hipMemcpyHostToDevice, stream));
    for (int g = 0; g < h; ++g)
      if (mat->n[g] > 0)
        HIPCHK(hipMemcpyAsync(P.qpos[g], Posh + goff[g], size_t(mat->n[g]) * 4, hipMemcpyHostToDevice, stream));
    {
      Span sp(11, 1, stream);
      CdGemmBatch GB{};
      for (int g = 0; g < h; ++g) {
        if (nqg[g] == 0) continue;
        HIPCHK(launch_cd_gather_cols(mat->V[g], mat->n[g], dqr + qbeg[g], nqg[g], P.M[g], P.qcap[g], stream));
        if (k[g] > 0) {
          CdGemm &G = GB.g[GB.n++];
          G.A = P.L1[g];
          G.B = P.L1[g];
          G.C = P.M[g];
          G.brows = dqr + qbeg[g];
          G.M = int(mat->n[g]);
          G.N = nqg[g];
          G.K = k[g];
          G.lda = G.ldb = int(mat->n[g]);
          G.ldc = P.qcap[g];
          G.alpha = -1.0;
          G.beta = 1.0;
        }
      }
      HIPCHK(launch_cd_gemm_nt(GB, stream));
    }
    int nsteps = 0;
    {
      // micro iterations of all irreps side by side, in chunks; the device
      // ends each irrep (done flags).  One more step than the longest
      // irrep list: the last one marks that irrep done.
      Span sp(12, 1, stream);
      for (int launched = 0; launched <= maxq;) {
        const int c = std::min(kCdChunk, maxq + 1 - launched);
        HIPCHK(launch_cd_micro(dqr, QL, P, nmax, h, dst, ddq, qmax, launched, c, stream));
        launched += c;
        HIPCHK(hipMemcpyAsync(Sh, dst + (launched & 1), sizeof(CdState), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        bool done = true;
        for (int g = 0; g < h; ++g) done = done && Sh->gdone[g] != 0;
        if (done) break;
      }
      for (int g = 0; g < h; ++g) nsteps += Sh->steps[g];
    }
    if ((rc = pull_D()) != CDCC_OK) return rc;
    for (int e = 0; e < nq; ++e) Posh[goff[Qh[e].g] + Qh[e].r] = -1;
    for (int g = 0; g < h; ++g) k[g] = Sh->k[g];
    if (nsteps == 0) return CDCC_EDEVICE;  // cannot happen: the largest qualified diagonal always pivots
    for (int64_t i = 0; i < ntot; ++i)
      if (Ph[i] && !(Dh[i] >= tau)) Ph[i] = 0;
    if ((rc = push_P()) != CDCC_OK) return rc;
  }
  // pivots back to the caller
  std::vector<int32_t> tmp;
  for (int g = 0; g < h; ++g) {
    npiv[g] = k[g];
    if (k[g] == 0) continue;
    tmp.resize(size_t(k[g]));
    HIPCHK(hipMemcpyAsync(tmp.data(), P.piv[g], size_t(k[g]) * 4, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    for (int i = 0; i < k[g]; ++i) piv_out[g][i] = tmp[size_t(i)];
  }
  for (int g = h; g < CDCC_MAX_IRREP; ++g) npiv[g] = 0;
  return CDCC_OK;
}

int run_cd_vectors(const cdcc_cd_matrix_t *mat, const int64_t *const piv[CDCC_MAX_IRREP],
                   const int64_t npiv[CDCC_MAX_IRREP], double *const L[CDCC_MAX_IRREP], hipStream_t stream) {
  int rc = validate_cd_matrix(mat);
  if (rc != CDCC_OK) return rc;
  if (!piv || !npiv || !L) return CDCC_EINVAL;
  const int h = mat->nirrep;
  int64_t tot = 256;
  for (int g = 0; g < h; ++g) {
    const int64_t n = mat->n[g], np = npiv[g];
    if (np < 0 || np > n || (np > 0 && (!piv[g] || !L[g]))) return CDCC_EINVAL;
    for (int64_t i = 0; i < np; ++i)
      if (piv[g][i] < 0 || piv[g][i] >= n) return CDCC_EINVAL;
    tot += align_up(np * np * 8) + align_up(np * 4) + align_up((np + 63) / 64 * 64 * 64 * 8);
  }
  DevBuf dev;
  if ((rc = dev.alloc(size_t(tot))) != CDCC_OK) return rc;
  char *base = static_cast<char *>(dev.p);
  int *bad = reinterpret_cast<int *>(base);
  int64_t o = 256;
  HostBuf hp;
  int64_t maxnp = 0;
  for (int g = 0; g < h; ++g) maxnp = std::max(maxnp, npiv[g]);
  if ((rc = hp.alloc(size_t(std::max<int64_t>(maxnp, 1)) * 4 * h + 16)) != CDCC_OK) return rc;
  int32_t *ph = static_cast<int32_t *>(hp.p);
  HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), stream));
  {
    Span sp(13, 1, stream);
    // per irrep: metric K (np x np), pivot list, inverses of the diagonal blocks
    double *Km[8] = {nullptr}, *Kinv[8] = {nullptr};
    int nps[8] = {0}, nbmax = 0;
    for (int g = 0; g < h; ++g) {
      const int64_t n = mat->n[g];
      const int np = int(npiv[g]);
      nps[g] = np;
      if (np == 0) continue;
      Km[g] = reinterpret_cast<double *>(base + o);
      o += align_up(int64_t(np) * np * 8);
      int32_t *dp = reinterpret_cast<int32_t *>(base + o);
      o += align_up(int64_t(np) * 4);
      Kinv[g] = reinterpret_cast<double *>(base + o);
      o += align_up(int64_t(np + 63) / 64 * 64 * 64 * 8);
      int32_t *hpg = ph + int64_t(g) * maxnp;
      for (int i = 0; i < np; ++i) hpg[i] = int32_t(piv[g][i]);
      HIPCHK(hipMemcpyAsync(dp, hpg, size_t(np) * 4, hipMemcpyHostToDevice, stream));
      HIPCHK(launch_cd_gather_metric(mat->V[g], n, dp, np, Km[g], L[g], stream));
      nbmax = std::max(nbmax, (np + 63) / 64);
    }
    // X K_bb^-T in place for the w <= 64 columns at c0 of X (one tile column,
    // so each workgroup reads its rows before it overwrites them)
    auto block_solve = [](CdGemm &G, double *X, int64_t ldx, int64_t rows, int c0, int w, const double *kinv) {
      G = CdGemm{};
      G.A = X + c0;
      G.B = kinv;
      G.C = X + c0;
      G.M = int(rows);
      G.N = w;
      G.K = w;
      G.lda = int(ldx);
      G.ldb = 64;
      G.ldc = int(ldx);
      G.alpha = 1.0;
      G.beta = 0.0;
    };
    // blocked right-looking Cholesky of every metric, the irreps side by side
    for (int jb = 0; jb < nbmax; ++jb) {
      CdDiagBatch DB{};
      CdGemmBatch PB{}, TB{};
      for (int g = 0; g < h; ++g) {
        const int np = nps[g], j0 = jb * 64;
        if (j0 >= np) continue;
        const int w = std::min(64, np - j0);
        double *kinv = Kinv[g] + int64_t(jb) * 64 * 64;
        DB.K[DB.n] = Km[g];
        DB.Kinv[DB.n] = kinv;
        DB.ld[DB.n] = np;
        DB.j0[DB.n] = j0;
        DB.w[DB.n] = w;
        ++DB.n;
        if (j0 + w < np) {
          block_solve(PB.g[PB.n++], Km[g] + int64_t(j0 + w) * np, np, np - j0 - w, j0, w, kinv);
          CdGemm &G = TB.g[TB.n++];
          G.A = Km[g] + int64_t(j0 + w) * np + j0;
          G.B = G.A;
          G.C = Km[g] + int64_t(j0 + w) * np + j0 + w;
          G.M = G.N = np - j0 - w;
          G.K = w;
          G.lda = G.ldb = G.ldc = np;
          G.alpha = -1.0;
          G.beta = 1.0;
        }
      }
      HIPCHK(launch_cd_potrf_diag(DB, bad, stream));
      HIPCHK(launch_cd_gemm_nt(PB, stream));
      HIPCHK(launch_cd_gemm_nt(TB, stream));
    }
    // Y K^-T by 64-column blocks (Y = V[:, piv] already in L), irreps side by side
    for (int cb = 0; cb < nbmax; ++cb) {
      CdGemmBatch UB{}, SB{};
      for (int g = 0; g < h; ++g) {
        const int np = nps[g], c0 = cb * 64;
        if (c0 >= np) continue;
        const int w = std::min(64, np - c0);
        const int64_t n = mat->n[g];
        if (c0 > 0) {
          CdGemm &G = UB.g[UB.n++];
          G.A = L[g];
          G.B = Km[g] + int64_t(c0) * np;
          G.C = L[g] + c0;
          G.M = int(n);
          G.N = w;
          G.K = c0;
          G.lda = np;
          G.ldb = np;
          G.ldc = np;
          G.alpha = -1.0;
          G.beta = 1.0;
        }
        block_solve(SB.g[SB.n++], L[g], np, n, c0, w, Kinv[g] + int64_t(cb) * 64 * 64);
      }
      HIPCHK(launch_cd_gemm_nt(UB, stream));
      HIPCHK(launch_cd_gemm_nt(SB, stream));
    }
  }
  int hbad = 0;
  HIPCHK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  return hbad ? CDCC_EINVAL : CDCC_OK;
}

}  // namespace

extern "C" int cdcc_cd_basis(const cdcc_cd_matrix_t *mat, const cdcc_cd_params_t *params,
                             int64_t *const piv[CDCC_MAX_IRREP], int64_t npiv[CDCC_MAX_IRREP], void *stream) {
  std::lock_guard<std::mutex> lock(g_mu);
  return run_cd_basis(mat, params, piv, npiv, static_cast<hipStream_t>(stream));
}

extern "C" int cdcc_cd_vectors(const cdcc_cd_matrix_t *mat, const int64_t *const piv[CDCC_MAX_IRREP],
                               const int64_t npiv[CDCC_MAX_IRREP], double *const L[CDCC_MAX_IRREP], void *stream) {
  std::lock_guard<std::mutex> lock(g_mu);
  return run_cd_vectors(mat, piv, npiv, L, static_cast<hipStream_t>(stream));
}

extern "C" int cdcc_partial_contract(int32_t nsys, const cdcc_partial_problem_t *probs, const cdcc_opts_t *opts,
                                     void *stream) {
  return run_partial(nsys, probs, opts, stream);
}

// ===========================================================================
// The T2 ladder on a caller-provided device region (the allocation-free entry
// point in noalloc.hip passes the library's static scratch array).  Region
// layout: [0, kScratchTables) the plan's tables, then the workspace of the
// call (counters, pointer table, (ac|bd) batch, split-K partials, packed
// amplitudes, slices).  The batch cap is lowered until the workspace fits.
// Nothing is allocated: plans keep their tables on the host and copy them
// into the region, with the pointer table, by ordinary asynchronous copies;
// the launches are enqueued directly (no graph).  Every byte the kernels read
// is written in the same call before it is read (the queue counters are
// cleared by a fill kernel), so a region holding an earlier call's data gives
// the same result.
// ===========================================================================
namespace {
constexpr int64_t kScratchTables = int64_t(16) << 20;
PlanCache<Plan> g_scratch_plans(64);

struct ScratchHost {
  std::vector<SysPtrs> sysptrs;  // host source of the pointer table copy
  hipEvent_t ev = nullptr;       // the previous copy out of sysptrs has completed
  bool recorded = false;
};
std::map<int, ScratchHost> g_scratch_host;
}  // namespace

int run_ladder_in_region(int32_t nsys, const cdcc_problem_t *probs, const cdcc_opts_t *popts, void *vstream,
                         void *region, int64_t region_bytes) {
  cdcc_opts_t opts{};
  if (popts) opts = *popts;
  if (opts.precision != CDCC_FP64 && !is_split(opts.precision)) return CDCC_EINVAL;
  if (opts.tile_policy < 0 || opts.tile_policy > 4) return CDCC_EINVAL;
  if (opts.tile_policy == 4 && !is_split(opts.precision)) return CDCC_EINVAL;
  if (opts.contract_kseg < 0 || opts.contract_kseg > (1 << 20)) return CDCC_EINVAL;
  if (!region || region_bytes <= kScratchTables) return CDCC_EINVAL;
  int dressed = 0;
  int rc = validate(nsys, probs, 0, &dressed);
  if (rc != CDCC_OK) return rc;
  hipStream_t stream = static_cast<hipStream_t>(vstream);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_mu);
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0) g_num_cu = ncu;
  }
  char *tables = static_cast<char *>(region);
  const int64_t avail = region_bytes - kScratchTables;
  const std::string key = "region|" + std::to_string(reinterpret_cast<uintptr_t>(region)) + "|" +
                          std::to_string(region_bytes) + "|" + plan_key(dev, nsys, probs, 0, 0, opts, batch_cap(opts));
  std::shared_ptr<Plan> P = g_scratch_plans.find(key);
  if (!P) {
    // the batch cap: the caller's (or the default), lowered until the whole
    // workspace fits the region
    int64_t cap = std::min<int64_t>(batch_cap(opts), avail);
    for (int tries = 0;; ++tries) {
      auto Q = std::make_shared<Plan>();
      rc = build_plan(nsys, probs, 0, 0, opts, cap, *Q, tables);
      if (rc != CDCC_OK) return rc;
      if (int64_t(Q->host_tables.size()) > kScratchTables) return CDCC_ESCRATCH;
      const int64_t total = ws_layout(*Q).total;
      if (total <= avail) {
        P = Q;
        break;
      }
      const int64_t rest = total - Q->xbuf_elems * 8;  // everything but the batch buffer
      if (rest >= avail || tries >= 8 || cap <= (1 << 16)) return CDCC_ESCRATCH;
      cap = std::max<int64_t>(1 << 16, std::min(cap / 2, avail - rest));
    }
    g_scratch_plans.put(key, P);
  }
  const WsLayout W = ws_layout(*P);
  char *base = tables + kScratchTables;
  ScratchHost &H = g_scratch_host[dev];
  if (!H.ev && hipEventCreateWithFlags(&H.ev, hipEventDisableTiming) != hipSuccess) {
    H.ev = nullptr;
    return CDCC_EDEVICE;
  }
  if (H.recorded) HIPCHK(hipEventSynchronize(H.ev));
  H.sysptrs.resize(size_t(nsys));
  for (int s = 0; s < nsys; ++s) {
    const cdcc_problem_t &p = probs[s];
    SysPtrs q{};
    q.opnd = p.B;
    q.X = p.X;
    q.R = p.R;
    q.delta = p.delta;
    q.eps_occ = p.eps_occ;
    q.eps_vir = p.eps_vir;
    q.epair = p.pair_energy;
    q.eamp = p.energy_amps ? p.energy_amps : p.X;
    q.tauhat = reinterpret_cast<double *>(base + W.th[s]);
    q.B = p.B;
    q.slices = reinterpret_cast<unsigned char *>(base + W.sl[s]);
    q.rowscale = reinterpret_cast<double *>(base + W.sc[s]);
    H.sysptrs[size_t(s)] = q;
  }
  SysPtrs *dsp = reinterpret_cast<SysPtrs *>(base + W.sysptrs);
  HIPCHK(hipMemcpyAsync(tables, P->host_tables.data(), P->host_tables.size(), hipMemcpyHostToDevice, stream));
  HIPCHK(hipMemcpyAsync(dsp, H.sysptrs.data(), size_t(nsys) * sizeof(SysPtrs), hipMemcpyHostToDevice, stream));
  HIPCHK(hipEventRecord(H.ev, stream));
  H.recorded = true;
  int *counters = reinterpret_cast<int *>(base + W.counters);
  double *xbuf = reinterpret_cast<double *>(base + W.xbuf);
  double *part = reinterpret_cast<double *>(base + W.part);
  rc = enqueue_sequence(*P, dsp, counters, xbuf, part, stream);
  P->fence.mark(stream);
  return rc;
}

extern "C" int cdcc_tile_key(const cdcc_sym_t *sym, int32_t precision, int32_t lambda, char *buf, int32_t len) {
  if (!sym || !buf || len <= 0) return CDCC_EINVAL;
  if (!valid_sym(*sym)) return sym->nirrep >= 1 && sym->nirrep <= 8 ? CDCC_EUNSUPPORTED : CDCC_EINVAL;
  if (precision != CDCC_FP64 && !is_split(precision)) return CDCC_EINVAL;
  const std::string k = shape_bucket(*sym, precision, lambda ? 1 : 0);
  if (int64_t(k.size()) + 1 > len) return CDCC_EINVAL;
  std::memcpy(buf, k.c_str(), k.size() + 1);
  return CDCC_OK;
}

extern "C" int cdcc_tile_table_reload(const char *path) {
  std::lock_guard<std::mutex> lock(g_mu);
  delete g_tile_table;
  g_tile_table = nullptr;
  g_tile_table_path = path ? path : "";
  return CDCC_OK;
}

extern "C" int cdcc_ladder_t2(int32_t nsys, const cdcc_problem_t *probs, const cdcc_opts_t *opts, void *stream) {
  return run_ladder(nsys, probs, opts, stream, 0);
}

// ===========================================================================
// Dressed operand of the Lambda ladder, built once per Lambda solve
// (Appendix A: t^P_ab = sum_m t_m^a L^P_bm and W_AbEf depend on t1 and the
// Cholesky vectors only, not on lambda).  One dress job per (system, GP, Ga)
// block; the stack has the layout the ladder's FP64 path builds for itself.
// ===========================================================================
namespace {
struct DressPlan {
  void *dtab = nullptr;
  DressJob *jobs = nullptr;
  int2 *rows = nullptr;
  int nrows = 0;
  PlanFence fence;
  ~DressPlan() {
    fence.wait();
    if (dtab) (void)hipFree(dtab);
  }
};
PlanCache<DressPlan> g_dressplans(64);

int build_dress_plan(int nsys, const cdcc_dress_problem_t *probs, DressPlan &P) {
  std::vector<DressJob> jobs;
  std::vector<int2> rows;
  for (int s = 0; s < nsys; ++s) {
    const cdcc_layout_t &L = *probs[s].lay;
    const int h = L.sym.nirrep;
    const int32_t *no = L.sym.nocc, *nv = L.sym.nvir, *nc = L.sym.ncd;
    for (int gP = 0; gP < h; ++gP)
      for (int ga = 0; ga < h; ++ga) {
        const int ge = ga ^ gP;
        if (nc[gP] == 0 || nv[ga] == 0 || nv[ge] == 0) continue;
        DressJob D{};
        D.sys = s;
        D.va = nv[ga];
        D.ve = nv[ge];
        D.np = nc[gP];
        D.om = no[ge];
        D.u_off = 2 * L.b_off[gP][ga];
        D.b_off = L.b_off[gP][ge];
        D.bvo_off = L.bvo_off[gP][ga];
        D.t1_off = L.t1_off[ge];
        const int jid = int(jobs.size());
        jobs.push_back(D);
        for (int ae = 0; ae < nv[ga] * nv[ge]; ++ae) rows.push_back(int2{jid, ae});
      }
  }
  TableBuilder T;
  const int64_t o_j = T.add(jobs), o_r = T.add(rows);
  if (hipMalloc(&P.dtab, std::max<size_t>(T.bytes.size(), 256)) != hipSuccess) return CDCC_ENOMEM;
  if (hipMemcpy(P.dtab, T.bytes.data(), T.bytes.size(), hipMemcpyHostToDevice) != hipSuccess) return CDCC_EDEVICE;
  char *b = static_cast<char *>(P.dtab);
  P.jobs = reinterpret_cast<DressJob *>(b + o_j);
  P.rows = reinterpret_cast<int2 *>(b + o_r);
  P.nrows = int(rows.size());
  return CDCC_OK;
}

int run_dress(int32_t nsys, const cdcc_dress_problem_t *probs, void *vstream) {
  if (nsys < 0 || (nsys > 0 && !probs)) return CDCC_EINVAL;
  for (int s = 0; s < nsys; ++s) {
    const cdcc_dress_problem_t &p = probs[s];
    if (!p.lay || !p.B || !p.Bvo || !p.t1 || !p.U) return CDCC_EINVAL;
    if (!valid_sym(p.lay->sym)) return p.lay->sym.nirrep >= 1 && p.lay->sym.nirrep <= 8 ? CDCC_EUNSUPPORTED : CDCC_EINVAL;
    cdcc_layout_t chk;
    if (cdcc_irrep_layout(&p.lay->sym, &chk) != CDCC_OK) return CDCC_EINVAL;
    if (chk.b_size != p.lay->b_size || chk.bvo_size != p.lay->bvo_size || chk.t1_size != p.lay->t1_size)
      return CDCC_EINVAL;
  }
  if (nsys == 0) return CDCC_OK;
  hipStream_t stream = static_cast<hipStream_t>(vstream);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_mu);
  std::string key = "dress|" + std::to_string(dev) + "|" + std::to_string(nsys);
  for (int s = 0; s < nsys; ++s) {
    const cdcc_sym_t &y = probs[s].lay->sym;
    key += "|" + std::to_string(y.nirrep);
    for (int g = 0; g < y.nirrep; ++g)
      key += "," + std::to_string(y.nocc[g]) + "," + std::to_string(y.nvir[g]) + "," + std::to_string(y.ncd[g]);
  }
  std::shared_ptr<DressPlan> P = g_dressplans.find(key);
  if (!P) {
    P = std::make_shared<DressPlan>();
    const int rc = build_dress_plan(nsys, probs, *P);
    if (rc != CDCC_OK) return rc;
    g_dressplans.put(key, P);
  }
  Workspace *ws = nullptr;
  const int64_t bytes = align_up(int64_t(nsys) * int64_t(sizeof(SysPtrs)));
  int rc = get_workspace(dev, stream, bytes, int64_t(nsys) * int64_t(sizeof(SysPtrs)), ws);
  if (rc != CDCC_OK) return rc;
  if (ws->ev_recorded) HIPCHK(hipEventSynchronize(ws->ev));
  SysPtrs *hs = static_cast<SysPtrs *>(ws->staging);
  for (int s = 0; s < nsys; ++s) {
    SysPtrs q{};
    q.opnd = probs[s].U;  // written by the dress kernel
    q.B = probs[s].B;
    q.Bvo = probs[s].Bvo;
    q.t1 = probs[s].t1;
    hs[s] = q;
  }
  SysPtrs *dsp = static_cast<SysPtrs *>(ws->dev);
  HIPCHK(hipMemcpyAsync(dsp, hs, size_t(nsys) * sizeof(SysPtrs), hipMemcpyHostToDevice, stream));
  HIPCHK(hipEventRecord(ws->ev, stream));
  ws->ev_recorded = true;
  {
    Span sp(0, P->nrows > 0, stream);
    HIPCHK(launch_dress(P->jobs, P->rows, P->nrows, dsp, stream));
  }
  P->fence.mark(stream);
  return CDCC_OK;
}
}  // namespace

extern "C" int cdcc_lambda_dress(int32_t nsys, const cdcc_dress_problem_t *probs, void *stream) {
  return run_dress(nsys, probs, stream);
}

extern "C" int cdcc_ladder_lambda(int32_t nsys, const cdcc_problem_t *probs, const cdcc_opts_t *opts, void *stream) {
  return run_ladder(nsys, probs, opts, stream, 1);
}

extern "C" int cdcc_workspace_bytes(int32_t nsys, const cdcc_problem_t *probs, const cdcc_opts_t *popts,
                                    int32_t lambda, int64_t *bytes) {
  if (!bytes) return CDCC_EINVAL;
  cdcc_opts_t opts{};
  if (popts) opts = *popts;
  int dressed = 0;
  int rc = validate(nsys, probs, lambda, &dressed);
  if (rc != CDCC_OK) return rc;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CDCC_EDEVICE;
  std::lock_guard<std::mutex> lock(g_mu);
  std::shared_ptr<Plan> P;
  rc = get_plan(dev, nsys, probs, lambda, dressed, opts, P);
  if (rc != CDCC_OK) return rc;
  *bytes = ws_layout(*P).total;
  return CDCC_OK;
}

extern "C" int cdcc_timing_enable(int32_t on) {
  std::lock_guard<std::mutex> lock(g_mu);
  g_timing = on != 0;
  return CDCC_OK;
}

extern "C" int cdcc_timing_read(double ms[CDCC_TIMING_CLASSES], int64_t launches[CDCC_TIMING_CLASSES]) {
  if (!ms || !launches) return CDCC_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  for (int k = 0; k < CDCC_TIMING_CLASSES; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  int rc = CDCC_OK;
  for (const TimedSpan &t : g_spans) {
    float e = 0.f;
    if (hipEventSynchronize(t.b) != hipSuccess || hipEventElapsedTime(&e, t.a, t.b) != hipSuccess) rc = CDCC_EDEVICE;
    ms[t.cls] += e;
    launches[t.cls] += t.launches;
    g_event_pool.push_back(t.a);
    g_event_pool.push_back(t.b);
  }
  g_spans.clear();
  return rc;
}

extern "C" int cdcc_vvvv_density(int32_t nsys, const cdcc_density_problem_t *probs, const cdcc_opts_t *opts,
                                 void *stream) {
  return run_density(nsys, probs, opts, stream);
}

extern "C" int cdcc_release(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  delete g_tile_table;  // re-read on the next plan
  g_tile_table = nullptr;
  if (hipDeviceSynchronize() != hipSuccess) return CDCC_EDEVICE;
  g_dplans.clear();
  g_pmplans.clear();
  g_ws.clear();
  g_plans.clear();
  g_dressplans.clear();
  g_scratch_plans.clear();
  for (auto &h : g_scratch_host)
    if (h.second.ev) (void)hipEventDestroy(h.second.ev);
  g_scratch_host.clear();
  for (auto &c : g_capture_streams) (void)hipStreamDestroy(c.second);
  g_capture_streams.clear();
  for (const TimedSpan &t : g_spans) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  g_spans.clear();
  for (hipEvent_t e : g_event_pool) (void)hipEventDestroy(e);
  g_event_pool.clear();
  return CDCC_OK;
}
