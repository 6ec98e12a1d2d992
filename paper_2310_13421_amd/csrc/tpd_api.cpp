// tpd_api.cpp -- C ABI of libtpd: argument validation, sweep scheduling,
// workspaces, plans (graph-capturable execution), timing, and a host replay
// of the device schedule for CPU-side testing of the index algebra.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <atomic>
#include <fstream>
#include <sstream>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/tpd.h"
#include "tpd_internal.h"

namespace {
// roctx range over a scope: the library's passes and entry points appear as
// named host ranges in rocprofv3 --marker-trace (no cost without a tool)
struct TpdRange {
  explicit TpdRange(const char* name) { roctxRangePush(name); }
  ~TpdRange() { roctxRangePop(); }
  TpdRange(const TpdRange&) = delete;
  TpdRange& operator=(const TpdRange&) = delete;
};
}  // namespace

namespace tpd {
// seeded uniform noise in [-1, 1) over `scalars` doubles (f64) or floats
// (tpd_kernels.hip): the in-place autotuners' refill between timed runs
hipError_t launch_fill_noise(void* p, uint64_t scalars, bool f64, uint64_t seed, hipStream_t st);
}  // namespace tpd

using namespace tpd;

namespace {

constexpr int kMaxQubits = 17;  // the largest n of any dtype (see max_qubits)
constexpr int kMaxBatchQubits = 9;

bool log_on() {
  static const bool on = [] {
    const char* e = std::getenv("TPD_LOG");
    return e && e[0] == '1';
  }();
  return on;
}
void logf(const char* fmt, ...) {
  if (!log_on()) return;
  va_list ap;
  va_start(ap, fmt);
  std::fprintf(stderr, "[tpd] ");
  std::vfprintf(stderr, fmt, ap);
  std::fprintf(stderr, "\n");
  va_end(ap);
}

size_t elem_bytes(Dtype dt) { return dt == DT_C128 ? 16 : dt == DT_R32 ? 4 : 8; }  // C64 and R64: 8
// Largest n: the two-sweep schedule covers n <= 17 (a first sweep of 9
// levels); complex128 stops at 16, where one n = 17 matrix would take 256 GiB.
int max_qubits(Dtype dt) { return dt == DT_C128 ? 16 : kMaxQubits; }

const char* dtype_name(Dtype dt) {
  return dt == DT_C128 ? "c128" : dt == DT_C64 ? "c64" : dt == DT_R64 ? "r64" : "r32";
}

// ---------------------------------------------------------------------------
// schedule
// ---------------------------------------------------------------------------
struct Schedule {
  int n = 0;
  Dtype dt = DT_C128;
  bool matrix_layout = false;
  bool in_place = false;
  bool prune = false;
  int nsweep = 0;
  SweepDesc sw[2];
  int n1 = 0, n2 = 0;
  uint64_t bitmap_words = 0;
  // chunked order (general two-sweep schedules): > 0 runs sweep 1 then
  // sweep 2 over 2^chunk_bits first-sweep d-groups at a time, so a chunk's
  // intermediate can still sit in the memory-side cache when sweep 2 reads
  // it; 0: each sweep over the whole matrix
  int chunk_bits = 0;
  // pipelined chunks (with chunk_bits > 0): >= 2 runs sweep 2 of chunk c on
  // a second stream while sweep 1 of chunks c+1 .. c+window-1 runs on the
  // caller's, so the GPU never drains between the launches of a chunk; 0:
  // both sweeps of one chunk, then the next, on the caller's stream
  int chunk_window = 0;
  // Hermitian input, real weights in a separate array (L_CANR): sweep 1 in
  // place in the matrix buffer, the last sweep from it into the weights
  bool real_out = false;
};
constexpr int kMaxWindow = 8;

int single_db(int n) {
  static const int t[9] = {0, 1, 2, 3, 4, 5, 6, 5, 4};
  return t[n];
}

// Tunable choices of a two-sweep schedule: tile width 2^db diagonals,
// 2^r elements per thread, and the grid (0 = one workgroup per tile, k > 0 =
// persistent grid of k workgroups per CU).  None of them changes results:
// every element sees the same operations in the same order.
struct Tuned {
  int db = 0, r = 4, grid = 0;
  int order2 = 0;  // second sweep's tile order (SweepDesc::tile_order)
  int chunk = 0;   // Schedule::chunk_bits
  int window = 0;  // Schedule::chunk_window
};
struct TuneKey {
  int n, dt, matrix, in_place, herm;
  bool operator<(const TuneKey& o) const {
    if (n != o.n) return n < o.n;
    if (dt != o.dt) return dt < o.dt;
    if (matrix != o.matrix) return matrix < o.matrix;
    if (in_place != o.in_place) return in_place < o.in_place;
    return herm < o.herm;
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, Tuned> g_tuned;  // n = -1: batched kernel grid per dtype
bool g_tune_loaded = false;
std::atomic<int> g_cus{0};

// default tile width: runs of 256 B where the second sweep's x bits allow
// Levels of the two sweeps: n1 top levels (sweep 1, rows 2^n2 apart) and n2
// bottom levels (sweep 2, consecutive rows).  n1 = ceil(n/2), except n = 17,
// where the ninth level goes to the sweep of consecutive rows: 9-level tiles
// of 512 rows 2^8 apart ran at about half the bandwidth, 512 consecutive
// rows at the full rate (complex64 n = 17 in place: 143 -> 110 ms).
void split_levels(int n, int* n1, int* n2) {
  *n1 = n == 17 ? 8 : (n + 1) / 2;
  *n2 = n - *n1;
}

int default_db(Dtype dt, int n2) {
  const int want = dt == DT_C128 ? 4 : dt == DT_R32 ? 6 : 5;
  return want < n2 ? want : (n2 > 4 ? n2 : 4);
}

void load_tune_cache();

tpd_status_t make_schedule_with(int n, Dtype dt, unsigned flags, bool in_place, const Tuned* force, Schedule* s) {
  if (n < 0 || n > max_qubits(dt)) return TPD_ERROR_UNSUPPORTED;
  *s = Schedule{};
  s->n = n;
  s->dt = dt;
  s->matrix_layout = (flags & TPD_FLAG_LAYOUT_MATRIX) != 0;
  s->in_place = in_place;
  if (n == 0) return TPD_SUCCESS;
  const int out_l = s->matrix_layout ? L_MAT : L_CAN;
  if (n <= 8) {
    if (in_place && !s->matrix_layout && n > 6) return TPD_ERROR_UNSUPPORTED;
    s->nsweep = 1;
    SweepDesc& w = s->sw[0];
    w.xlo = 0;
    w.xb = n;
    w.db = single_db(n);
    w.in_layout = L_MAT;
    w.out_layout = out_l;
    w.bitmap_mode = 0;
    w.order = 0;
    w.r = 4;
    w.grid = 0;
    w.is_one = true;
    w.herm = 0;
    w.inv = false;
    w.ntiles = (uint64_t)1 << (n - w.db);
    return TPD_SUCCESS;
  }
  if (in_place && !s->matrix_layout) return TPD_ERROR_UNSUPPORTED;
  s->nsweep = 2;
  split_levels(n, &s->n1, &s->n2);
  Tuned t;
  t.db = default_db(dt, s->n2);
  const bool bottom = (flags & TPD_FLAG_ORDER_BOTTOM) != 0;
  if (force) {
    t = *force;
  } else if (!bottom) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) load_tune_cache();
    auto it = g_tuned.find(TuneKey{n, (int)dt, s->matrix_layout ? 1 : 0, in_place ? 1 : 0,
                                   (flags & TPD_FLAG_HERMITIAN) ? 1 : 0});
    if (it != g_tuned.end()) t = it->second;
  }
  // tiles of 2^(levels + db) elements: at most 1024 threads of 16 elements
  // and 128 KiB of LDS (n = 17 has a sweep of 9 levels).  For real float32
  // in the matrix layout without the Hermitian mode each sweep takes the
  // requested width up to its own cap (n = 17: 2^6 in the 8-level sweep, 2^5
  // in the 9-level one; the pruning bits follow the second sweep's
  // d-groups); otherwise both sweeps share one width (MID order, Hermitian
  // representatives, and a split that did not pay in the 8-byte kernels).
  const int max_tile_bits = dt == DT_C128 ? 13 : 14;
  const int cap1 = max_tile_bits - s->n1, cap2 = max_tile_bits - s->n2;
  const bool split_db = dt == DT_R32 && s->matrix_layout && !(flags & TPD_FLAG_HERMITIAN) && s->n1 >= 5;
  int db1 = t.db, db2 = t.db;
  if (split_db) {
    if (!force && db1 > cap1) db1 = cap1;
    if (db2 > cap2) db2 = cap2;
    if (db1 > db2 + 1) db1 = db2 + 1;
  } else if (!force) {
    const int cap = cap1 < cap2 ? cap1 : cap2;
    if (db1 > cap) db1 = db2 = cap;
  }
  if (db2 > s->n2) return TPD_ERROR_INVALID_VALUE;  // MID needs the low db x bits in sweep 2
  const int db = db1;
  // chunks of first-sweep d-groups: at least two chunks; not with the
  // Hermitian mode, whose first sweep enumerates representative tiles over
  // the whole matrix
  if (t.chunk > 0) {
    const bool ok = !(flags & TPD_FLAG_HERMITIAN) && t.chunk < n - db1;
    if (!ok && force) return TPD_ERROR_INVALID_VALUE;
    s->chunk_bits = ok ? t.chunk : 0;
  }
  if (t.window) {
    const bool ok = s->chunk_bits > 0 && t.window >= 2 && t.window <= kMaxWindow;
    if (!ok && force) return TPD_ERROR_INVALID_VALUE;
    s->chunk_window = ok ? t.window : 0;
  }
  s->prune = (flags & TPD_FLAG_NO_PRUNE) == 0;
  const int cus = g_cus > 0 ? (int)g_cus : 256;
  SweepDesc& a = s->sw[0];
  a.xlo = s->n2;
  a.xb = s->n1;
  a.db = db;
  a.in_layout = L_MAT;
  a.out_layout = s->matrix_layout ? L_MAT : L_MID;
  a.bitmap_mode = s->prune ? 1 : 0;
  a.order = 0;
  a.r = t.r;
  a.grid = t.grid > 0 ? t.grid * cus : 0;
  a.is_one = false;
  a.herm = (flags & TPD_FLAG_HERMITIAN) ? 1 : 0;
  a.inv = false;
  // Hermitian: only the tiles holding representatives (herm_first_tile)
  a.ntiles = a.herm ? herm_first_tiles(s->n2, db, n - db) : ((uint64_t)1 << s->n2) << (n - db);
  SweepDesc& b = s->sw[1];
  b.xlo = 0;
  b.xb = s->n2;
  b.db = db2;
  b.in_layout = s->matrix_layout ? L_MAT : L_MID;
  b.out_layout = out_l;
  b.bitmap_mode = s->prune ? 2 : 0;
  b.order = bottom ? 1 : 0;
  b.r = bottom ? 4 : t.r;
  b.grid = a.grid;
  b.is_one = false;
  b.herm = a.herm;
  b.inv = false;
  b.ntiles = ((uint64_t)1 << s->n1) << (n - db2);
  b.tile_order = ((flags & TPD_FLAG_ROTATE_TILES) || t.order2) ? 1 : 0;
  const uint64_t bits = ((uint64_t)1 << s->n1) << (n - db2);
  s->bitmap_words = (bits + 31) / 32;
  for (int i = 0; i < 2; ++i)
    if (!sweep_supported(dt, s->sw[i])) return force ? TPD_ERROR_INVALID_VALUE : TPD_ERROR_INTERNAL;
  return TPD_SUCCESS;
}

tpd_status_t make_schedule(int n, Dtype dt, unsigned flags, bool in_place, Schedule* s) {
  return make_schedule_with(n, dt, flags, in_place, nullptr, s);
}

// Hermitian matrix -> real weights: the in-place Hermitian schedule of the
// matrix layout (its tuned choices), whose last sweep stores into the
// separate real array in canonical order instead of back into the matrix.
constexpr int kRealOutKeyMatrix = 3;  // TuneKey.matrix of the real-weights schedule's entries

tpd_status_t make_real_out_schedule(int n, Dtype dt, unsigned flags, Schedule* s, const Tuned* force = nullptr) {
  if (dt != DT_C128 && dt != DT_C64) return TPD_ERROR_INVALID_VALUE;
  // the real-weights autotuner's choice, else that of the in-place
  // Hermitian mode (make_schedule_with's own lookup)
  Tuned tuned;
  if (!force && n > 8) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) load_tune_cache();
    auto it = g_tuned.find(TuneKey{n, (int)dt, kRealOutKeyMatrix, 1, 1});
    if (it != g_tuned.end()) {
      tuned = it->second;
      force = &tuned;
    }
  }
  tpd_status_t st =
      make_schedule_with(n, dt, flags | TPD_FLAG_HERMITIAN | TPD_FLAG_LAYOUT_MATRIX, true, n > 8 ? force : nullptr, s);
  if (st) return st;
  s->real_out = true;
  s->in_place = false;
  s->matrix_layout = false;
  s->chunk_bits = 0;
  s->chunk_window = 0;
  if (s->nsweep >= 1) {
    SweepDesc& w = s->sw[s->nsweep - 1];
    w.out_layout = L_CANR;
    if (!sweep_supported(dt, w)) return TPD_ERROR_INTERNAL;
  }
  return TPD_SUCCESS;
}

// partial decomposition: the same sweeps, the second one always checking
// its tile bitmap (requests, ANDed with the live tiles when pruning)
tpd_status_t make_partial_schedule(int n, Dtype dt, unsigned flags, bool in_place, const Tuned* force,
                                   Schedule* s) {
  // the narrowest tile width: a d-group holding one requested string costs
  // one tile per row block, so narrower groups read less for sparse requests
  Tuned narrow;
  narrow.db = dt == DT_C128 ? 3 : 4;
  if (!force && n > 8 && !(flags & TPD_FLAG_ORDER_BOTTOM)) force = &narrow;
  tpd_status_t st = make_schedule_with(n, dt, flags, in_place, force, s);
  if (st) return st;
  if (s->nsweep == 2) {
    s->sw[0].bitmap_mode = s->prune ? 1 : 0;
    s->sw[1].bitmap_mode = 2;
  }
  return TPD_SUCCESS;
}

uint64_t group_words_of(const Schedule& s) {
  return s.nsweep == 2 ? ((((uint64_t)1 << (s.n - s.sw[0].db)) + 31) / 32) : 0;
}

// Inverse transform (synthesis A = sum_t w_t sigma^t): the same levels with
// the inverse butterfly.  n <= 8: one sweep CAN|MAT -> MAT.  n >= 9: the low
// n2 levels first (tiles of fixed high rows, reading the canonical order's
// closed 16-run sets, writing 2^db-column runs of A), then the high n1 levels
// in place on A.
tpd_status_t make_synth_schedule(int n, Dtype dt, unsigned flags, bool in_place, Schedule* s) {
  if (n < 0 || n > max_qubits(dt)) return TPD_ERROR_UNSUPPORTED;
  *s = Schedule{};
  s->n = n;
  s->dt = dt;
  s->matrix_layout = (flags & TPD_FLAG_LAYOUT_MATRIX) != 0;
  s->in_place = in_place;
  if (n == 0) return TPD_SUCCESS;
  const int in_l = s->matrix_layout ? L_MAT : L_CAN;
  auto base = [&](SweepDesc& w) {
    w.in_layout = in_l;
    w.out_layout = L_MAT;
    w.bitmap_mode = 0;
    w.order = 0;
    w.r = 4;
    w.grid = 0;
    w.herm = 0;
    w.inv = true;
  };
  if (n <= 8) {
    if (in_place && !s->matrix_layout && n > 6) return TPD_ERROR_UNSUPPORTED;
    s->nsweep = 1;
    SweepDesc& w = s->sw[0];
    base(w);
    w.xlo = 0;
    w.xb = n;
    w.db = single_db(n);
    w.is_one = true;
    w.ntiles = (uint64_t)1 << (n - w.db);
  } else {
    if (in_place && !s->matrix_layout) return TPD_ERROR_UNSUPPORTED;
    s->nsweep = 2;
    split_levels(n, &s->n1, &s->n2);
    const int dd = default_db(dt, s->n2);
    const int db = dd < 5 ? dd : 5;  // the inverse kernels come in tile widths 2^4 and 2^5
    SweepDesc& a = s->sw[0];
    base(a);
    a.xlo = 0;
    a.xb = s->n2;
    a.db = db;
    a.is_one = false;
    a.ntiles = ((uint64_t)1 << s->n1) << (n - db);
    SweepDesc& b = s->sw[1];
    base(b);
    b.in_layout = L_MAT;
    b.xlo = s->n2;
    b.xb = s->n1;
    b.db = db;
    b.is_one = false;
    b.ntiles = ((uint64_t)1 << s->n2) << (n - db);
  }
  for (int i = 0; i < s->nsweep; ++i)
    if (!sweep_supported(dt, s->sw[i])) return TPD_ERROR_INTERNAL;
  return TPD_SUCCESS;
}

// Autotune cache: TPD_AUTOTUNE_CACHE names a text file of lines
//   tpd-tune-v2 <arch> <cus> <dtype> <n> <matrix> <in_place> <hermitian> <db> <r> <grid> [<order2> [<chunk> [<window>]]]
// Unreadable or foreign lines are ignored (the built-in defaults apply).
void load_tune_cache() {
  g_tune_loaded = true;
  const char* path = std::getenv("TPD_AUTOTUNE_CACHE");
  if (!path || !path[0]) return;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string tag, arch;
    int cus, dt, n, mat, inp, herm, db, r, grid, order2 = 0, chunk = 0, window = 0;
    if (!(is >> tag >> arch >> cus >> dt >> n >> mat >> inp >> herm >> db >> r >> grid)) continue;
    if (!(is >> order2)) order2 = 0;  // optional field: the second sweep's tile order
    else if (!(is >> chunk) || chunk < 0 || chunk > 16) chunk = 0;  // optional field: chunked order
    else if (!(is >> window) || window < 0 || window > kMaxWindow) window = 0;  // optional: pipelined chunks
    if (tag != "tpd-tune-v2" || arch != "gfx950") continue;
    if (g_cus > 0 && cus != g_cus) continue;
    if (dt < 0 || dt > 3 || n < -1 || n > kMaxQubits || r != 4 || grid < 0 || grid > 64) continue;
    Tuned t;
    t.db = db;
    t.r = r;
    t.grid = grid;
    t.order2 = order2 ? 1 : 0;
    t.chunk = chunk;
    t.window = window;
    g_tuned[TuneKey{n, dt, mat, inp, herm}] = t;
  }
}

void save_tune_entry(const TuneKey& k, const Tuned& t) {
  const char* path = std::getenv("TPD_AUTOTUNE_CACHE");
  if (!path || !path[0]) return;
  std::ofstream f(path, std::ios::app);
  f << "tpd-tune-v2 gfx950 " << (g_cus > 0 ? (int)g_cus : 0) << " " << k.dt << " " << k.n << " " << k.matrix << " "
    << k.in_place << " " << k.herm << " " << t.db << " " << t.r << " " << t.grid << " " << t.order2 << " "
    << t.chunk << " " << t.window << "\n";
}

const char* layout_name(int l) {
  return l == L_MAT ? "MAT" : (l == L_CAN ? "CAN" : (l == L_CANR ? "CANR" : "MID"));
}

std::string describe(const Schedule& s) {
  char buf[512];
  const size_t eb = elem_bytes(s.dt);
  const uint64_t count = (uint64_t)1 << (2 * s.n);
  std::string j;
  std::snprintf(buf, sizeof buf,
                "{\"n\":%d,\"dtype\":\"%s\",\"layout\":\"%s\",\"in_place\":%s,\"prune\":%s,"
                "\"hermitian\":%s,\"elements\":%llu,\"algorithmic_bytes\":%llu,\"bitmap_words\":%llu,"
                "\"chunk_bits\":%d,\"chunk_window\":%d,\"real_weights\":%s,\"sweeps\":[",
                s.n, dtype_name(s.dt), s.matrix_layout ? "matrix" : "canonical",
                s.in_place ? "true" : "false", s.prune ? "true" : "false",
                (s.nsweep == 2 && s.sw[0].herm) ? "true" : "false", (unsigned long long)count,
                (unsigned long long)(2 * count * eb), (unsigned long long)s.bitmap_words, s.chunk_bits,
                s.chunk_window, s.real_out ? "true" : "false");
  j += buf;
  for (int i = 0; i < s.nsweep; ++i) {
    const SweepDesc& w = s.sw[i];
    const int B = w.xb + w.db;
    int R = w.r > B ? B : w.r;
    if (B - R > 10) R = B - 10;
    std::snprintf(buf, sizeof buf,
                  "%s{\"xlo\":%d,\"xb\":%d,\"db\":%d,\"in\":\"%s\",\"out\":\"%s\",\"bitmap\":\"%s\","
                  "\"order\":%d,\"tile_order\":%d,\"r\":%d,\"grid\":%d,\"tiles\":%llu,\"tile_elems\":%d,"
                  "\"threads\":%d}",
                  i ? "," : "", w.xlo, w.xb, w.db, layout_name(w.in_layout), layout_name(w.out_layout),
                  w.bitmap_mode == 1 ? "set" : (w.bitmap_mode == 2 ? "check" : "none"), w.order, w.tile_order, R,
                  w.grid, (unsigned long long)w.ntiles, 1 << B, 1 << (B - R));
    j += buf;
  }
  j += "]}";
  return j;
}

tpd_status_t copy_out(const std::string& s, char* buf, size_t len) {
  if (!buf || len == 0) return TPD_ERROR_INVALID_VALUE;
  if (s.size() + 1 > len) return TPD_ERROR_INVALID_VALUE;
  std::memcpy(buf, s.c_str(), s.size() + 1);
  return TPD_SUCCESS;
}

// ---------------------------------------------------------------------------
// validation helpers
// ---------------------------------------------------------------------------
// complex dtypes only: the host replays (test aids) cover no real input
tpd_status_t check_dtype_flags_complex(int dtype, unsigned flags) {
  if (dtype == TPD_R64 || dtype == TPD_R32) return TPD_ERROR_UNSUPPORTED;
  if (dtype != TPD_C128 && dtype != TPD_C64) return TPD_ERROR_INVALID_VALUE;
  if (flags & ~TPD_FLAGS_ALL) return TPD_ERROR_INVALID_VALUE;
  return TPD_SUCCESS;
}

// every device entry point: the complex dtypes and the real input
tpd_status_t check_dtype_flags(int dtype, unsigned flags) {
  if (dtype == TPD_R64 || dtype == TPD_R32) return (flags & ~TPD_FLAGS_ALL) ? TPD_ERROR_INVALID_VALUE : TPD_SUCCESS;
  return check_dtype_flags_complex(dtype, flags);
}

tpd_status_t check_buffers(const void* A, void* C, int n, Dtype dt) {
  if (!A || !C) return TPD_ERROR_INVALID_VALUE;
  const size_t eb = elem_bytes(dt);
  if (((uintptr_t)A % eb) || ((uintptr_t)C % eb)) return TPD_ERROR_INVALID_VALUE;
  if (A != C) {
    const uint64_t bytes = ((uint64_t)1 << (2 * n)) * eb;
    const uintptr_t a0 = (uintptr_t)A, c0 = (uintptr_t)C;
    if (a0 < c0 + bytes && c0 < a0 + bytes) return TPD_ERROR_INVALID_VALUE;
  }
  return TPD_SUCCESS;
}

// ---------------------------------------------------------------------------
// device checks and workspaces
// ---------------------------------------------------------------------------
std::mutex g_mu;
std::map<int, int> g_dev_ok;  // device -> 1 gfx950, 0 not

tpd_status_t current_device(int* dev) {
  int d = -1;
  if (hipGetDevice(&d) != hipSuccess || d < 0) return TPD_ERROR_NO_DEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_dev_ok.find(d);
  if (it == g_dev_ok.end()) {
    hipDeviceProp_t p;
    int ok = 0;
    if (hipGetDeviceProperties(&p, d) == hipSuccess) {
      ok = std::strncmp(p.gcnArchName, "gfx950", 6) == 0;
      if (ok) g_cus = p.multiProcessorCount;
    }
    it = g_dev_ok.emplace(d, ok).first;
    logf("device %d arch ok=%d", d, ok);
  }
  if (!it->second) return TPD_ERROR_NO_DEVICE;
  *dev = d;
  return TPD_SUCCESS;
}

bool fail_alloc_hook() {
  const char* e = std::getenv("TPD_TEST_FAIL_ALLOC");
  return e && e[0] == '1';
}

tpd_status_t dev_alloc(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return TPD_SUCCESS;
  if (fail_alloc_hook()) return TPD_ERROR_OUT_OF_MEMORY;
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return TPD_ERROR_OUT_OF_MEMORY;
  }
  return TPD_SUCCESS;
}

// Second stream and events of the pipelined chunk order (created on first
// use, kept for the owner's lifetime; the stream has the default priority).
struct Pipe {
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  hipEvent_t s1[kMaxWindow + 1] = {}, s2[kMaxWindow + 1] = {};
  tpd_status_t ensure() {
    if (side) return TPD_SUCCESS;
    if (fail_alloc_hook()) return TPD_ERROR_OUT_OF_MEMORY;
    bool ok = hipStreamCreateWithFlags(&side, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&fork, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&join, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i <= kMaxWindow && ok; ++i)
      ok = hipEventCreateWithFlags(&s1[i], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&s2[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      destroy();
      return TPD_ERROR_OUT_OF_MEMORY;
    }
    return TPD_SUCCESS;
  }
  void destroy() {
    if (side) (void)hipStreamSynchronize(side);
    for (hipEvent_t* e : {&fork, &join})
      if (*e) (void)hipEventDestroy(*e), *e = nullptr;
    for (int i = 0; i <= kMaxWindow; ++i) {
      if (s1[i]) (void)hipEventDestroy(s1[i]), s1[i] = nullptr;
      if (s2[i]) (void)hipEventDestroy(s2[i]), s2[i] = nullptr;
    }
    if (side) (void)hipStreamDestroy(side), side = nullptr;
  }
};

struct Workspace {
  uint32_t* bitmap = nullptr;
  uint64_t bitmap_words = 0;
  uint32_t* req = nullptr;  // partial decomposition: d-group bits, then second-sweep tile bits
  uint64_t req_words = 0;
  uint32_t* lists = nullptr;  // partial decomposition: 2 counts (padded), d-group list, tile list
  uint64_t list_words = 0;
  void* sel = nullptr;  // compaction: per-chunk counts and offsets, total
  size_t sel_bytes = 0;
  unsigned long long* counter = nullptr;
  void* table = nullptr;  // batched tables (perm, items, pointer arrays)
  size_t table_bytes = 0;
  void* host_table = nullptr;  // pinned staging copy of the table
  size_t host_bytes = 0;
  hipEvent_t staged = nullptr;  // recorded after the last staging copy
  Pipe pipe;                    // pipelined chunk order
};
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

tpd_status_t ensure_bitmap(Workspace& w, uint64_t words) {
  if (w.bitmap_words >= words) return TPD_SUCCESS;
  if (w.bitmap) (void)hipFree(w.bitmap);
  w.bitmap = nullptr;
  w.bitmap_words = 0;
  void* p;
  tpd_status_t st = dev_alloc(&p, words * 4);
  if (st) return st;
  w.bitmap = (uint32_t*)p;
  w.bitmap_words = words;
  return TPD_SUCCESS;
}

tpd_status_t ensure_words(uint32_t** p, uint64_t* have, uint64_t words) {
  if (*have >= words) return TPD_SUCCESS;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *have = 0;
  void* q;
  tpd_status_t st = dev_alloc(&q, words * 4);
  if (st) return st;
  *p = (uint32_t*)q;
  *have = words;
  return TPD_SUCCESS;
}

tpd_status_t ensure_sel(Workspace& w, size_t bytes) {
  if (w.sel_bytes >= bytes) return TPD_SUCCESS;
  if (w.sel) (void)hipFree(w.sel);
  w.sel = nullptr;
  w.sel_bytes = 0;
  tpd_status_t st = dev_alloc(&w.sel, bytes);
  if (st) return st;
  w.sel_bytes = bytes;
  return TPD_SUCCESS;
}

// device table plus a pinned host staging buffer; the staging buffer is
// only rewritten after the previous copy out of it has completed.
tpd_status_t ensure_table(Workspace& w, size_t bytes) {
  if (!w.staged && hipEventCreateWithFlags(&w.staged, hipEventDisableTiming) != hipSuccess) {
    w.staged = nullptr;
    return TPD_ERROR_OUT_OF_MEMORY;
  }
  if (w.host_table && hipEventSynchronize(w.staged) != hipSuccess) return TPD_ERROR_LAUNCH;
  if (w.table_bytes < bytes) {
    if (w.table) (void)hipFree(w.table);
    w.table = nullptr;
    w.table_bytes = 0;
    tpd_status_t st = dev_alloc(&w.table, bytes);
    if (st) return st;
    w.table_bytes = bytes;
  }
  if (w.host_bytes < bytes) {
    if (w.host_table) (void)hipHostFree(w.host_table);
    w.host_table = nullptr;
    w.host_bytes = 0;
    if (fail_alloc_hook() || hipHostMalloc(&w.host_table, bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      w.host_table = nullptr;
      return TPD_ERROR_OUT_OF_MEMORY;
    }
    w.host_bytes = bytes;
  }
  return TPD_SUCCESS;
}

// ---------------------------------------------------------------------------
// timing (plans with TPD_FLAG_TIMING)
// ---------------------------------------------------------------------------
constexpr int kMaxKernels = 3;
constexpr int kEventPool = 256;
struct Timing {
  bool on = false;
  int nk = 0;
  std::vector<hipEvent_t> ev;  // [k][slot][2]
  int used[kMaxKernels] = {0, 0, 0};
  double ms[kMaxKernels] = {0, 0, 0};
  uint64_t cnt[kMaxKernels] = {0, 0, 0};
  hipEvent_t& at(int k, int slot, int which) { return ev[((size_t)k * kEventPool + slot) * 2 + which]; }
  tpd_status_t create(int nkern) {
    nk = nkern;
    ev.assign((size_t)kMaxKernels * kEventPool * 2, nullptr);
    for (auto& e : ev)
      if (hipEventCreate(&e) != hipSuccess) return TPD_ERROR_OUT_OF_MEMORY;
    on = true;
    return TPD_SUCCESS;
  }
  void destroy() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    ev.clear();
  }
  void drain(int k) {
    for (int s = 0; s < used[k]; ++s) {
      float t = 0;
      if (hipEventSynchronize(at(k, s, 1)) == hipSuccess &&
          hipEventElapsedTime(&t, at(k, s, 0), at(k, s, 1)) == hipSuccess) {
        ms[k] += t;
        cnt[k] += 1;
      }
    }
    used[k] = 0;
  }
  int begin(int k, hipStream_t st) {
    if (!on) return -1;
    if (used[k] == kEventPool) drain(k);
    const int s = used[k]++;
    (void)hipEventRecord(at(k, s, 0), st);
    return s;
  }
  void end(int k, int s, hipStream_t st) {
    if (s >= 0) (void)hipEventRecord(at(k, s, 1), st);
  }
};

// ---------------------------------------------------------------------------
// single-matrix execution
// ---------------------------------------------------------------------------
tpd_status_t launch_sweep_io(const Schedule& s, int i, const void* in, void* out, uint32_t* bitmap,
                             const uint32_t* req, hipStream_t st, int64_t chunk = -1) {
  TpdRange range_("tpd sweep");
  const SweepDesc& w = s.sw[i];
  SweepArgs a{};
  a.in = in;
  a.out = out;
  a.n = s.n;
  a.xlo = w.xlo;
  a.db = w.db;
  a.nfix_d = s.n - w.db;
  a.bitmap = bitmap;
  a.bitmap_mode = w.bitmap_mode;
  a.bm_xbits = s.n1;
  a.bm_db = s.nsweep == 2 ? s.sw[1].db : w.db;
  a.herm = w.herm;
  a.req = req;
  a.ntiles = w.ntiles;
  a.tile_order = w.tile_order;
  if (chunk >= 0) {
    // chunk `chunk` of 2^chunk_bits first-sweep d-groups; in d-groups of
    // this sweep's width (the second sweep's may be half as wide)
    a.chunk_bits = s.chunk_bits + s.sw[0].db - w.db;
    a.td_base = (uint64_t)chunk << a.chunk_bits;
    a.ntiles = ((uint64_t)1 << (s.n - w.xb)) << a.chunk_bits;
  }
  const hipError_t e = launch_sweep(s.dt, w, a, st);
  if (e != hipSuccess) {
    logf("sweep %d launch failed: %s", i, hipGetErrorString(e));
    return TPD_ERROR_LAUNCH;
  }
  return TPD_SUCCESS;
}

// sweep i of a schedule that reads A, then works in C
tpd_status_t launch_sweep_i(const Schedule& s, int i, const void* A, void* C, uint32_t* bitmap,
                            const uint32_t* req, hipStream_t st, int64_t chunk = -1) {
  return launch_sweep_io(s, i, i == 0 ? A : C, C, bitmap, req, st, chunk);
}

// Hermitian matrix -> real weights (make_real_out_schedule): the first sweep
// in place in A, the last from A into W; n = 0 copies the real part.
tpd_status_t run_real_out(const Schedule& s, void* A, void* W, uint32_t* bitmap, hipStream_t st, Timing* tm) {
  TpdRange range_("tpd decompose hermitian real");
  const size_t eb = elem_bytes(s.dt);
  if (s.n == 0)
    return hipMemcpyAsync(W, A, eb / 2, hipMemcpyDeviceToDevice, st) == hipSuccess ? TPD_SUCCESS : TPD_ERROR_LAUNCH;
  if (s.prune && s.nsweep == 2 && launch_fill_u32(bitmap, s.bitmap_words, 0u, st) != hipSuccess)
    return TPD_ERROR_LAUNCH;
  for (int i = 0; i < s.nsweep; ++i) {
    const bool last = i == s.nsweep - 1;
    const int slot = tm ? tm->begin(i, st) : -1;
    const tpd_status_t e = launch_sweep_io(s, i, A, last ? W : A, bitmap, nullptr, st);
    if (tm) tm->end(i, slot, st);
    if (e) return e;
  }
  return TPD_SUCCESS;
}

// Pipelined chunk order: sweep 1 of every chunk on the caller's stream,
// sweep 2 of chunk c on the pipe's stream after sweep 1 of chunk c, and
// sweep 1 of chunk c only after sweep 2 of chunk c - window (so at most
// `window` chunks are between their two sweeps).  Chunks touch disjoint
// elements (every tile lies in one d-group), so the two streams' launches
// may overlap in any way these dependencies allow.  The caller's stream
// waits for the last sweep 2 before anything queued after this call.
tpd_status_t run_pipelined(const Schedule& s, const void* A, void* C, uint32_t* bitmap, hipStream_t st,
                           Pipe& p) {
  TpdRange range_("tpd pipelined chunks");
  const uint64_t nchunks = (uint64_t)1 << (s.n - s.sw[0].db - s.chunk_bits);
  const uint64_t W = (uint64_t)s.chunk_window, K = W + 1;
  if (hipEventRecord(p.fork, st) != hipSuccess || hipStreamWaitEvent(p.side, p.fork, 0) != hipSuccess)
    return TPD_ERROR_LAUNCH;
  tpd_status_t e = TPD_SUCCESS;
  for (uint64_t c = 0; c < nchunks && !e; ++c) {
    if (c >= W && hipStreamWaitEvent(st, p.s2[(c - W) % K], 0) != hipSuccess) e = TPD_ERROR_LAUNCH;
    if (!e) e = launch_sweep_i(s, 0, A, C, bitmap, nullptr, st, (int64_t)c);
    if (!e && (hipEventRecord(p.s1[c % K], st) != hipSuccess ||
               hipStreamWaitEvent(p.side, p.s1[c % K], 0) != hipSuccess))
      e = TPD_ERROR_LAUNCH;
    if (!e) e = launch_sweep_i(s, 1, A, C, bitmap, nullptr, p.side, (int64_t)c);
    if (!e && hipEventRecord(p.s2[c % K], p.side) != hipSuccess) e = TPD_ERROR_LAUNCH;
  }
  // join even after a failed launch: nothing queued on the caller's stream
  // later may overtake what the pipe's stream still runs
  if (hipEventRecord(p.join, p.side) != hipSuccess || hipStreamWaitEvent(st, p.join, 0) != hipSuccess)
    return TPD_ERROR_LAUNCH;
  return e;
}

tpd_status_t run_schedule(const Schedule& s, const void* A, void* C, uint32_t* bitmap, hipStream_t st,
                          Timing* tm, Pipe* pipe = nullptr) {
  TpdRange range_("tpd decompose");
  const size_t eb = elem_bytes(s.dt);
  if (s.n == 0) {
    if (A != C && hipMemcpyAsync(C, A, eb, hipMemcpyDeviceToDevice, st) != hipSuccess) return TPD_ERROR_LAUNCH;
    return TPD_SUCCESS;
  }
  if (s.prune && s.nsweep == 2) {
    if (launch_fill_u32(bitmap, s.bitmap_words, 0u, st) != hipSuccess) return TPD_ERROR_LAUNCH;
  }
  if (s.nsweep == 2 && s.chunk_bits > 0) {
    // sweep 1 then sweep 2 over one chunk of d-groups at a time (the
    // sweeps' tiles never cross a d-group, so each chunk is closed); timing
    // records the whole loop as kernel 0
    // (a schedule with a chunk window runs pipelined when the caller passes
    // a pipe; without one, chunk after chunk on one stream)
    const uint64_t nchunks = (uint64_t)1 << (s.n - s.sw[0].db - s.chunk_bits);
    const int slot = tm ? tm->begin(0, st) : -1;
    tpd_status_t e = TPD_SUCCESS;
    if (s.chunk_window >= 2 && pipe) {
      e = run_pipelined(s, A, C, bitmap, st, *pipe);
    } else {
      for (uint64_t c = 0; c < nchunks && !e; ++c)
        for (int i = 0; i < 2 && !e; ++i) e = launch_sweep_i(s, i, A, C, bitmap, nullptr, st, (int64_t)c);
    }
    if (tm) tm->end(0, slot, st);
    return e;
  }
  for (int i = 0; i < s.nsweep; ++i) {
    const int slot = tm ? tm->begin(i, st) : -1;
    const tpd_status_t e = launch_sweep_i(s, i, A, C, bitmap, nullptr, st);
    if (tm) tm->end(i, slot, st);
    if (e) return e;
  }
  return TPD_SUCCESS;
}

// Partial decomposition (the paper's Algorithm 3 at tile granularity): the
// d-groups of the first sweep that hold a requested string, and the
// second-sweep tiles that hold one (and, with pruning, are live), become
// device work lists; each sweep then runs a persistent grid over its list
// only, so the launch costs nothing for the groups and tiles left out.  The
// requested weights are then gathered.  n <= 8: the whole single sweep,
// then the gather.  Hermitian first sweeps keep their own tile enumeration
// and skip unrequested d-groups by the bitmap (in a persistent grid too).
struct PartialLists {
  uint32_t* counts;  // [0]: d-groups, [1]: second-sweep tiles
  uint32_t* groups;  // list of d-groups
  uint32_t* tiles;   // list of second-sweep tiles
};

tpd_status_t run_partial(const Schedule& s, const void* A, void* C, const uint64_t* req, uint64_t count,
                         void* values, uint32_t* live, uint32_t* groups, uint64_t group_words, uint32_t* tiles,
                         const PartialLists& pl, hipStream_t st) {
  TpdRange range_("tpd decompose partial");
  if (s.nsweep == 2) {
    const int cus = g_cus > 0 ? (int)g_cus : 256;
    if (launch_fill_u32(groups, group_words + s.bitmap_words, 0u, st) != hipSuccess) return TPD_ERROR_LAUNCH;
    if (launch_fill_u32(pl.counts, 2, 0u, st) != hipSuccess) return TPD_ERROR_LAUNCH;
    if (launch_mark_requests(req, count, s.n, s.n1, s.sw[0].db, s.sw[1].db, groups, tiles, st) != hipSuccess)
      return TPD_ERROR_LAUNCH;
    const bool group_list = !s.sw[0].herm;
    if (group_list && launch_bits_to_list(groups, group_words, pl.groups, &pl.counts[0], st) != hipSuccess)
      return TPD_ERROR_LAUNCH;
    if (s.prune && launch_fill_u32(live, s.bitmap_words, 0u, st) != hipSuccess) return TPD_ERROR_LAUNCH;
    for (int i = 0; i < 2; ++i) {
      SweepDesc w = s.sw[i];
      if (w.grid <= 0) w.grid = 2 * cus;  // persistent over the work list
      SweepArgs a{};
      a.in = i == 0 ? A : C;
      a.out = C;
      a.n = s.n;
      a.xlo = w.xlo;
      a.db = w.db;
      a.nfix_d = s.n - w.db;
      a.bm_xbits = s.n1;
      a.bm_db = s.sw[1].db;
      a.herm = w.herm;
      if (i == 0) {
        a.bitmap = live;
        a.bitmap_mode = w.bitmap_mode;  // sets the live bits when pruning
        if (group_list) {
          a.list = pl.groups;
          a.list_count = &pl.counts[0];
          a.list_shift = w.xlo;  // the first sweep fixes the low n2 x bits
        } else {
          a.req = groups;
        }
      } else {
        // Hermitian mode: requested zero tiles stay in the list and the
        // kernel stores their mirrored rows, which the first sweep never
        // wrote; otherwise the list holds requested and live tiles only
        const bool herm_zero = s.prune && w.herm;
        if (s.prune && !herm_zero && launch_and_u32(tiles, live, s.bitmap_words, st) != hipSuccess)
          return TPD_ERROR_LAUNCH;
        if (launch_bits_to_list(tiles, s.bitmap_words, pl.tiles, &pl.counts[1], st) != hipSuccess)
          return TPD_ERROR_LAUNCH;
        a.bitmap = herm_zero ? live : nullptr;
        a.bitmap_mode = herm_zero ? 2 : 0;
        a.list = pl.tiles;
        a.list_count = &pl.counts[1];
        a.list_shift = 0;
      }
      a.ntiles = w.ntiles;
      const hipError_t e = launch_sweep(s.dt, w, a, st);
      if (e != hipSuccess) {
        logf("partial sweep %d launch failed: %s", i, hipGetErrorString(e));
        return TPD_ERROR_LAUNCH;
      }
    }
  } else {
    tpd_status_t e = run_schedule(s, A, C, nullptr, st, nullptr);
    if (e) return e;
  }
  if (launch_gather(s.dt, C, s.n, s.matrix_layout, req, count, values, st) != hipSuccess) return TPD_ERROR_LAUNCH;
  return TPD_SUCCESS;
}

// ---------------------------------------------------------------------------
// batched work tables
// ---------------------------------------------------------------------------
struct BatchTables {
  std::vector<uint32_t> perm;  // position -> caller's matrix index
  std::vector<BatchItem> items;
  std::vector<BatchSeg> segs;  // runs of one shape, in item order
};

// per-n shape codes of the batched kernel (see BatchSeg): the tuner's
// choice for (dtype, n) if any, else 0 (full tile, prefetch)
constexpr int kBatchedKeyMatrix = 2;  // TuneKey.matrix of per-n batched entries
void batch_codes(Dtype dt, int codes[kMaxBatchQubits + 1]) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (!g_tune_loaded) load_tune_cache();
  for (int n = 0; n <= kMaxBatchQubits; ++n) {
    codes[n] = 0;
    auto it = g_tuned.find(TuneKey{n, (int)dt, kBatchedKeyMatrix, 0, 0});
    if (it != g_tuned.end() && batch_code_ok(n, it->second.db)) codes[n] = it->second.db;
  }
}

tpd_status_t check_batch_ns(const int* ns, int count, bool in_place, unsigned flags) {
  const bool matrix_layout = (flags & TPD_FLAG_LAYOUT_MATRIX) != 0;
  for (int i = 0; i < count; ++i) {
    if (ns[i] < 0 || ns[i] > kMaxBatchQubits) return TPD_ERROR_UNSUPPORTED;
    if (in_place && !matrix_layout && ns[i] > 6) return TPD_ERROR_UNSUPPORTED;
  }
  return TPD_SUCCESS;
}

// Work table: matrices sorted largest n first (stable), each n's matrices
// cut into items of that n's geometry; `only` >= 0 keeps the matrices of
// that n alone (the per-n tuner).  codes == null: the tuned/default codes.
tpd_status_t build_batch(const int* ns, int count, bool in_place, unsigned flags, Dtype dt, BatchTables* bt,
                         const int* codes = nullptr, int only = -1) {
  tpd_status_t st = check_batch_ns(ns, count, in_place, flags);
  if (st) return st;
  int def[kMaxBatchQubits + 1];
  if (!codes) {
    batch_codes(dt, def);
    codes = def;
  }
  bt->perm.clear();
  for (int i = 0; i < count; ++i)
    if (only < 0 || ns[i] == only) bt->perm.push_back((uint32_t)i);
  // largest first, stable within a size
  std::stable_sort(bt->perm.begin(), bt->perm.end(), [&](uint32_t a, uint32_t b) { return ns[a] > ns[b]; });
  bt->items.clear();
  bt->segs.clear();
  const int m_all = (int)bt->perm.size();
  int pos = 0;
  while (pos < m_all) {
    const int n = ns[bt->perm[pos]];
    int end = pos;
    while (end < m_all && ns[bt->perm[end]] == n) ++end;
    const int code = batch_code_ok(n, codes[n]) ? codes[n] : 0;
    const int v = batch_code_variant(code);
    const BatchGeom g = batch_geom(n, batch_tile_bits(dt), v);
    BatchSeg sg{};
    sg.first = (uint32_t)bt->items.size();
    sg.shape = (uint32_t)(n * kBatchCodes + code);
    if (g.mb > 0) {
      const int per = 1 << g.mb;
      for (int m = pos; m < end; m += per) {
        BatchItem it{};
        it.mat0 = (uint32_t)m;
        it.n = (uint16_t)n;
        it.nmat = (uint16_t)std::min(per, end - m);
        it.tile = 0;
        it.variant = (uint32_t)v;
        bt->items.push_back(it);
      }
    } else {
      const uint32_t tiles = 1u << (n - g.db);
      for (int m = pos; m < end; ++m)
        for (uint32_t t = 0; t < tiles; ++t) {
          BatchItem it{};
          it.mat0 = (uint32_t)m;
          it.n = (uint16_t)n;
          it.nmat = 1;
          it.tile = t;
          it.variant = (uint32_t)v;
          bt->items.push_back(it);
        }
    }
    sg.end = (uint32_t)bt->items.size();
    bt->segs.push_back(sg);
    pos = end;
  }
  return TPD_SUCCESS;
}

// a batched work table on the device (plans and the tuner); grows as needed
struct DevBatch {
  uint32_t* perm = nullptr;
  BatchItem* items = nullptr;
  BatchSeg* segs = nullptr;
  size_t perm_cap = 0, items_cap = 0, segs_cap = 0;
  uint32_t nitems = 0, nseg = 0;

  template <class T>
  static tpd_status_t put(T** dst, size_t* cap, const std::vector<T>& src) {
    if (src.size() > *cap) {
      if (*dst) (void)hipFree(*dst);
      *dst = nullptr;
      *cap = 0;
      void* mem = nullptr;
      tpd_status_t st = dev_alloc(&mem, sizeof(T) * src.size());
      if (st) return st;
      *dst = (T*)mem;
      *cap = src.size();
    }
    if (!src.empty() && hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice) != hipSuccess)
      return TPD_ERROR_LAUNCH;
    return TPD_SUCCESS;
  }
  tpd_status_t upload(const BatchTables& bt) {
    tpd_status_t st = put(&perm, &perm_cap, bt.perm);
    if (!st) st = put(&items, &items_cap, bt.items);
    if (!st) st = put(&segs, &segs_cap, bt.segs);
    nitems = st ? 0 : (uint32_t)bt.items.size();
    nseg = st ? 0 : (uint32_t)bt.segs.size();
    return st;
  }
  void release() {
    if (perm) (void)hipFree(perm);
    if (items) (void)hipFree(items);
    if (segs) (void)hipFree(segs);
    *this = DevBatch{};
  }
};

int batched_grid(Dtype dt, uint32_t nitems) {
  const int cus = g_cus > 0 ? (int)g_cus : 256;
  int per_cu = 2;  // LDS-limited residency of the item loop (64 KiB tile per workgroup)
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) load_tune_cache();
    auto it = g_tuned.find(TuneKey{-1, (int)dt, 0, 0, 0});
    if (it != g_tuned.end()) per_cu = it->second.grid;  // 0: one workgroup per item
  }
  if (per_cu <= 0) return (int)nitems;
  const int g = cus * per_cu;
  return (uint32_t)g > nitems ? (int)nitems : g;
}

}  // namespace

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
struct tpd_plan_s {
  bool batched = false;
  int device = 0;
  Dtype dt = DT_C128;
  unsigned flags = 0;
  bool in_place = false;
  Schedule sched;
  uint32_t* bitmap = nullptr;
  unsigned long long* counter = nullptr;
  // batched
  int count = 0;
  int grid = 0;
  std::vector<int> ns;                // qubit counts in the caller's order
  int codes[kMaxBatchQubits + 1] = {};  // per-n shape codes of the table
  DevBatch tab;
  Timing timing;
  Pipe pipe;  // pipelined chunk order (schedules with a chunk window)
};

// tpd_decompose_hermitian_real, optionally with a forced tile width and grid
// arguments of tpd_decompose_hermitian_real
tpd_status_t check_hermitian_real(void* A, int n, void* weights, tpd_dtype_t dtype, unsigned flags) {
  if (dtype != TPD_C128 && dtype != TPD_C64) return TPD_ERROR_INVALID_VALUE;
  if (flags & ~TPD_FLAG_NO_PRUNE) return TPD_ERROR_INVALID_VALUE;
  if (n < 0 || n > max_qubits((Dtype)dtype)) return TPD_ERROR_UNSUPPORTED;
  if (!A || !weights) return TPD_ERROR_INVALID_VALUE;
  const size_t eb = elem_bytes((Dtype)dtype);
  if (((uintptr_t)A % eb) || ((uintptr_t)weights % (eb / 2))) return TPD_ERROR_INVALID_VALUE;
  const uint64_t count = (uint64_t)1 << (2 * n);
  const uintptr_t a0 = (uintptr_t)A, w0 = (uintptr_t)weights;
  if (a0 < w0 + count * (eb / 2) && w0 < a0 + count * eb) return TPD_ERROR_INVALID_VALUE;
  return TPD_SUCCESS;
}

tpd_status_t hermitian_real(void* A, int n, void* weights, tpd_dtype_t dtype, unsigned flags, const Tuned* force,
                            tpd_stream_t stream) {
  tpd_status_t st0 = check_hermitian_real(A, n, weights, dtype, flags);
  if (st0) return st0;
  const Dtype dt = (Dtype)dtype;
  Schedule s;
  tpd_status_t st = make_real_out_schedule(n, dt, flags, &s, force);
  if (st) return st;
  int dev;
  st = current_device(&dev);
  if (st) return st;
  hipStream_t hs = (hipStream_t)stream;
  uint32_t* bm = nullptr;
  // held until the kernels are enqueued (see tpd_decompose_ex)
  std::unique_lock<std::mutex> lk(g_mu, std::defer_lock);
  if (s.prune && s.nsweep == 2) {
    lk.lock();
    Workspace& w = g_ws[{dev, hs}];
    st = ensure_bitmap(w, s.bitmap_words);
    if (st) return st;
    bm = w.bitmap;
  }
  logf("decompose hermitian real n=%d %s", n, describe(s).c_str());
  return run_real_out(s, A, weights, bm, hs, nullptr);
}

extern "C" {

int tpd_max_qubits(tpd_dtype_t dtype) {
  if (dtype != TPD_C128 && dtype != TPD_C64 && dtype != TPD_R64 && dtype != TPD_R32) return -1;
  return max_qubits((Dtype)dtype);
}

const char* tpd_status_string(tpd_status_t s) {
  switch (s) {
    case TPD_SUCCESS: return "TPD_SUCCESS";
    case TPD_ERROR_INVALID_VALUE: return "TPD_ERROR_INVALID_VALUE";
    case TPD_ERROR_UNSUPPORTED: return "TPD_ERROR_UNSUPPORTED";
    case TPD_ERROR_OUT_OF_MEMORY: return "TPD_ERROR_OUT_OF_MEMORY";
    case TPD_ERROR_LAUNCH: return "TPD_ERROR_LAUNCH";
    case TPD_ERROR_INTERNAL: return "TPD_ERROR_INTERNAL";
    case TPD_ERROR_NO_DEVICE: return "TPD_ERROR_NO_DEVICE";
  }
  return "TPD_ERROR_UNKNOWN";
}

uint64_t tpd_index_from_string(const char* s) {
  if (!s || !s[0]) return UINT64_MAX;
  uint64_t q = 0;
  int len = 0;
  for (const char* p = s; *p; ++p) {
    int t;
    switch (*p) {
      case 'I': t = 0; break;
      case 'X': t = 1; break;
      case 'Y': t = 2; break;
      case 'Z': t = 3; break;
      default: return UINT64_MAX;
    }
    if (++len > 32) return UINT64_MAX;
    q = q * 4 + (uint64_t)t;
  }
  return q;
}

int tpd_string_from_index(uint64_t q, int n, char* buf, size_t len) {
  if (!buf || n < 0 || n > 32 || len < (size_t)n + 1) return 1;
  if (n < 32 && (q >> (2 * n)) != 0) return 1;
  for (int k = 1; k <= n; ++k) buf[k - 1] = "IXYZ"[(q >> (2 * (n - k))) & 3u];
  buf[n] = 0;
  return 0;
}

tpd_status_t tpd_schedule_describe(int n, tpd_dtype_t dtype, unsigned flags, int in_place, char* buf, size_t len) {
  tpd_status_t st = check_dtype_flags(dtype, flags);
  if (st) return st;
  Schedule s;
  st = make_schedule(n, (Dtype)dtype, flags, in_place != 0, &s);
  if (st) return st;
  return copy_out(describe(s), buf, len);
}

tpd_status_t tpd_decompose_ex(const void* A, int n, void* coeffs, tpd_dtype_t dtype, unsigned flags,
                              tpd_stream_t stream) {
  tpd_status_t st = check_dtype_flags(dtype, flags);
  if (st) return st;
  if (n < 0 || n > max_qubits((Dtype)dtype)) return TPD_ERROR_UNSUPPORTED;
  const Dtype dt = (Dtype)dtype;
  st = check_buffers(A, coeffs, n, dt);
  if (st) return st;
  Schedule s;
  st = make_schedule(n, dt, flags, A == coeffs, &s);
  if (st) return st;
  int dev;
  st = current_device(&dev);
  if (st) return st;
  hipStream_t hs = (hipStream_t)stream;
  uint32_t* bm = nullptr;
  // the lock is held until the kernels are enqueued: another thread on the
  // same stream could otherwise grow (free and reallocate) the workspace
  // between this thread taking its pointer and launching on it
  std::unique_lock<std::mutex> lk(g_mu, std::defer_lock);
  Pipe* pipe = nullptr;
  if ((s.prune && s.nsweep == 2) || s.chunk_window) {
    lk.lock();
    Workspace& w = g_ws[{dev, hs}];
    if (s.prune && s.nsweep == 2) {
      st = ensure_bitmap(w, s.bitmap_words);
      if (st) return st;
      bm = w.bitmap;
    }
    if (s.chunk_window) {
      st = w.pipe.ensure();
      if (st) return st;
      pipe = &w.pipe;
    }
  }
  logf("decompose n=%d %s", n, describe(s).c_str());
  return run_schedule(s, A, coeffs, bm, hs, nullptr, pipe);
}

tpd_status_t tpd_decompose_hermitian_real(void* A, int n, void* weights, tpd_dtype_t dtype, unsigned flags,
                                          tpd_stream_t stream) {
  return hermitian_real(A, n, weights, dtype, flags, nullptr, stream);
}

tpd_status_t tpd_synthesize_ex(const void* coeffs, int n, void* A, tpd_dtype_t dtype, unsigned flags,
                               tpd_stream_t stream) {
  tpd_status_t st = check_dtype_flags(dtype, flags);
  if (st) return st;
  if (flags & ~(TPD_FLAG_LAYOUT_MATRIX | TPD_FLAG_NO_PRUNE)) return TPD_ERROR_INVALID_VALUE;
  if (n < 0 || n > max_qubits((Dtype)dtype)) return TPD_ERROR_UNSUPPORTED;
  const Dtype dt = (Dtype)dtype;
  st = check_buffers(coeffs, A, n, dt);
  if (st) return st;
  Schedule s;
  st = make_synth_schedule(n, dt, flags, coeffs == A, &s);
  if (st) return st;
  int dev;
  st = current_device(&dev);
  if (st) return st;
  return run_schedule(s, coeffs, A, nullptr, (hipStream_t)stream, nullptr);
}

tpd_status_t tpd_decompose_partial(const void* A, int n, void* coeffs, const uint64_t* req, uint64_t count,
                                   void* values, tpd_dtype_t dtype, unsigned flags, tpd_stream_t stream) {
  tpd_status_t st = check_dtype_flags(dtype, flags);
  if (st) return st;
  if (flags & TPD_FLAG_TIMING) return TPD_ERROR_INVALID_VALUE;
  if (n < 0 || n > max_qubits((Dtype)dtype)) return TPD_ERROR_UNSUPPORTED;
  const Dtype dt = (Dtype)dtype;
  st = check_buffers(A, coeffs, n, dt);
  if (st) return st;
  if (count > 0 && (!req || !values)) return TPD_ERROR_INVALID_VALUE;
  if (((uintptr_t)req % 8) || ((uintptr_t)values % elem_bytes(dt))) return TPD_ERROR_INVALID_VALUE;
  Schedule s;
  st = make_partial_schedule(n, dt, flags, A == coeffs, nullptr, &s);
  if (st) return st;
  if (count == 0) return TPD_SUCCESS;
  int dev;
  st = current_device(&dev);
  if (st) return st;
  hipStream_t hs = (hipStream_t)stream;
  uint32_t *live = nullptr, *groups = nullptr, *tiles = nullptr;
  PartialLists pl{nullptr, nullptr, nullptr};
  const uint64_t gw = group_words_of(s);
  if (n == 0) {
    if (A != coeffs && hipMemcpyAsync(coeffs, A, elem_bytes(dt), hipMemcpyDeviceToDevice, hs) != hipSuccess)
      return TPD_ERROR_LAUNCH;
    return launch_gather(dt, coeffs, 0, s.matrix_layout, req, count, values, hs) == hipSuccess ? TPD_SUCCESS
                                                                                              : TPD_ERROR_LAUNCH;
  }
  std::unique_lock<std::mutex> lk(g_mu, std::defer_lock);  // held until the kernels are enqueued
  if (s.nsweep == 2) {
    lk.lock();
    Workspace& w = g_ws[{dev, hs}];
    if (s.prune) {
      st = ensure_bitmap(w, s.bitmap_words);
      if (st) return st;
      live = w.bitmap;
    }
    st = ensure_words(&w.req, &w.req_words, gw + s.bitmap_words);
    if (st) return st;
    groups = w.req;
    tiles = w.req + gw;
    st = ensure_words(&w.lists, &w.list_words, 64 + 32 * (gw + s.bitmap_words));
    if (st) return st;
    pl.counts = w.lists;
    pl.groups = w.lists + 64;
    pl.tiles = w.lists + 64 + 32 * gw;
  }
  logf("decompose_partial n=%d count=%llu %s", n, (unsigned long long)count, describe(s).c_str());
  return run_partial(s, A, coeffs, req, count, values, live, groups, gw, tiles, pl, hs);
}

tpd_status_t tpd_compact(const void* coeffs, int n, tpd_dtype_t dtype, unsigned flags, double tol, uint64_t* q_out,
                         void* w_out, uint64_t capacity, uint64_t* count, tpd_stream_t stream) {
  TpdRange range_("tpd compact");
  tpd_status_t st = check_dtype_flags(dtype, flags);
  if (st) return st;
  if (flags & ~TPD_FLAG_LAYOUT_MATRIX) return TPD_ERROR_INVALID_VALUE;
  if (n < 0 || n > max_qubits((Dtype)dtype)) return TPD_ERROR_UNSUPPORTED;
  const Dtype dt = (Dtype)dtype;
  if (!coeffs || !count || ((uintptr_t)coeffs % elem_bytes(dt)) || ((uintptr_t)count % 8))
    return TPD_ERROR_INVALID_VALUE;
  if (!(tol >= 0.0)) return TPD_ERROR_INVALID_VALUE;  // negative or NaN
  if (capacity > 0 && (!q_out || !w_out || ((uintptr_t)q_out % 8) || ((uintptr_t)w_out % elem_bytes(dt))))
    return TPD_ERROR_INVALID_VALUE;
  int dev;
  st = current_device(&dev);
  if (st) return st;
  hipStream_t hs = (hipStream_t)stream;
  const uint64_t elems = (uint64_t)1 << (2 * n);
  const uint64_t nchunks = (elems + kCompactChunk - 1) / kCompactChunk;
  uint32_t* counts;
  uint64_t* offsets;
  std::lock_guard<std::mutex> lk(g_mu);  // held until the kernels are enqueued
  {
    Workspace& w = g_ws[{dev, hs}];
    const size_t cbytes = ((nchunks * 4 + 255) / 256) * 256;
    st = ensure_sel(w, cbytes + nchunks * 8);
    if (st) return st;
    counts = (uint32_t*)w.sel;
    offsets = (uint64_t*)((char*)w.sel + cbytes);
  }
  const bool mat = (flags & TPD_FLAG_LAYOUT_MATRIX) != 0;
  if (launch_compact_count(dt, coeffs, elems, tol, counts, hs) != hipSuccess) return TPD_ERROR_LAUNCH;
  if (launch_compact_scan(counts, nchunks, offsets, count, hs) != hipSuccess) return TPD_ERROR_LAUNCH;
  if (launch_compact_write(dt, coeffs, n, mat, tol, counts, offsets, capacity, q_out, w_out, hs) != hipSuccess)
    return TPD_ERROR_LAUNCH;
  return TPD_SUCCESS;
}

tpd_status_t tpd_decompose(const void* A, int n, void* coeffs, tpd_stream_t stream) {
  return tpd_decompose_ex(A, n, coeffs, TPD_C128, 0u, stream);
}

tpd_status_t tpd_decompose_noalloc(const void* A, int n, void* coeffs, tpd_dtype_t dtype, unsigned flags,
                                   tpd_stream_t stream) {
  tpd_status_t st = check_dtype_flags(dtype, flags);
  if (st) return st;
  if (flags & TPD_FLAG_TIMING) return TPD_ERROR_INVALID_VALUE;
  if (n < 0 || n > max_qubits((Dtype)dtype)) return TPD_ERROR_UNSUPPORTED;
  const Dtype dt = (Dtype)dtype;
  st = check_buffers(A, coeffs, n, dt);
  if (st) return st;
  Schedule s;
  st = make_schedule(n, dt, flags, A == coeffs, &s);
  if (st) return st;
  if (s.bitmap_words > kNoallocScratchWords) return TPD_ERROR_UNSUPPORTED;  // never for a schedule of this library
  int dev;
  st = current_device(&dev);
  if (st) return st;
  uint32_t* bm = nullptr;
  if (s.prune && s.nsweep == 2) {
    // the device's copy of the static scratch array (tpd_scratch.hip),
    // cleared by run_schedule's fill kernel
    if (noalloc_scratch(dev, &bm) != hipSuccess) return TPD_ERROR_LAUNCH;
  }
  return run_schedule(s, A, coeffs, bm, (hipStream_t)stream, nullptr);
}

tpd_status_t tpd_release_workspace(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_ws) {
    Workspace& w = kv.second;
    if (w.staged) (void)hipEventSynchronize(w.staged);
    if (w.bitmap) (void)hipFree(w.bitmap);
    if (w.req) (void)hipFree(w.req);
    if (w.lists) (void)hipFree(w.lists);
    if (w.sel) (void)hipFree(w.sel);
    if (w.counter) (void)hipFree(w.counter);
    if (w.table) (void)hipFree(w.table);
    if (w.host_table) (void)hipHostFree(w.host_table);
    if (w.staged) (void)hipEventDestroy(w.staged);
    w.pipe.destroy();
  }
  g_ws.clear();
  return TPD_SUCCESS;
}

tpd_status_t tpd_plan_create(int n, tpd_dtype_t dtype, unsigned flags, int in_place, tpd_plan_t* plan) {
  if (!plan) return TPD_ERROR_INVALID_VALUE;
  *plan = nullptr;
  tpd_status_t st = check_dtype_flags(dtype, flags);
  if (st) return st;
  Schedule s;
  st = make_schedule(n, (Dtype)dtype, flags, in_place != 0, &s);
  if (st) return st;
  int dev;
  st = current_device(&dev);
  if (st) return st;
  tpd_plan_s* p = new (std::nothrow) tpd_plan_s();
  if (!p) return TPD_ERROR_OUT_OF_MEMORY;
  p->device = dev;
  p->dt = (Dtype)dtype;
  p->flags = flags;
  p->in_place = in_place != 0;
  p->sched = s;
  void* mem = nullptr;
  st = dev_alloc(&mem, (size_t)s.bitmap_words * 4);
  if (!st) {
    p->bitmap = (uint32_t*)mem;
    st = dev_alloc(&mem, sizeof(unsigned long long) * 2);
    p->counter = (unsigned long long*)mem;
  }
  if (!st && (flags & TPD_FLAG_TIMING)) st = p->timing.create(kMaxKernels);
  if (!st && s.chunk_window) st = p->pipe.ensure();
  if (st) {
    tpd_plan_destroy(p);
    return st;
  }
  *plan = p;
  return TPD_SUCCESS;
}

tpd_status_t tpd_plan_create_batched(const int* ns, int count, tpd_dtype_t dtype, unsigned flags, int in_place,
                                     tpd_plan_t* plan) {
  if (!plan) return TPD_ERROR_INVALID_VALUE;
  *plan = nullptr;
  tpd_status_t st = check_dtype_flags(dtype, flags);
  if (st) return st;
  if (count < 0 || (count > 0 && !ns)) return TPD_ERROR_INVALID_VALUE;
  int codes[kMaxBatchQubits + 1];
  batch_codes((Dtype)dtype, codes);
  BatchTables bt;
  st = build_batch(ns, count, in_place != 0, flags, (Dtype)dtype, &bt, codes);
  if (st) return st;
  int dev;
  st = current_device(&dev);
  if (st) return st;
  tpd_plan_s* p = new (std::nothrow) tpd_plan_s();
  if (!p) return TPD_ERROR_OUT_OF_MEMORY;
  p->batched = true;
  p->device = dev;
  p->dt = (Dtype)dtype;
  p->flags = flags;
  p->in_place = in_place != 0;
  p->count = count;
  p->ns.assign(ns, ns + count);
  std::memcpy(p->codes, codes, sizeof codes);
  p->grid = batched_grid(p->dt, (uint32_t)bt.items.size());
  st = p->tab.upload(bt);
  if (!st && (flags & TPD_FLAG_TIMING)) st = p->timing.create(kMaxKernels);
  if (st) {
    tpd_plan_destroy(p);
    return st;
  }
  *plan = p;
  return TPD_SUCCESS;
}

tpd_status_t tpd_plan_execute(tpd_plan_t plan, const void* A, void* coeffs, tpd_stream_t stream) {
  if (!plan || plan->batched) return TPD_ERROR_INVALID_VALUE;
  tpd_status_t st = check_buffers(A, coeffs, plan->sched.n, plan->dt);
  if (st) return st;
  if ((A == coeffs) != plan->in_place) return TPD_ERROR_INVALID_VALUE;
  return run_schedule(plan->sched, A, coeffs, plan->bitmap, (hipStream_t)stream,
                      plan->timing.on ? &plan->timing : nullptr, &plan->pipe);
}

tpd_status_t tpd_plan_execute_batched(tpd_plan_t plan, const void* const* d_ptrs, void* const* d_out_ptrs,
                                      tpd_stream_t stream) {
  TpdRange range_("tpd batched");
  if (!plan || !plan->batched) return TPD_ERROR_INVALID_VALUE;
  if (plan->count == 0) return TPD_SUCCESS;
  if (!d_ptrs) return TPD_ERROR_INVALID_VALUE;
  if (!d_out_ptrs && !plan->in_place) return TPD_ERROR_INVALID_VALUE;
  hipStream_t hs = (hipStream_t)stream;
  const int slot = plan->timing.on ? plan->timing.begin(0, hs) : -1;
  const hipError_t e =
      launch_batched_perm(plan->dt, d_ptrs, d_out_ptrs ? d_out_ptrs : (void* const*)d_ptrs, plan->tab.perm,
                          plan->tab.items, plan->tab.nitems, plan->tab.segs, plan->tab.nseg,
                          (plan->flags & TPD_FLAG_LAYOUT_MATRIX) ? L_MAT : L_CAN, plan->grid, hs);
  if (plan->timing.on) plan->timing.end(0, slot, hs);
  return e == hipSuccess ? TPD_SUCCESS : TPD_ERROR_LAUNCH;
}

tpd_status_t tpd_plan_destroy(tpd_plan_t plan) {
  if (!plan) return TPD_ERROR_INVALID_VALUE;
  if (plan->bitmap) (void)hipFree(plan->bitmap);
  if (plan->counter) (void)hipFree(plan->counter);
  plan->tab.release();
  plan->timing.destroy();
  plan->pipe.destroy();
  delete plan;
  return TPD_SUCCESS;
}

int tpd_plan_num_kernels(tpd_plan_t plan) {
  if (!plan) return -1;
  return plan->batched ? 1 : plan->sched.nsweep;
}

tpd_status_t tpd_plan_timing(tpd_plan_t plan, double* ms, uint64_t* counts, int reset) {
  if (!plan || !ms || !counts) return TPD_ERROR_INVALID_VALUE;
  if (!plan->timing.on) return TPD_ERROR_UNSUPPORTED;
  const int nk = tpd_plan_num_kernels(plan);
  for (int k = 0; k < nk; ++k) {
    plan->timing.drain(k);
    ms[k] = plan->timing.ms[k];
    counts[k] = plan->timing.cnt[k];
    if (reset) {
      plan->timing.ms[k] = 0;
      plan->timing.cnt[k] = 0;
    }
  }
  return TPD_SUCCESS;
}

tpd_status_t tpd_plan_prune_stats(tpd_plan_t plan, uint64_t* live_tiles, uint64_t* total_tiles,
                                  uint64_t* live_prefixes, int* prefix_level, tpd_stream_t stream) {
  if (!plan || plan->batched || !live_tiles || !total_tiles || !live_prefixes || !prefix_level)
    return TPD_ERROR_INVALID_VALUE;
  const Schedule& s = plan->sched;
  if (!s.prune || s.nsweep != 2) return TPD_ERROR_UNSUPPORTED;
  hipStream_t hs = (hipStream_t)stream;
  if (hipMemsetAsync(plan->counter, 0, sizeof(unsigned long long), hs) != hipSuccess) return TPD_ERROR_LAUNCH;
  if (launch_popcount(plan->bitmap, s.bitmap_words, plan->counter, hs) != hipSuccess) return TPD_ERROR_LAUNCH;
  unsigned long long c = 0;
  if (hipMemcpyAsync(&c, plan->counter, sizeof c, hipMemcpyDeviceToHost, hs) != hipSuccess) return TPD_ERROR_LAUNCH;
  std::vector<uint32_t> words(s.bitmap_words);
  if (hipMemcpyAsync(words.data(), plan->bitmap, 4 * s.bitmap_words, hipMemcpyDeviceToHost, hs) != hipSuccess)
    return TPD_ERROR_LAUNCH;
  if (hipStreamSynchronize(hs) != hipSuccess) return TPD_ERROR_LAUNCH;
  *live_tiles = c;
  *total_tiles = s.sw[1].ntiles;
  // a level-n1 CMW is the set of tiles sharing x_hi and the top n1 d bits;
  // bit index = (td << n1) | x_hi, td = d >> db2 (the bitmap has one bit per
  // second-sweep tile, whose width may differ from the first sweep's)
  const int db = s.sw[1].db;
  const int lowd = s.n2 - db;  // d bits [db, n2) vary inside one CMW
  std::vector<uint8_t> live(((size_t)1 << (2 * s.n1)), 0);
  const uint64_t nb = s.sw[1].ntiles;
  for (uint64_t b = 0; b < nb; ++b) {
    if (!((words[b >> 5] >> (b & 31)) & 1u)) continue;
    const uint64_t xhi = b & (((uint64_t)1 << s.n1) - 1);
    const uint64_t td = b >> s.n1;
    const uint64_t dhi = td >> lowd;
    live[(size_t)((xhi << s.n1) | dhi)] = 1;
  }
  uint64_t lp = 0;
  for (uint8_t v : live) lp += v;
  *live_prefixes = lp;
  *prefix_level = s.n1;
  return TPD_SUCCESS;
}

tpd_status_t tpd_plan_describe(tpd_plan_t plan, char* buf, size_t len) {
  if (!plan) return TPD_ERROR_INVALID_VALUE;
  if (!plan->batched) return copy_out(describe(plan->sched), buf, len);
  // per n present: the shape code (0: full tile with prefetch, 1: full tile
  // without, 2: half tile with prefetch) and its geometry
  std::string j;
  char tmp[256];
  std::snprintf(tmp, sizeof tmp,
                "{\"batched\":true,\"count\":%d,\"items\":%u,\"segments\":%u,\"grid\":%d,\"dtype\":\"%s\","
                "\"tile_bits\":%d,\"threads\":%d,\"per_n\":[",
                plan->count, plan->tab.nitems, plan->tab.nseg, plan->grid, dtype_name(plan->dt),
                batch_tile_bits(plan->dt), 1 << (batch_tile_bits(plan->dt) - 4));
  j += tmp;
  bool first = true;
  for (int n = kMaxBatchQubits; n >= 0; --n) {
    if (std::find(plan->ns.begin(), plan->ns.end(), n) == plan->ns.end()) continue;
    const int code = plan->codes[n];
    const BatchGeom g = batch_geom(n, batch_tile_bits(plan->dt), batch_code_variant(code));
    std::snprintf(tmp, sizeof tmp,
                  "%s{\"n\":%d,\"code\":%d,\"prefetch\":%s,\"variant\":%d,\"db\":%d,\"matrices_per_item\":%d,"
                  "\"elements_per_thread\":%d}",
                  first ? "" : ",", n, code, batch_code_prefetch(code) ? "true" : "false", batch_code_variant(code),
                  g.db, 1 << g.mb, 1 << g.r);
    j += tmp;
    first = false;
  }
  j += "]}";
  return copy_out(j, buf, len);
}

tpd_status_t tpd_decompose_batched(const void* const* ptrs, const int* ns, int count, void* const* out_ptrs,
                                   tpd_dtype_t dtype, unsigned flags, tpd_stream_t stream) {
  TpdRange range_("tpd batched");
  tpd_status_t st = check_dtype_flags(dtype, flags);
  if (st) return st;
  if (count < 0) return TPD_ERROR_INVALID_VALUE;
  if (count == 0) return TPD_SUCCESS;
  if (!ptrs || !ns) return TPD_ERROR_INVALID_VALUE;
  const Dtype dt = (Dtype)dtype;
  const bool in_place = out_ptrs == nullptr;
  BatchTables bt;
  st = build_batch(ns, count, in_place, flags, dt, &bt);
  if (st) return st;
  for (int i = 0; i < count; ++i) {
    void* o = in_place ? (void*)ptrs[i] : out_ptrs[i];
    st = check_buffers(ptrs[i], o, ns[i], dt);
    if (st) return st;
  }
  int dev;
  st = current_device(&dev);
  if (st) return st;
  hipStream_t hs = (hipStream_t)stream;
  // table: perm[count] | pad | items[nitems] | segs[nseg] | in ptrs[count] | out ptrs[count]
  const size_t off_items = ((sizeof(uint32_t) * (size_t)count + 15) / 16) * 16;
  const size_t off_segs = off_items + sizeof(BatchItem) * bt.items.size();
  const size_t off_in = off_segs + sizeof(BatchSeg) * bt.segs.size();
  const size_t off_out = off_in + sizeof(void*) * (size_t)count;
  const size_t total = off_out + sizeof(void*) * (size_t)count;
  unsigned char* dtab = nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  Workspace& w = g_ws[{dev, hs}];
  st = ensure_table(w, total);
  if (st) return st;
  dtab = (unsigned char*)w.table;
  unsigned char* host = (unsigned char*)w.host_table;
  std::memcpy(host, bt.perm.data(), sizeof(uint32_t) * (size_t)count);
  std::memcpy(host + off_items, bt.items.data(), sizeof(BatchItem) * bt.items.size());
  std::memcpy(host + off_segs, bt.segs.data(), sizeof(BatchSeg) * bt.segs.size());
  std::memcpy(host + off_in, ptrs, sizeof(void*) * (size_t)count);
  std::memcpy(host + off_out, in_place ? (const void*)ptrs : (const void*)out_ptrs, sizeof(void*) * (size_t)count);
  if (hipMemcpyAsync(dtab, host, total, hipMemcpyHostToDevice, hs) != hipSuccess) return TPD_ERROR_LAUNCH;
  if (hipEventRecord(w.staged, hs) != hipSuccess) return TPD_ERROR_LAUNCH;
  const hipError_t e =
      launch_batched_perm(dt, (const void* const*)(dtab + off_in), (void* const*)(dtab + off_out),
                          (const uint32_t*)dtab, (const BatchItem*)(dtab + off_items), (uint32_t)bt.items.size(),
                          (const BatchSeg*)(dtab + off_segs), (uint32_t)bt.segs.size(),
                          (flags & TPD_FLAG_LAYOUT_MATRIX) ? L_MAT : L_CAN, batched_grid(dt, (uint32_t)bt.items.size()),
                          hs);
  return e == hipSuccess ? TPD_SUCCESS : TPD_ERROR_LAUNCH;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// host-side schedule access for the emulator (tpd_emulate.cpp)
// ---------------------------------------------------------------------------
namespace tpd {
tpd_status_t host_schedule(int n, int dtype, unsigned flags, bool in_place, const int* tune, SweepDesc* sw,
                           int* nsweep, int* n1, uint64_t* bitmap_words, int* chunk_bits, int* chunk_window) {
  tpd_status_t st = check_dtype_flags_complex(dtype, flags);
  if (st) return st;
  Schedule s;
  Tuned t;
  if (tune) {
    t.db = tune[0];
    t.r = tune[1];
    t.grid = tune[2];
    t.chunk = tune[3];
    t.window = tune[4];
  }
  st = make_schedule_with(n, (Dtype)dtype, flags, in_place, tune && n > 8 ? &t : nullptr, &s);
  if (st) return st;
  for (int i = 0; i < s.nsweep; ++i) sw[i] = s.sw[i];
  *nsweep = s.nsweep;
  *n1 = s.n1;
  *bitmap_words = s.bitmap_words;
  *chunk_bits = s.chunk_bits;
  *chunk_window = s.chunk_window;
  return TPD_SUCCESS;
}

tpd_status_t host_real_out_schedule(int n, int dtype, unsigned flags, SweepDesc* sw, int* nsweep, int* n1,
                                    uint64_t* bitmap_words, int* prune) {
  if (dtype != TPD_C128 && dtype != TPD_C64) return TPD_ERROR_INVALID_VALUE;
  if (flags & ~TPD_FLAG_NO_PRUNE) return TPD_ERROR_INVALID_VALUE;
  Schedule s;
  tpd_status_t st = make_real_out_schedule(n, (Dtype)dtype, flags, &s);
  if (st) return st;
  for (int i = 0; i < s.nsweep; ++i) sw[i] = s.sw[i];
  *nsweep = s.nsweep;
  *n1 = s.n1;
  *bitmap_words = s.bitmap_words;
  *prune = s.prune ? 1 : 0;
  return TPD_SUCCESS;
}

tpd_status_t host_partial_schedule(int n, int dtype, unsigned flags, bool in_place, SweepDesc* sw, int* nsweep,
                                   int* n1, uint64_t* bitmap_words, int* prune) {
  tpd_status_t st = check_dtype_flags_complex(dtype, flags);
  if (st) return st;
  if (flags & TPD_FLAG_TIMING) return TPD_ERROR_INVALID_VALUE;
  Schedule s;
  st = make_partial_schedule(n, (Dtype)dtype, flags, in_place, nullptr, &s);
  if (st) return st;
  for (int i = 0; i < s.nsweep; ++i) sw[i] = s.sw[i];
  *nsweep = s.nsweep;
  *n1 = s.n1;
  *bitmap_words = s.bitmap_words;
  *prune = s.prune ? 1 : 0;
  return TPD_SUCCESS;
}

tpd_status_t host_synth_schedule(int n, int dtype, unsigned flags, bool in_place, SweepDesc* sw, int* nsweep) {
  tpd_status_t st = check_dtype_flags_complex(dtype, flags);
  if (st) return st;
  Schedule s;
  st = make_synth_schedule(n, (Dtype)dtype, flags, in_place, &s);
  if (st) return st;
  for (int i = 0; i < s.nsweep; ++i) sw[i] = s.sw[i];
  *nsweep = s.nsweep;
  return TPD_SUCCESS;
}

tpd_status_t host_batch_tables(const int* ns, int count, bool in_place, unsigned flags, int dtype, const int* codes,
                               std::vector<uint32_t>* perm, std::vector<BatchItem>* items) {
  tpd_status_t st = check_dtype_flags_complex(dtype, flags);
  if (st) return st;
  if (codes)
    for (int n = 0; n <= kMaxBatchQubits; ++n)
      if (!batch_code_ok(n, codes[n])) return TPD_ERROR_INVALID_VALUE;
  BatchTables bt;
  st = build_batch(ns, count, in_place, flags, (Dtype)dtype, &bt, codes);
  if (st) return st;
  *perm = std::move(bt.perm);
  *items = std::move(bt.items);
  return TPD_SUCCESS;
}
}  // namespace tpd

// ---------------------------------------------------------------------------
// autotuning
// ---------------------------------------------------------------------------
namespace {
double median3(std::vector<float>& v) {
  std::sort(v.begin(), v.end());
  return v.empty() ? 0.0 : v[v.size() / 2];
}
}  // namespace

extern "C" tpd_status_t tpd_debug_decompose_tuned(const void* A, int n, void* coeffs, tpd_dtype_t dtype,
                                                  unsigned flags, int db, int r, int grid_per_cu, int chunk_bits,
                                                  int chunk_window, tpd_stream_t stream) {
  tpd_status_t st = check_dtype_flags(dtype, flags);
  if (st) return st;
  if (n < 0 || n > max_qubits((Dtype)dtype)) return TPD_ERROR_UNSUPPORTED;
  if (grid_per_cu < 0 || grid_per_cu > 64 || chunk_bits < 0 || chunk_window < 0) return TPD_ERROR_INVALID_VALUE;
  const Dtype dt = (Dtype)dtype;
  st = check_buffers(A, coeffs, n, dt);
  if (st) return st;
  int dev;
  st = current_device(&dev);
  if (st) return st;
  Tuned t;
  t.db = db;
  t.r = r;
  t.grid = grid_per_cu;
  t.chunk = chunk_bits;
  t.window = chunk_window;
  Schedule s;
  st = make_schedule_with(n, dt, flags, A == coeffs, n > 8 ? &t : nullptr, &s);
  if (st) return st;
  hipStream_t hs = (hipStream_t)stream;
  uint32_t* bm = nullptr;
  // the lock is held until the kernels are enqueued: another thread on the
  // same stream could otherwise grow (free and reallocate) the workspace
  // between this thread taking its pointer and launching on it
  std::unique_lock<std::mutex> lk(g_mu, std::defer_lock);
  Pipe* pipe = nullptr;
  if ((s.prune && s.nsweep == 2) || s.chunk_window) {
    lk.lock();
    Workspace& w = g_ws[{dev, hs}];
    if (s.prune && s.nsweep == 2) {
      st = ensure_bitmap(w, s.bitmap_words);
      if (st) return st;
      bm = w.bitmap;
    }
    if (s.chunk_window) {
      st = w.pipe.ensure();
      if (st) return st;
      pipe = &w.pipe;
    }
  }
  return run_schedule(s, A, coeffs, bm, hs, nullptr, pipe);
}

extern "C" tpd_status_t tpd_debug_decompose_hermitian_real_tuned(void* A, int n, void* weights, tpd_dtype_t dtype,
                                                                unsigned flags, int db, int grid_per_cu,
                                                                tpd_stream_t stream) {
  if (grid_per_cu < 0 || grid_per_cu > 64) return TPD_ERROR_INVALID_VALUE;
  Tuned t;
  t.db = db;
  t.grid = grid_per_cu;
  return hermitian_real(A, n, weights, dtype, flags, db > 0 ? &t : nullptr, stream);
}

extern "C" tpd_status_t tpd_autotune_hermitian_real(void* A, int n, void* weights, tpd_dtype_t dtype,
                                                    unsigned flags, tpd_stream_t stream, char* report, size_t len) {
  TpdRange range_("tpd autotune hermitian real");
  tpd_status_t st = check_hermitian_real(A, n, weights, dtype, flags);
  if (st) return st;
  const Dtype dt = (Dtype)dtype;
  Schedule base;
  st = make_real_out_schedule(n, dt, flags, &base);
  if (st) return st;
  int dev;
  st = current_device(&dev);
  if (st) return st;
  std::string rep;
  if (base.nsweep != 2) {
    rep = "{\"tuned\":false,\"reason\":\"single-sweep schedule has no tunables\"}";
    return report ? copy_out(rep, report, len) : TPD_SUCCESS;
  }
  hipStream_t hs = (hipStream_t)stream;
  const int dbs128[3] = {3, 4, 5}, dbs64[3] = {4, 5, 6};
  const int* dbs = dt == DT_C128 ? dbs128 : dbs64;
  const int grids[5] = {0, 1, 2, 4, 8};
  std::vector<Tuned> cands;
  uint64_t max_words = 0;
  for (int i = 0; i < 3; ++i)
    for (int g : grids) {
      Tuned t;
      t.db = dbs[i];
      t.grid = g;
      Schedule sc;
      if (make_real_out_schedule(n, dt, flags, &sc, &t) != TPD_SUCCESS) continue;
      cands.push_back(t);
      if (sc.bitmap_words > max_words) max_words = sc.bitmap_words;
    }
  if (cands.empty()) return TPD_ERROR_INTERNAL;
  uint32_t* bm = nullptr;
  {
    void* p = nullptr;
    st = dev_alloc(&p, (size_t)max_words * 4);
    if (st) return st;
    bm = (uint32_t*)p;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    (void)hipFree(bm);
    return TPD_ERROR_OUT_OF_MEMORY;
  }
  double best = 1e300;
  Tuned best_t = cands[0];
  rep = "{\"tuned\":true,\"n\":" + std::to_string(n) + ",\"dtype\":\"" + dtype_name(dt) + "\",\"candidates\":[";
  bool first = true;
  // the first sweep transforms A in place: A is refilled with seeded noise
  // before every run (untimed), as the values of repeated transforms would
  // decay towards zero and time differently
  const uint64_t scalars = (uint64_t)2 << (2 * n);
  uint64_t seed = 0x7470645f74756e65ull;
  auto refill = [&]() {
    if (launch_fill_noise(A, scalars, dt == DT_C128, seed++, hs) != hipSuccess) st = TPD_ERROR_LAUNCH;
  };
  for (const Tuned& t : cands) {
    Schedule sc;
    if (make_real_out_schedule(n, dt, flags, &sc, &t) != TPD_SUCCESS) continue;
    refill();
    if (!st) st = run_real_out(sc, A, weights, bm, hs, nullptr);  // warm-up
    std::vector<float> ms;
    for (int r = 0; r < 3 && !st; ++r) {
      refill();
      if (!st && hipEventRecord(e0, hs) != hipSuccess) st = TPD_ERROR_LAUNCH;
      if (!st) st = run_real_out(sc, A, weights, bm, hs, nullptr);
      if (!st && hipEventRecord(e1, hs) != hipSuccess) st = TPD_ERROR_LAUNCH;
      float t_ms = 0;
      if (!st && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t_ms, e0, e1) != hipSuccess))
        st = TPD_ERROR_LAUNCH;
      ms.push_back(t_ms);
    }
    if (st) break;
    const double med = median3(ms);
    char buf[128];
    std::snprintf(buf, sizeof buf, "%s{\"db\":%d,\"grid_per_cu\":%d,\"ms\":%.4f}", first ? "" : ",", t.db, t.grid,
                  med);
    rep += buf;
    first = false;
    if (med < best) {
      best = med;
      best_t = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(hs);
  (void)hipFree(bm);
  if (st) return st;
  const TuneKey key{n, (int)dt, kRealOutKeyMatrix, 1, 1};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) load_tune_cache();
    g_tuned[key] = best_t;
    save_tune_entry(key, best_t);
  }
  char buf[128];
  std::snprintf(buf, sizeof buf, "],\"chosen\":{\"db\":%d,\"grid_per_cu\":%d,\"ms\":%.4f}}", best_t.db, best_t.grid,
                best);
  rep += buf;
  logf("autotune hermitian real %s", rep.c_str());
  return report ? copy_out(rep, report, len) : TPD_SUCCESS;
}

extern "C" tpd_status_t tpd_autotune(const void* A, int n, void* coeffs, tpd_dtype_t dtype, unsigned flags,
                                     tpd_stream_t stream, char* report, size_t len) {
  TpdRange range_("tpd autotune");
  tpd_status_t st = check_dtype_flags(dtype, flags);
  if (st) return st;
  if (n < 0 || n > max_qubits((Dtype)dtype)) return TPD_ERROR_UNSUPPORTED;
  const Dtype dt = (Dtype)dtype;
  st = check_buffers(A, coeffs, n, dt);
  if (st) return st;
  const bool in_place = A == coeffs;
  Schedule base;
  st = make_schedule(n, dt, flags & ~TPD_FLAG_ORDER_BOTTOM, in_place, &base);
  if (st) return st;
  int dev;
  st = current_device(&dev);
  if (st) return st;
  std::string rep;
  if (base.nsweep != 2) {
    rep = "{\"tuned\":false,\"reason\":\"single-sweep schedule has no tunables\"}";
    return report ? copy_out(rep, report, len) : TPD_SUCCESS;
  }
  hipStream_t hs = (hipStream_t)stream;
  // in place the buffer is refilled with seeded noise before every run
  // (untimed): the values of repeated transforms decay towards zero, and on
  // all-zero data the first sweep's pruning epilogue sets no bits and the
  // second sweep skips every tile, which times the candidates differently
  // (real float32 n = 16: a chunked schedule at 12.5 ms on decayed data that
  // takes 18.0 ms on data that stays live)
  const unsigned tflags = flags & ~TPD_FLAG_ORDER_BOTTOM;
  const int dbs128[3] = {3, 4, 5}, dbs64[3] = {4, 5, 6};
  const int* dbs = dt == DT_C128 ? dbs128 : dbs64;
  const int rs[1] = {4};
  const int grids[5] = {0, 1, 2, 4, 8};
  std::vector<Tuned> cands;
  uint64_t max_words = 0;
  for (int i = 0; i < 3; ++i)
    for (int r : rs)
      for (int g : grids) {
        Tuned t;
        t.db = dbs[i];
        t.r = r;
        t.grid = g;
        Schedule sc;
        if (make_schedule_with(n, dt, tflags, in_place, &t, &sc) != TPD_SUCCESS) continue;
        cands.push_back(t);
        if (sc.bitmap_words > max_words) max_words = sc.bitmap_words;
      }
  if (cands.empty()) return TPD_ERROR_INTERNAL;
  uint32_t* bm = nullptr;
  {
    void* p = nullptr;
    st = dev_alloc(&p, (size_t)max_words * 4);
    if (st) return st;
    bm = (uint32_t*)p;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    (void)hipFree(bm);
    return TPD_ERROR_OUT_OF_MEMORY;
  }
  Pipe pipe;  // pipelined chunk candidates (created when first timed)
  double best = 1e300;
  Tuned best_t = cands[0];
  rep = "{\"tuned\":true,\"n\":" + std::to_string(n) + ",\"dtype\":\"" + dtype_name(dt) +
        "\",\"candidates\":[";
  bool first = true;
  const uint64_t scalars = (uint64_t)(dt == DT_C128 || dt == DT_C64 ? 2 : 1) << (2 * n);
  uint64_t seed = 0x7470645f74756e65ull;
  auto refill = [&]() {
    if (in_place && launch_fill_noise(coeffs, scalars, dt == DT_C128 || dt == DT_R64, seed++, hs) != hipSuccess)
      st = TPD_ERROR_LAUNCH;
  };
  // median of three timed runs after a warm-up; false if the schedule does
  // not exist or a call failed (st set)
  auto time_candidate = [&](const Tuned& t, double* med) -> bool {
    Schedule sc;
    if (make_schedule_with(n, dt, tflags, in_place, &t, &sc) != TPD_SUCCESS) return false;
    if (sc.chunk_window) {
      st = pipe.ensure();
      if (st) return false;
    }
    refill();
    if (!st) st = run_schedule(sc, A, coeffs, bm, hs, nullptr, &pipe);  // warm-up
    if (st) return false;
    std::vector<float> ms;
    for (int rep_i = 0; rep_i < 3 && !st; ++rep_i) {
      refill();
      if (!st && hipEventRecord(e0, hs) != hipSuccess) st = TPD_ERROR_LAUNCH;
      if (!st) st = run_schedule(sc, A, coeffs, bm, hs, nullptr, &pipe);
      if (!st && hipEventRecord(e1, hs) != hipSuccess) st = TPD_ERROR_LAUNCH;
      float t_ms = 0;
      if (!st && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t_ms, e0, e1) != hipSuccess))
        st = TPD_ERROR_LAUNCH;
      ms.push_back(t_ms);
    }
    if (st) return false;
    *med = median3(ms);
    char buf[192];
    std::snprintf(buf, sizeof buf,
                  "%s{\"db\":%d,\"r\":%d,\"grid_per_cu\":%d,\"order2\":%d,\"chunk_bits\":%d,"
                  "\"chunk_window\":%d,\"ms\":%.4f}",
                  first ? "" : ",", t.db, t.r, t.grid, t.order2, t.chunk, t.window, *med);
    rep += buf;
    first = false;
    return true;
  };
  for (const Tuned& t : cands) {
    double med;
    if (!time_candidate(t, &med)) {
      if (st) break;
      continue;
    }
    if (med < best) {
      best = med;
      best_t = t;
    }
  }
  // then the winner with the second sweep's rotated tile order (which tiles
  // run side by side changes; which bytes move does not)
  if (!st && best < 1e300) {
    Tuned t = best_t;
    t.order2 = 1;
    double med;
    if (time_candidate(t, &med) && med < best) {
      best = med;
      best_t = t;
    }
  }
  // then the winner in the chunked order, sweep 1 and sweep 2 over 32-512 MB
  // of d-groups at a time: the second sweep may then read the chunk from the
  // 256 MB memory-side cache, but each chunk is a strip of columns across
  // all rows, so the sweeps lose row locality in HBM; on one stream every
  // chunk's two launches also drain the GPU, which the pipelined form
  // (sweep 2 on a second stream) avoids
  if (!st && best < 1e300 && !(flags & TPD_FLAG_HERMITIAN)) {
    const Tuned base_t = best_t;
    Schedule sc;
    if (make_schedule_with(n, dt, tflags, in_place, &base_t, &sc) == TPD_SUCCESS && sc.nsweep == 2) {
      const uint64_t group_bytes = ((uint64_t)elem_bytes(dt) << n) << sc.sw[0].db;
      for (uint64_t mb = 32; mb <= 512 && !st; mb *= 2) {
        int cb = 0;
        while ((group_bytes << (cb + 1)) <= (mb << 20)) ++cb;
        if (cb < 1 || cb >= n - sc.sw[0].db || (group_bytes << cb) != (mb << 20)) continue;
        // one stream (64 MB and up), or pipelined over two streams with 2 or
        // 4 chunks between their two sweeps
        for (int w : {0, 2, 4}) {
          if (w == 0 && mb < 64) continue;
          Tuned t = base_t;
          t.chunk = cb;
          t.window = w;
          double med;
          if (time_candidate(t, &med) && med < best) {
            best = med;
            best_t = t;
          }
          if (st) break;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(hs);
  pipe.destroy();
  (void)hipFree(bm);
  if (st) return st;
  const TuneKey key{n, (int)dt, (flags & TPD_FLAG_LAYOUT_MATRIX) ? 1 : 0, in_place ? 1 : 0,
                    (flags & TPD_FLAG_HERMITIAN) ? 1 : 0};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) load_tune_cache();
    g_tuned[key] = best_t;
    save_tune_entry(key, best_t);
  }
  char buf[256];
  std::snprintf(buf, sizeof buf,
                "],\"chosen\":{\"db\":%d,\"r\":%d,\"grid_per_cu\":%d,\"order2\":%d,\"chunk_bits\":%d,"
                "\"chunk_window\":%d,\"ms\":%.4f}}",
                best_t.db, best_t.r, best_t.grid, best_t.order2, best_t.chunk, best_t.window, best);
  rep += buf;
  logf("autotune %s", rep.c_str());
  return report ? copy_out(rep, report, len) : TPD_SUCCESS;
}

extern "C" tpd_status_t tpd_autotune_batched(tpd_plan_t plan, const void* const* d_ptrs, void* const* d_out_ptrs,
                                             tpd_stream_t stream, char* report, size_t len) {
  TpdRange range_("tpd autotune batched");
  if (!plan || !plan->batched || !d_ptrs) return TPD_ERROR_INVALID_VALUE;
  if (!d_out_ptrs && !plan->in_place) return TPD_ERROR_INVALID_VALUE;
  if (plan->tab.nitems == 0) return TPD_SUCCESS;
  hipStream_t hs = (hipStream_t)stream;
  const int cus = g_cus > 0 ? (int)g_cus : 256;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return TPD_ERROR_OUT_OF_MEMORY;
  }
  const int layout = (plan->flags & TPD_FLAG_LAYOUT_MATRIX) ? L_MAT : L_CAN;
  void* const* outs = d_out_ptrs ? d_out_ptrs : (void* const*)d_ptrs;
  tpd_status_t st = TPD_SUCCESS;
  // median of five timed launches after a warm-up
  auto time_table = [&](const DevBatch& tb, int grid, double* med) {
    std::vector<float> ms;
    for (int k = 0; k < 6 && !st; ++k) {
      if (hipEventRecord(e0, hs) != hipSuccess) st = TPD_ERROR_LAUNCH;
      if (!st && launch_batched_perm(plan->dt, d_ptrs, outs, tb.perm, tb.items, tb.nitems, tb.segs, tb.nseg, layout,
                                     grid, hs) != hipSuccess)
        st = TPD_ERROR_LAUNCH;
      if (!st && hipEventRecord(e1, hs) != hipSuccess) st = TPD_ERROR_LAUNCH;
      float t_ms = 0;
      if (!st && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t_ms, e0, e1) != hipSuccess))
        st = TPD_ERROR_LAUNCH;
      if (k > 0) ms.push_back(t_ms);  // the first launch is a warm-up
    }
    *med = st ? 0.0 : median3(ms);
    return st == TPD_SUCCESS;
  };
  std::string rep = "{\"tuned\":true,\"batched\":true,\"per_n\":[";
  // 1. per n present: every shape code on the matrices of that n alone
  //    (the others keep their codes), at the plan's grid
  int codes[kMaxBatchQubits + 1];
  std::memcpy(codes, plan->codes, sizeof codes);
  DevBatch sub;
  bool first_n = true;
  for (int n = kMaxBatchQubits; n >= 0 && !st; --n) {
    if (std::find(plan->ns.begin(), plan->ns.end(), n) == plan->ns.end()) continue;
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s{\"n\":%d,\"candidates\":[", first_n ? "" : ",", n);
    rep += buf;
    first_n = false;
    double best = 1e300;
    int best_code = codes[n];
    bool first_c = true;
    for (int code = 0; code < kBatchCodes && !st; ++code) {
      if (!batch_code_ok(n, code)) continue;
      int cc[kMaxBatchQubits + 1];
      std::memcpy(cc, codes, sizeof cc);
      cc[n] = code;
      BatchTables bt;
      st = build_batch(plan->ns.data(), plan->count, plan->in_place, plan->flags, plan->dt, &bt, cc, n);
      if (!st) st = sub.upload(bt);
      double med = 0;
      const int grid = std::min<int>(plan->grid, (int)sub.nitems);
      if (st || !time_table(sub, grid, &med)) break;
      std::snprintf(buf, sizeof buf, "%s{\"code\":%d,\"items\":%u,\"ms\":%.4f}", first_c ? "" : ",", code, sub.nitems,
                    med);
      rep += buf;
      first_c = false;
      if (med < best) {
        best = med;
        best_code = code;
      }
    }
    codes[n] = best_code;
    std::snprintf(buf, sizeof buf, "],\"chosen\":%d}", best_code);
    rep += buf;
  }
  sub.release();
  // 2. the whole table with the chosen codes
  if (!st) {
    BatchTables bt;
    st = build_batch(plan->ns.data(), plan->count, plan->in_place, plan->flags, plan->dt, &bt, codes);
    if (!st) st = plan->tab.upload(bt);
    if (!st) std::memcpy(plan->codes, codes, sizeof codes);
  }
  // 3. the grid: 1, 2, 3, 4, 6 or 8 workgroups per CU, or one per item
  rep += "],\"grid_candidates\":[";
  const int mults[7] = {1, 2, 3, 4, 6, 8, 0};
  double best = 1e300;
  int best_m = 2, best_grid = plan->grid;
  for (int i = 0; i < 7 && !st; ++i) {
    const int m = mults[i];
    int grid = m > 0 ? m * cus : (int)plan->tab.nitems;
    if ((uint32_t)grid > plan->tab.nitems) grid = (int)plan->tab.nitems;
    double med = 0;
    if (!time_table(plan->tab, grid, &med)) break;
    char buf[128];
    std::snprintf(buf, sizeof buf, "%s{\"grid_per_cu\":%d,\"grid\":%d,\"ms\":%.4f}", i ? "," : "", m, grid, med);
    rep += buf;
    if (med < best) {
      best = med;
      best_m = m;
      best_grid = grid;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  plan->grid = best_grid;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) load_tune_cache();
    Tuned t;
    t.db = 0;
    t.r = 4;
    t.grid = best_m;
    const TuneKey key{-1, (int)plan->dt, 0, 0, 0};
    g_tuned[key] = t;
    save_tune_entry(key, t);
    for (int n = 0; n <= kMaxBatchQubits; ++n) {
      if (std::find(plan->ns.begin(), plan->ns.end(), n) == plan->ns.end()) continue;
      Tuned tn;
      tn.db = codes[n];  // the shape code, stored in the tile-width field
      tn.r = 4;
      tn.grid = 0;
      const TuneKey kn{n, (int)plan->dt, kBatchedKeyMatrix, 0, 0};
      g_tuned[kn] = tn;
      save_tune_entry(kn, tn);
    }
  }
  char buf[256];
  std::snprintf(buf, sizeof buf, "],\"chosen\":{\"grid_per_cu\":%d,\"grid\":%d,\"ms\":%.4f,\"codes\":[", best_m,
                best_grid, best);
  rep += buf;
  for (int n = 0; n <= kMaxBatchQubits; ++n) {
    std::snprintf(buf, sizeof buf, "%s%d", n ? "," : "", codes[n]);
    rep += buf;
  }
  rep += "]}}";
  return report ? copy_out(rep, report, len) : TPD_SUCCESS;
}

extern "C" tpd_status_t tpd_debug_plan_batched_codes(tpd_plan_t plan, const int* codes) {
  if (!plan || !plan->batched || !codes) return TPD_ERROR_INVALID_VALUE;
  for (int n = 0; n <= kMaxBatchQubits; ++n)
    if (!batch_code_ok(n, codes[n])) return TPD_ERROR_INVALID_VALUE;
  BatchTables bt;
  tpd_status_t st = build_batch(plan->ns.data(), plan->count, plan->in_place, plan->flags, plan->dt, &bt, codes);
  if (st) return st;
  st = plan->tab.upload(bt);
  if (st) return st;
  std::memcpy(plan->codes, codes, sizeof plan->codes);
  return TPD_SUCCESS;
}
