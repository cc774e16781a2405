// Binary tensor contractions on the device.
//
// ctr() maps C[lc] = alpha * sum A[la] B[lb] + beta C[lc] onto one batched
// complex GEMM: labels shared by A, B and C are batch dimensions, labels of A
// and C are M, of B and C are N, of A and B are K.  An operand is used in
// place when each of its label groups is contiguous and in the canonical
// order (then every group collapses to a single stride); otherwise it is first
// permuted into [batch][M][K] / [batch][N][K] (K contiguous) by the permute
// kernel.  The product goes straight into C when C is [batch][M][N] or
// [batch][N][M], and through a temporary plus a permute otherwise.
#include <algorithm>
#include <cstring>
#include <cstdio>
#include <map>
#include <mutex>
#include <stdexcept>

#include "internal.h"

namespace adc {

// ------------------------------------------------------------------ pool
std::shared_mutex& capture_gate() {
  static std::shared_mutex gate;
  return gate;
}

Pool::~Pool() { release_all(); }

double2* Pool::get(int64_t n) {
  const size_t bytes = std::max<size_t>(256, (size_t)n * sizeof(double2));
  if (arena_base_) {
    const size_t need = (bytes + 255) / 256 * 256;
    for (size_t i = 0; i < arena_free_.size(); ++i) {
      Span& f = arena_free_[i];
      if (f.len < need) continue;
      const size_t off = f.off;
      f.off += need;
      f.len -= need;
      if (f.len == 0) arena_free_.erase(arena_free_.begin() + i);
      arena_used_.push_back({off, need});
      arena_peak_ = std::max(arena_peak_, off + need);
      return (double2*)(arena_base_ + off);
    }
    throw ArenaFull{need};
  }
  if (hold_) {
    // reuse a block this capture has already released
    int cb = -1;
    size_t cbytes = 0;
    for (size_t i = 0; i < cap_free_.size(); ++i)
      for (const Blk& u : used_)
        if (u.p == cap_free_[i] && u.bytes >= bytes && u.bytes <= 2 * bytes + (1 << 20) &&
            (cb < 0 || u.bytes < cbytes)) {
          cb = (int)i;
          cbytes = u.bytes;
        }
    if (cb >= 0) {
      void* p = cap_free_[cb];
      cap_free_.erase(cap_free_.begin() + cb);
      return (double2*)p;
    }
  }
  int best = -1;
  for (size_t i = 0; i < free_.size(); ++i) {
    if (free_[i].bytes >= bytes && free_[i].bytes <= 2 * bytes + (1 << 20)) {
      if (best < 0 || free_[i].bytes < free_[best].bytes) best = (int)i;
    }
  }
  Blk b;
  if (best >= 0) {
    b = free_[best];
    free_.erase(free_.begin() + best);
  } else {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      // while this pool's stream is being captured nothing may wait on the
      // device: report the shortage (the caller then runs the step eagerly)
      if (hold_) throw HipError{hipErrorOutOfMemory, "pool (during graph capture)"};
      // drop cached blocks and retry once
      {
        std::unique_lock<std::shared_mutex> lk(capture_gate());
        (void)hipDeviceSynchronize();
        for (auto& f : free_) (void)hipFree(f.p);
      }
      free_.clear();
      e = hipMalloc(&p, bytes);
      if (e != hipSuccess) throw HipError{hipErrorOutOfMemory, "pool"};
    }
    b = {p, bytes};
  }
  used_.push_back(b);
  in_use_ += b.bytes;
  if (tape) tape->add(b.p, b.bytes, false);
  if (hold_) touched_.push_back(b.p);
  return (double2*)b.p;
}

void Pool::begin_hold() {
  hold_ = true;
  touched_.clear();
  cap_free_.clear();
}

std::vector<double2*> Pool::end_hold() {
  hold_ = false;
  std::vector<double2*> out;
  for (void* p : touched_) out.push_back((double2*)p);
  touched_.clear();
  cap_free_.clear();
  return out;
}

void Pool::begin_arena(void* base, size_t bytes) {
  arena_base_ = (char*)base;
  arena_bytes_ = bytes / 256 * 256;
  arena_peak_ = 0;
  arena_free_.assign(1, Span{0, arena_bytes_});
  arena_used_.clear();
}

size_t Pool::end_arena() {
  const size_t peak = arena_peak_;
  arena_base_ = nullptr;
  arena_bytes_ = arena_peak_ = 0;
  arena_free_.clear();
  arena_used_.clear();
  return peak;
}

void Pool::put(double2* p) {
  if (!p) return;
  if (arena_base_ && (char*)p >= arena_base_ && (char*)p < arena_base_ + arena_bytes_) {
    const size_t off = (size_t)((char*)p - arena_base_);
    for (size_t i = 0; i < arena_used_.size(); ++i) {
      if (arena_used_[i].off != off) continue;
      Span sp = arena_used_[i];
      arena_used_.erase(arena_used_.begin() + i);
      // insert in offset order and merge with the neighbours
      size_t j = 0;
      while (j < arena_free_.size() && arena_free_[j].off < sp.off) ++j;
      arena_free_.insert(arena_free_.begin() + j, sp);
      if (j + 1 < arena_free_.size() && arena_free_[j].off + arena_free_[j].len == arena_free_[j + 1].off) {
        arena_free_[j].len += arena_free_[j + 1].len;
        arena_free_.erase(arena_free_.begin() + j + 1);
      }
      if (j > 0 && arena_free_[j - 1].off + arena_free_[j - 1].len == arena_free_[j].off) {
        arena_free_[j - 1].len += arena_free_[j].len;
        arena_free_.erase(arena_free_.begin() + j);
      }
      return;
    }
    return;
  }
  if (hold_ && std::find(touched_.begin(), touched_.end(), (void*)p) != touched_.end()) {
    cap_free_.push_back(p);
    return;
  }
  if (tape) {
    const int i = tape->find(p);
    if (i >= 0 && tape->allocs[i].base == (uintptr_t)p) {
      if (tape->allocs[i].ref) {
        tape->deferred.push_back(p);
        return;
      }
      tape->allocs.erase(tape->allocs.begin() + i);
    }
  }
  for (size_t i = 0; i < used_.size(); ++i) {
    if (used_[i].p == p) {
      in_use_ -= used_[i].bytes;
      free_.push_back(used_[i]);
      used_.erase(used_.begin() + i);
      return;
    }
  }
}

void Pool::trim() {
  if (!free_.empty()) {
    std::unique_lock<std::shared_mutex> lk(capture_gate());
    for (auto& b : free_) (void)hipFree(b.p);
  }
  free_.clear();
}

void Pool::release_all() {
  if (!free_.empty() || !used_.empty()) {
    std::unique_lock<std::shared_mutex> lk(capture_gate());
    for (auto& b : free_) (void)hipFree(b.p);
    for (auto& b : used_) (void)hipFree(b.p);
  }
  free_.clear();
  used_.clear();
  in_use_ = 0;
}

// ------------------------------------------------------------------ GEMM driver
// Heuristic split-K: outputs with too few tiles to fill the 256 CUs split the
// K loop into chunks whose partial sums a reduction kernel adds up.
bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) {
    (void)hipGetLastError();
    return true;
  }
  return st != hipStreamCaptureStatusNone;
}

namespace {

int64_t heuristic_nsplit(int64_t M, int64_t N, int64_t K, int64_t batch, int64_t kmin) {
  const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64) * batch;
  int64_t nsplit = 1;
  if (tiles < 512 && K >= 2 * kmin) {
    nsplit = std::min<int64_t>({(1024 + tiles - 1) / tiles, K / kmin, 256});
    if (batch * nsplit > 65535) nsplit = 65535 / batch;
  }
  return std::max<int64_t>(1, nsplit);
}

void run_zgemm(Ctx& cx, GemmDesc g, int tile, int64_t nsplit) {
  g.tile = tile;
  if (cx.verbose >= 2)
    std::fprintf(stderr, "[gemm] %s M %lld N %lld K %lld batch %lld split %lld\n", cx.prec == 1 ? "fp32" : "fp64",
                 (long long)g.M, (long long)g.N, (long long)g.K, (long long)g.batch, (long long)nsplit);
  if (nsplit <= 1) {
    g.nsplit = 1;
    g.kchunk = g.K;
    launch_zgemm(g, cx.prec, cx.stream);
    return;
  }
  int64_t chunk = (g.K + nsplit - 1) / nsplit;
  chunk = (chunk + 15) / 16 * 16;
  nsplit = (g.K + chunk - 1) / chunk;
  g.kchunk = chunk;
  g.nsplit = (int)nsplit;
  g.P = cx.pool.get(nsplit * g.batch * g.M * g.N);
  launch_zgemm(g, cx.prec, cx.stream);
  launch_splitk_reduce(g, cx.stream);
  cx.pool.put(g.P);
}

void log_bf16p(const Ctx& cx, const BfGemm& g) {
  if (cx.verbose < 2) return;
  std::fprintf(stderr, "[gemm] bf16x3 tag %d M %lld N %lld Kp %lld split %d tile %d rows(", g.tag, (long long)g.M,
               (long long)g.N, (long long)g.Kp, g.nsplit, g.tile < 0 ? bf16p_pick_tile(g) : g.tile);
  for (int q = 0; q < g.om.nm; ++q) std::fprintf(stderr, " %lldx%lld", (long long)g.om.md[q], (long long)g.om.ms[q]);
  std::fprintf(stderr, " | %lld) cols(", (long long)g.scm);
  for (int q = 0; q < g.om.nn; ++q) std::fprintf(stderr, " %lldx%lld", (long long)g.om.nd[q], (long long)g.om.ns[q]);
  std::fprintf(stderr, " | %lld) beta %d\n", (long long)g.scn, (g.beta.re != 0.0 || g.beta.im != 0.0) ? 1 : 0);
}

void run_bf16p(Ctx& cx, BfGemm g, int tile, int64_t nsplit) {
  g.tile = tile;
  if (nsplit <= 1) {
    g.nsplit = 1;
    g.kchunk = g.Kp;
    log_bf16p(cx, g);
    launch_bf16p(g, cx.stream);
    return;
  }
  int64_t chunk = (g.Kp + nsplit - 1) / nsplit;
  chunk = (chunk + 31) / 32 * 32;
  nsplit = (g.Kp + chunk - 1) / chunk;
  g.kchunk = chunk;
  g.nsplit = (int)nsplit;
  log_bf16p(cx, g);
  g.P = cx.pool.get(nsplit * g.M * g.N);
  launch_bf16p(g, cx.stream);
  launch_splitk_reduce_bf(g, cx.stream);
  cx.pool.put(g.P);
}

// ------------------------------------------------------------------ autotuner
// Shape classes: kernel family, arithmetic, instance tag, and ceil(log2) of
// M, N, K and the batch count.  The first GEMM of a class times every
// candidate (tile size x split-K factor) on a scratch output and keeps the
// fastest for the rest of the process.  Skipped while a stream is being
// captured (timing needs host synchronisation) and for outputs above 2^26
// elements (the scratch copy would be too large).
struct TuneKey {
  int fam, prec, tag, lm, ln, lk, lb;
  bool operator<(const TuneKey& o) const {
    const int a[7] = {fam, prec, tag, lm, ln, lk, lb}, b[7] = {o.fam, o.prec, o.tag, o.lm, o.ln, o.lk, o.lb};
    for (int i = 0; i < 7; ++i)
      if (a[i] != b[i]) return a[i] < b[i];
    return false;
  }
};
struct TuneChoice {
  int tile;
  int64_t nsplit;
};

std::mutex g_tune_mu;
std::map<TuneKey, TuneChoice> g_tune;

int lg2(int64_t n) {
  int l = 0;
  while (((int64_t)1 << l) < n) ++l;
  return l;
}

std::vector<TuneChoice> candidates(int64_t heur, const std::vector<int>& tiles) {
  std::vector<int64_t> ns = {heur};
  if (heur > 1) ns.push_back(1);
  if (heur > 2) ns.push_back(heur / 2);
  if (heur * 2 <= 256 && heur > 1) ns.push_back(heur * 2);
  std::vector<TuneChoice> c;
  for (int t : tiles)
    for (int64_t n : ns) c.push_back({t, n});
  return c;
}

// time fn(choice) for every candidate (one warm-up, two timed runs)
template <class F>
TuneChoice tune(Ctx& cx, const std::vector<TuneChoice>& cand, F&& fn) {
  hipEvent_t e0, e1;
  hipcheck(hipEventCreate(&e0), "tune ev");
  hipcheck(hipEventCreate(&e1), "tune ev");
  TuneChoice best = cand[0];
  float tbest = 1e30f;
  for (const TuneChoice& c : cand) {
    fn(c);
    hipcheck(hipEventRecord(e0, cx.stream), "tune rec");
    fn(c);
    fn(c);
    hipcheck(hipEventRecord(e1, cx.stream), "tune rec");
    hipcheck(hipEventSynchronize(e1), "tune sync");
    float ms = 0.f;
    hipcheck(hipEventElapsedTime(&ms, e0, e1), "tune time");
    if (ms < tbest) {
      tbest = ms;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

}  // namespace

// Tuned choices as text, one shape class per line:
//   fam prec tag lm ln lk lb tile nsplit
// Loading merges the file into the process-wide table (entries already
// present win); saving writes the whole table.  Returns the number of
// entries read or written, or -1 if the file cannot be opened.
int tune_cache_load(const char* path) {
  if (!path || !*path) return 0;
  FILE* f = std::fopen(path, "r");
  if (!f) return -1;
  int n = 0;
  TuneKey k{};
  TuneChoice c{};
  long long ns = 0;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  while (std::fscanf(f, "%d %d %d %d %d %d %d %d %lld", &k.fam, &k.prec, &k.tag, &k.lm, &k.ln, &k.lk, &k.lb,
                     &c.tile, &ns) == 9) {
    c.nsplit = std::max<int64_t>(1, (int64_t)ns);
    if (g_tune.emplace(k, c).second) ++n;
  }
  std::fclose(f);
  return n;
}

int tune_cache_save(const char* path) {
  if (!path || !*path) return 0;
  FILE* f = std::fopen(path, "w");
  if (!f) return -1;
  int n = 0;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  for (const auto& e : g_tune) {
    const TuneKey& k = e.first;
    std::fprintf(f, "%d %d %d %d %d %d %d %d %lld\n", k.fam, k.prec, k.tag, k.lm, k.ln, k.lk, k.lb, e.second.tile,
                 (long long)e.second.nsplit);
    ++n;
  }
  return std::fclose(f) == 0 ? n : -1;
}

double* Ctx::pinned(size_t n) {
  if (n > pinned_n_) {
    // freeing page-locked memory synchronises the device
    std::unique_lock<std::shared_mutex> gate(capture_gate());
    if (pinned_) (void)hipHostFree(pinned_);
    pinned_ = nullptr;
    pinned_n_ = 0;
    const size_t want = std::max<size_t>(n, 256);
    hipcheck(hipHostMalloc((void**)&pinned_, sizeof(double) * want), "pinned report buffer");
    pinned_n_ = want;
  }
  return pinned_;
}

Ctx::~Ctx() {
  if (pinned_) {
    std::unique_lock<std::shared_mutex> gate(capture_gate());
    (void)hipHostFree(pinned_);
  }
}

void gemm(Ctx& cx, GemmDesc g) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0 || g.K <= 0) return;
  const int64_t heur = heuristic_nsplit(g.M, g.N, g.K, g.batch, 128);
  const int64_t out = g.M * g.N * g.batch;
  if (!cx.autotune || cx.prec == 2 || out > ((int64_t)1 << 26)) {
    run_zgemm(cx, g, -1, heur);
    return;
  }
  const TuneKey key{0, cx.prec, g.tag, lg2(g.M), lg2(g.N), lg2(g.K), lg2(g.batch)};
  TuneChoice ch{-1, heur};
  bool found = false;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) { ch = it->second; found = true; }
  }
  if (!found && !capturing(cx.stream)) {
    double2* scratch = cx.pool.get(out);
    GemmDesc t = g;
    t.C = scratch; t.scm = g.N; t.scn = 1; t.scb = g.M * g.N;
    t.beta = {0.0, 0.0};
    t.om = OutMap{};
    ch = tune(cx, candidates(heur, cx.prec == 1 ? std::vector<int>{0, 1, 2} : std::vector<int>{0, 1}),
              [&](const TuneChoice& c) { run_zgemm(cx, t, c.tile, c.nsplit); });
    cx.pool.put(scratch);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[key] = ch;
  }
  run_zgemm(cx, g, ch.tile, std::min<int64_t>(ch.nsplit, std::max<int64_t>(1, g.K / 16)));
}

// Tile and split-K of a split-bf16 GEMM from a cost model: the time of the
// matrix work (padded tile work at the rate the tile sustains, per wave of
// workgroups the chip holds at once), of the operand planes (each row block of
// A is read once per column tile and vice versa), and of the output (split-K
// partials written and read back); the matrix and operand terms overlap.
static TuneChoice bf16_choice(int64_t M, int64_t N, int64_t Kp, bool beta) {
  struct Cand { int tile, bm, bn; double rate; int64_t slots; };
  const Cand cand[4] = {{9, 128, 128, 0.41, 256}, {13, 64, 256, 0.35, 256}, {2, 128, 64, 0.35, 512},
                        {0, 64, 64, 0.31, 1024}};
  const double peak = 2.5e15, bw = 4.0e12, wbw = 3.5e12;
  TuneChoice best{0, 1};
  double tbest = -1.0;
  for (const Cand& c : cand) {
    const int64_t tm = (M + c.bm - 1) / c.bm, tn = (N + c.bn - 1) / c.bn, tiles = tm * tn;
    // split-K so that the grid fills 1..4 waves of slots, each chunk at
    // least 8 slices of 32
    std::vector<int64_t> splits = {1};
    for (int64_t w = 1; w <= 4; ++w) {
      const int64_t ns = std::min<int64_t>({(w * c.slots + tiles - 1) / tiles, Kp / 256, 256});
      if (ns > 1) splits.push_back(ns);
    }
    for (int64_t ns0 : splits) {
      const int64_t chunk = ((Kp + ns0 - 1) / ns0 + 31) / 32 * 32, ns = (Kp + chunk - 1) / chunk;
      const int64_t nwg = tiles * ns, waves = (nwg + c.slots - 1) / c.slots;
      if (c.tile != 0 && 2 * nwg < c.slots) continue;
      const double t_mma = (double)waves * c.bm * c.bn * (double)chunk * 24.0 / (c.rate * peak / c.slots);
      // an operand of a few MB stays in the L2 and is fetched once
      const double pa = (double)M * Kp * 8.0, pb = (double)N * Kp * 8.0;
      const double t_in = ((pa > 4e6 ? (double)tn : 1.0) * pa + (pb > 4e6 ? (double)tm : 1.0) * pb) / bw;
      const double out = (double)M * N * 16.0;
      const double t_out = ns > 1 ? (2.0 * ns * out + out * (beta ? 2.0 : 1.0)) / bw + 5e-6
                                  : out * (beta ? 2.0 : 1.0) / wbw;
      const double t = std::max(t_mma, t_in) + t_out;
      if (tbest < 0.0 || t < tbest) { tbest = t; best = {c.tile, ns}; }
    }
  }
  return best;
}

void gemm_bf16p(Ctx& cx, BfGemm g) {
  if (g.M <= 0 || g.N <= 0 || g.Kp <= 0) return;
  const bool beta = g.beta.re != 0.0 || g.beta.im != 0.0;
  const TuneChoice model = bf16_choice(g.M, g.N, g.Kp, beta);
  const int64_t heur = model.nsplit;
  const int64_t out = g.M * g.N;
  if (!cx.autotune || out > ((int64_t)1 << 26)) {
    run_bf16p(cx, g, model.tile, model.nsplit);
    return;
  }
  const TuneKey key{1, 2, g.tag, lg2(g.M), lg2(g.N), lg2(g.Kp), 0};
  TuneChoice ch = model;
  bool found = false;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) { ch = it->second; found = true; }
  }
  if (!found && !capturing(cx.stream)) {
    double2* scratch = cx.pool.get(out);
    BfGemm t = g;
    t.C = scratch; t.scm = g.N; t.scn = 1;
    t.beta = {0.0, 0.0};
    t.om = OutMap{};
    ch = tune(cx, candidates(heur, {0, 2, 9, 10, 11, 12, 13}), [&](const TuneChoice& c) { run_bf16p(cx, t, c.tile, c.nsplit); });
    cx.pool.put(scratch);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[key] = ch;
  }
  run_bf16p(cx, g, ch.tile, std::min<int64_t>(ch.nsplit, std::max<int64_t>(1, g.Kp / 32)));
}

Tensor tnew(Ctx& cx, std::vector<int64_t> d, bool zero) {
  Tensor t;
  t.d = std::move(d);
  t.p = cx.pool.get(std::max<int64_t>(1, t.size()));
  if (zero) launch_fill(t.p, t.size(), C0(), cx.stream);
  return t;
}

Tensor tnew32(Ctx& cx, std::vector<int64_t> d) {
  Tensor t;
  t.d = std::move(d);
  t.p = cx.pool.get(std::max<int64_t>(1, (t.size() + 1) / 2));
  t.f32 = true;
  return t;
}

void tfree(Ctx& cx, Tensor& t) {
  cx.pool.put(t.p);
  t.p = nullptr;
}

// ------------------------------------------------------------------ helpers
namespace {

struct View {
  // strides of each label (complex elements)
  std::map<char, int64_t> stride;
  std::map<char, int64_t> size;
};

View view_of(const Tensor& t, const char* l) {
  const int n = (int)std::strlen(l);
  if (n != (int)t.d.size()) throw std::invalid_argument(std::string("label/rank mismatch: ") + l);
  View v;
  int64_t s = 1;
  for (int i = n - 1; i >= 0; --i) {
    if (v.stride.count(l[i])) throw std::invalid_argument(std::string("repeated label: ") + l);
    v.stride[l[i]] = t.st.empty() ? s : t.st[i];
    v.size[l[i]] = t.d[i];
    s *= t.d[i];
  }
  return v;
}

// Can the labels `grp` (in this order) of view v be collapsed into one stride?
// Returns the stride of the fused index (stride of the last label) or -1.
int64_t fused_stride(const View& v, const std::string& grp) {
  if (grp.empty()) return 0;
  for (size_t i = 0; i + 1 < grp.size(); ++i) {
    const char a = grp[i], b = grp[i + 1];
    if (v.stride.at(a) != v.stride.at(b) * v.size.at(b)) return -1;
  }
  return v.stride.at(grp.back());
}

int64_t prod(const View& v, const std::string& grp) {
  int64_t p = 1;
  for (char c : grp) p *= v.size.at(c);
  return p;
}

// Mixed-radix digits (at most four) of the label group `grp` of view v, with
// adjacent labels that fuse merged; an empty group is one digit of extent 1.
bool split_digits(const View& v, const std::string& grp, int& n, int64_t* d, int64_t* st) {
  std::vector<int64_t> dd, ss;
  for (char c : grp) {
    const int64_t sz = v.size.at(c), sd = v.stride.at(c);
    if (!dd.empty() && ss.back() == sd * sz) {
      dd.back() *= sz;
      ss.back() = sd;
    } else {
      dd.push_back(sz);
      ss.push_back(sd);
    }
  }
  if (dd.empty()) {
    dd.push_back(1);
    ss.push_back(0);
  }
  if (dd.size() > 4) return false;
  n = (int)dd.size();
  for (int q = 0; q < n; ++q) {
    d[q] = dd[q];
    st[q] = ss[q];
  }
  return true;
}

// Output layout of one label group of C: a single stride when the group fuses,
// else a mixed-radix map of at most three digits (adjacent labels that fuse
// are merged first).  Returns false when neither applies.
bool group_map(const View& v, const std::string& grp, int64_t& stride, int& n, int64_t* d, int64_t* st) {
  n = 0;
  if (grp.empty()) {
    stride = 0;
    return true;
  }
  const int64_t f = fused_stride(v, grp);
  if (f >= 0) {
    stride = f;
    return true;
  }
  if (prod(v, grp) >= ((int64_t)1 << 31)) return false;
  std::vector<int64_t> dd, ss;
  for (char c : grp) {
    const int64_t sz = v.size.at(c), sd = v.stride.at(c);
    if (!dd.empty() && ss.back() == sd * sz) {
      dd.back() *= sz;
      ss.back() = sd;
    } else {
      dd.push_back(sz);
      ss.push_back(sd);
    }
  }
  if (dd.size() > 3) return false;
  n = (int)dd.size();
  for (int q = 0; q < n; ++q) {
    d[q] = dd[q];
    st[q] = ss[q];
  }
  stride = 1;
  return true;
}

// copy/accumulate view v of src into dst, iterating the labels `ord`;
// dst strides per label come from dv (or contiguous in `ord` when null)
void permute_into(Ctx& cx, const Tensor& src, const View& v, const std::string& ord, bool conj, double2* dst,
                  cplx alpha, cplx beta, const View* dv = nullptr) {
  std::vector<int64_t> od, is, os;
  for (char c : ord) {
    od.push_back(v.size.at(c));
    is.push_back(v.stride.at(c));
  }
  if (dv) {
    for (char c : ord) os.push_back(dv->stride.at(c));
  } else {
    os.resize(ord.size());
    int64_t s = 1;
    for (int i = (int)ord.size() - 1; i >= 0; --i) {
      os[i] = s;
      s *= od[i];
    }
  }
  // merge consecutive dims that are contiguous in both (fewer divisions)
  std::vector<int64_t> od2, is2, os2;
  for (size_t i = 0; i < od.size(); ++i) {
    if (!od2.empty() && is2.back() == is[i] * od[i] && os2.back() == os[i] * od[i]) {
      od2.back() *= od[i];
      is2.back() = is[i];
      os2.back() = os[i];
    } else {
      od2.push_back(od[i]);
      is2.push_back(is[i]);
      os2.push_back(os[i]);
    }
  }
  if (od2.size() > 8) throw std::invalid_argument("rank > 8");
  launch_permute((int)od2.size(), od2.data(), is2.data(), os2.data(), src.p, dst, alpha, beta, conj ? 1 : 0,
                 cx.stream);
}

}  // namespace

void tape_record(Ctx& cx, TapeOp op) {
  Tape* t = cx.tape;
  if (!t || !t->recording) return;
  if (op.kind != TapeOp::LADDER) op.prec = cx.prec;
  bool rg = op.kind == TapeOp::LADDER;  // the ladder always reads L_vv
  for (const Tensor* x : {&op.A, &op.B}) rg = rg || (x->p && t->rg(x->p));
  const int ic = op.C.p ? t->find(op.C.p) : -1;
  // an op is kept when a gradient can flow through it, or when it overwrites
  // a tensor that carries one (the sweep must then clear that gradient)
  if (!rg && !(ic >= 0 && t->allocs[ic].rg)) return;
  // the sweep reads operand values of products (and the ladder's trial
  // vectors); a later write into such a buffer would corrupt them
  if (ic >= 0 && t->allocs[ic].needed)
    throw std::logic_error("recorded op overwrites a buffer whose values the reverse sweep needs");
  if (rg && ic >= 0) t->allocs[ic].rg = true;
  for (const Tensor* x : {&op.A, &op.B, &op.C}) {
    const int i = x->p ? t->find(x->p) : -1;
    if (i >= 0) t->allocs[i].ref = true;
  }
  auto need = [&](const Tensor& x) {
    const int i = x.p ? t->find(x.p) : -1;
    if (i >= 0) t->allocs[i].needed = true;
  };
  if (op.kind == TapeOp::CTR) {
    if (t->rg(op.B.p)) need(op.A);
    if (t->rg(op.A.p)) need(op.B);
  } else if (op.kind == TapeOp::LADDER) {
    need(op.A);
  }
  t->ops.push_back(std::move(op));
}

namespace {
struct Pause {
  Tape* t;
  bool was;
  explicit Pause(Ctx& cx) : t(cx.tape), was(cx.tape ? cx.tape->recording : false) {
    if (t) t->recording = false;
  }
  ~Pause() {
    if (t) t->recording = was;
  }
};
}  // namespace

void perm(Ctx& cx, cplx alpha, const Tensor& A, const char* la, bool cA, cplx beta, Tensor& C, const char* lc) {
  if (cx.tape && cx.tape->recording) {
    TapeOp op{};
    op.kind = TapeOp::PERM;
    op.A = A; op.C = C; op.la = la; op.lc = lc; op.cA = cA; op.alpha = alpha; op.beta = beta;
    tape_record(cx, op);
  }
  Pause pause(cx);
  View va = view_of(A, la);
  View vc = view_of(C, lc);
  for (auto& kv : vc.size)
    if (!va.size.count(kv.first) || va.size.at(kv.first) != kv.second)
      throw std::invalid_argument(std::string("perm: label mismatch ") + la + " -> " + lc);
  if (va.size.size() != vc.size.size()) throw std::invalid_argument("perm: rank mismatch");
  permute_into(cx, A, va, lc, cA, C.p, alpha, beta, &vc);
}

Tensor tslice(const Tensor& t, int dim, int64_t lo, int64_t hi) {
  Tensor v;
  v.d = t.d;
  if (t.st.empty()) {
    v.st.resize(t.d.size());
    int64_t s = 1;
    for (int i = (int)t.d.size() - 1; i >= 0; --i) {
      v.st[i] = s;
      s *= t.d[i];
    }
  } else {
    v.st = t.st;
  }
  v.p = t.f32 ? (double2*)((float2*)t.p + lo * v.st[dim]) : t.p + lo * v.st[dim];
  v.d[dim] = hi - lo;
  v.f32 = t.f32;
  return v;
}

// ------------------------------------------------------------------ split cache
namespace {

// digits (size, stride), merged where contiguous
std::vector<std::pair<int64_t, int64_t>> flat_digits(const int64_t* d0, const int64_t* s0, int n0, const int64_t* d1,
                                                     const int64_t* s1, int n1) {
  std::vector<std::pair<int64_t, int64_t>> d;
  auto add = [&](int64_t n, int64_t st) {
    if (n == 1) return;
    if (!d.empty() && d.back().second == n * st) {
      d.back().first *= n;
      d.back().second = st;
    } else {
      d.push_back({n, st});
    }
  };
  for (int q = 0; q < n0; ++q) add(d0[q], s0[q]);
  for (int q = 0; q < n1; ++q) add(d1[q], s1[q]);
  return d;
}

// two splits write identical planes when they read the same source in the
// same order: rows then K as one traversal when K needs no padding, else
// rows and K each (with equal row count, K and padding)
bool same_layout(const SplitNd& a, const SplitNd& b) {
  if (a.src != b.src || a.conj != b.conj) return false;
  if (a.K == a.Kp && b.K == b.Kp && a.rows * a.Kp == b.rows * b.Kp)
    return flat_digits(a.md, a.ms, a.nm, a.kd, a.ks, a.nk) == flat_digits(b.md, b.ms, b.nm, b.kd, b.ks, b.nk);
  if (a.rows != b.rows || a.K != b.K || a.Kp != b.Kp) return false;
  return flat_digits(a.md, a.ms, a.nm, nullptr, nullptr, 0) == flat_digits(b.md, b.ms, b.nm, nullptr, nullptr, 0) &&
         flat_digits(a.kd, a.ks, a.nk, nullptr, nullptr, 0) == flat_digits(b.kd, b.ks, b.nk, nullptr, nullptr, 0);
}

// scope of the frozen range that holds every element the split reads, or -1
int frozen_scope(const SplitCache& c, const SplitNd& sp) {
  int64_t hi = 0;
  for (int q = 0; q < sp.nm; ++q) {
    if (sp.ms[q] < 0) return -1;
    hi += (sp.md[q] - 1) * sp.ms[q];
  }
  for (int q = 0; q < sp.nk; ++q) {
    if (sp.ks[q] < 0) return -1;
    hi += (sp.kd[q] - 1) * sp.ks[q];
  }
  for (const auto& r : c.frozen)
    if (sp.src >= r.p && sp.src + hi < r.p + r.n) return r.scope;
  return -1;
}

}  // namespace

// planes of sp from the cache (splitting them into a new entry on a miss), or
// nullptr when the source is not frozen, while recording a tape, during graph
// capture (no entry may be created there) or when the persistent budget is spent
static unsigned short* split_cached(Ctx& cx, SplitNd sp, int64_t bytes, bool tiled) {
  SplitCache& c = cx.scache;
  if (cx.tape || c.frozen.empty()) return nullptr;
  const int scope = frozen_scope(c, sp);
  if (scope < 0) return nullptr;
  for (const auto& e : c.entries)
    if (same_layout(e.key, sp)) return e.planes;
  if (scope == 0 && c.persistent_bytes + bytes > c.limit) return nullptr;
  // an arena block lives for one call only: no persistent entry from it
  if (scope == 0 && cx.pool.in_arena()) return nullptr;
  if (capturing(cx.stream)) return nullptr;
  // a cached copy never takes the last eighth of the device memory, which
  // the temporaries of the contractions need
  {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    if ((int64_t)fr < bytes + (int64_t)(tot / 8)) return nullptr;
  }
  unsigned short* dst = (unsigned short*)cx.pool.get((bytes + 15) / 16);
  sp.dst = dst;
  launch_split_nd(sp, tiled ? 1 : 0, cx.stream);
  c.entries.push_back({sp, dst, bytes, scope});
  if (scope == 0) c.persistent_bytes += bytes;
  return dst;
}

unsigned short* split_planes_cached(Ctx& cx, const SplitNd& sp, int tiled) {
  return split_cached(cx, sp, sp.rows * sp.Kp * 8, tiled != 0);
}

void split_freeze(Ctx& cx, const double2* p, int64_t n, int64_t extra_bytes) {
  if (!p || n <= 0) return;
  cx.scache.frozen.push_back({p, n, 0});
  cx.scache.limit += extra_bytes;
}

static void drop_scope(Ctx& cx, int scope) {
  SplitCache& c = cx.scache;
  std::vector<SplitCache::Entry> keep;
  for (auto& e : c.entries) {
    if (e.scope == scope) {
      cx.pool.put((double2*)e.planes);
      if (scope == 0) c.persistent_bytes -= e.bytes;
    } else {
      keep.push_back(e);
    }
  }
  c.entries.swap(keep);
  std::vector<SplitCache::Range> fr;
  for (auto& r : c.frozen)
    if (r.scope != scope) fr.push_back(r);
  c.frozen.swap(fr);
  std::vector<SplitCache::Range> only;
  for (auto& o : c.only)
    if (o.scope != scope) only.push_back(o);
  c.only.swap(only);
}

void split_thaw_all(Ctx& cx) {
  drop_scope(cx, 0);
  cx.scache.limit = 0;
}

int split_scope_begin(Ctx& cx, const std::vector<std::pair<const double2*, int64_t>>& bufs) {
  if (cx.tape) return -1;
  const int scope = cx.scache.next_scope++;
  for (auto& b : bufs)
    if (b.first && b.second > 0) cx.scache.frozen.push_back({b.first, b.second, scope});
  return scope;
}

void split_scope_end(Ctx& cx, int scope) {
  if (scope > 0) drop_scope(cx, scope);
}

void split_cache_put_rows(Ctx& cx, int scope, const double2* src, int64_t rows, int64_t K, int64_t Kp,
                          unsigned short* planes) {
  SplitNd key{};
  key.src = src;
  key.rows = rows; key.K = K; key.Kp = Kp;
  key.nm = 1; key.md[0] = rows; key.ms[0] = K;
  key.nk = 1; key.kd[0] = K; key.ks[0] = 1;
  cx.scache.entries.push_back({key, planes, rows * Kp * 8, scope});
}

void split_cache_planes_only(Ctx& cx, int scope, const double2* src, int64_t n) {
  if (scope > 0 && src && n > 0) cx.scache.only.push_back({src, n, scope});
}

bool split_planes_only(const Ctx& cx, const double2* p) {
  for (const auto& o : cx.scache.only)
    if (p >= o.p && p < o.p + o.n) return true;
  return false;
}

void split_cache_put(Ctx& cx, int scope, const double2* src, int64_t n, unsigned short* planes) {
  SplitNd key{};
  key.src = src;
  key.rows = 1; key.K = n; key.Kp = n;
  key.nm = 1; key.md[0] = 1; key.ms[0] = n;
  key.nk = 1; key.kd[0] = n; key.ks[0] = 1;
  cx.scache.entries.push_back({key, planes, n * 8, scope});
}

void ctr(Ctx& cx, cplx alpha, const Tensor& A, const char* la, bool cA, const Tensor& B, const char* lb, bool cB,
         cplx beta, Tensor& C, const char* lc) {
  if (cx.tape && cx.tape->recording) {
    TapeOp op{};
    op.kind = TapeOp::CTR;
    op.A = A; op.B = B; op.C = C; op.la = la; op.lb = lb; op.lc = lc;
    op.cA = cA; op.cB = cB; op.alpha = alpha; op.beta = beta;
    tape_record(cx, op);
  }
  if (A.f32 || B.f32) throw std::logic_error("ctr: complex64 operands are not supported");
  Pause pause(cx);
  View va = view_of(A, la), vb = view_of(B, lb), vc = view_of(C, lc);
  std::string sa(la), sb(lb), sc(lc);
  std::string bat, Ml, Nl, Kl;
  for (char c : sc) {
    const bool inA = sa.find(c) != std::string::npos, inB = sb.find(c) != std::string::npos;
    if (inA && inB) bat += c;
    else if (inA) Ml += c;
    else if (inB) Nl += c;
    else throw std::invalid_argument(std::string("ctr: output label in neither input: ") + lc);
  }
  for (char c : sa) {
    const bool inB = sb.find(c) != std::string::npos, inC = sc.find(c) != std::string::npos;
    if (inB && !inC) Kl += c;
    if (!inB && !inC) throw std::invalid_argument(std::string("ctr: label summed in A only: ") + la);
  }
  for (char c : sb) {
    const bool inA = sa.find(c) != std::string::npos, inC = sc.find(c) != std::string::npos;
    if (!inA && !inC) throw std::invalid_argument(std::string("ctr: label summed in B only: ") + lb);
  }
  auto chk = [&](char c) {
    int64_t s = -1;
    if (va.size.count(c)) s = va.size[c];
    if (vb.size.count(c)) {
      if (s >= 0 && vb.size[c] != s) throw std::invalid_argument(std::string("ctr: size mismatch on ") + c);
      s = vb.size[c];
    }
    if (vc.size.count(c) && s >= 0 && vc.size[c] != s) throw std::invalid_argument(std::string("ctr: size mismatch on ") + c);
  };
  for (char c : sa + sb) chk(c);

  // GEMM epilogues give consecutive lanes consecutive columns: when C's unit
  // stride label is a row (M) label, swap the operands so that it becomes a
  // column label and the output writes coalesce
  {
    char unit = 0;
    for (char c : sc)
      if (vc.stride.at(c) == 1 && vc.size.at(c) > 1) unit = c;
    if (unit && Ml.find(unit) != std::string::npos) {
      ctr(cx, alpha, B, lb, cB, A, la, cA, beta, C, lc);
      return;
    }
  }
  // K order: as in A
  const int64_t Mn = prod(va, Ml), Nn = prod(vb, Nl), Kn = prod(va, Kl), Bn = prod(vc, bat);
  if (Mn == 0 || Nn == 0 || Bn == 0) return;

  // Bound the temporaries: if an operand (or the output) needs a permuted copy
  // larger than kChunk elements, split the contraction along its largest label
  // (an output label when possible, so that the pieces write disjoint parts of
  // C; otherwise a summed label, accumulating with beta = 1 after the first).
  {
    const int64_t kChunk = std::max<int64_t>(1, cx.max_temp);
    const bool pA = fused_stride(va, bat) < 0 || fused_stride(va, Ml) < 0 || fused_stride(va, Kl) < 0;
    const bool pB = fused_stride(vb, bat) < 0 || fused_stride(vb, Nl) < 0 || fused_stride(vb, Kl) < 0;
    bool pC = fused_stride(vc, bat) < 0;
    {
      int64_t st0 = 0;
      int nq = 0;
      int64_t dq[3], sq[3];
      pC = pC || !group_map(vc, Ml, st0, nq, dq, sq) || !group_map(vc, Nl, st0, nq, dq, sq);
    }
    const int64_t need = std::max({pA ? A.size() : 0, pB ? B.size() : 0, pC ? C.size() : 0});
    if (need > kChunk) {
      const Tensor* X = (pA && A.size() == need) ? &A : (pB && B.size() == need) ? &B : &C;
      const std::string& sx = (X == &A) ? sa : (X == &B) ? sb : sc;
      const View& vx = (X == &A) ? va : (X == &B) ? vb : vc;
      char best = 0;
      int64_t bext = 1;
      for (int pass = 0; pass < 2 && !best; ++pass)
        for (char c : sx) {
          const bool inC = sc.find(c) != std::string::npos;
          if ((pass == 0) != inC) continue;
          if (vx.size.at(c) > bext) { bext = vx.size.at(c); best = c; }
        }
      if (best) {
        const int64_t per = std::max<int64_t>(1, X->size() / bext);
        int64_t step = std::max<int64_t>(1, kChunk / per);
        step = std::min(step, (bext + 1) / 2);
        const bool inC = sc.find(best) != std::string::npos;
        auto sl = [&](const Tensor& t, const std::string& l, int64_t lo, int64_t hi) {
          const size_t pos = l.find(best);
          return pos == std::string::npos ? t : tslice(t, (int)pos, lo, hi);
        };
        for (int64_t lo = 0; lo < bext; lo += step) {
          const int64_t hi = std::min(bext, lo + step);
          Tensor As = sl(A, sa, lo, hi), Bs = sl(B, sb, lo, hi), Cs = sl(C, sc, lo, hi);
          const cplx be = (inC || lo == 0) ? beta : C1();
          ctr(cx, alpha, As, la, cA, Bs, lb, cB, be, Cs, lc);
        }
        return;
      }
    }
  }

  GemmDesc g{};
  g.M = Mn; g.N = Nn; g.K = Kn; g.batch = Bn;
  g.alpha = alpha; g.beta = beta;
  g.conjA = cA; g.conjB = cB;

  std::vector<double2*> tmps;
  // split-bf16 mode: contractions over fewer than 32 summed elements with a
  // small output run in FP64 (one launch instead of two splits and a GEMM);
  // large ones run on the pre-split planes with K padded to 32 (bound by
  // their output, where that path is the fastest)
  struct PrecGuard {
    Ctx& cx;
    int saved;
    ~PrecGuard() { cx.prec = saved; }
  } pg{cx, cx.prec};
  if (cx.prec == 2 && Kn < 32 && Mn * Nn * Bn <= ((int64_t)1 << 20)) cx.prec = 0;
  // ---- split-bf16: unbatched contractions run on pre-split operand planes
  if ((split_planes_only(cx, A.p) || split_planes_only(cx, B.p)) && !(cx.prec == 2 && bat.empty() && Kn > 0))
    throw std::logic_error("ctr: an operand held only as split-bf16 planes");
  if (cx.prec == 2 && bat.empty() && Kn > 0) {
    const int64_t Kp = (Kn + 31) / 32 * 32;
    // K order: decreasing stride in the larger operand, so that its split
    // reads run along its unit stride where the K labels allow it
    std::string Ko = Kl;
    {
      const View& vl = A.size() >= B.size() ? va : vb;
      std::stable_sort(Ko.begin(), Ko.end(), [&](char a, char b) { return vl.stride.at(a) > vl.stride.at(b); });
    }
    std::vector<double2*> planes_tmp;
    // planes of an operand: from the split cache when the source is frozen,
    // else split into a temporary
    auto split = [&](const Tensor& X, const View& vx, const std::string& rl, bool conj,
                     int64_t rows) -> unsigned short* {
      const int64_t pbytes = rows * Kp * 8;
      SplitNd sp{};
      sp.rows = rows;
      sp.K = Kn;
      sp.Kp = Kp;
      sp.conj = conj ? 1 : 0;
      if (rows < ((int64_t)1 << 31) && Kp < ((int64_t)1 << 31) && split_digits(vx, rl, sp.nm, sp.md, sp.ms) &&
          split_digits(vx, Ko, sp.nk, sp.kd, sp.ks)) {
        sp.src = X.p;
        const bool tiled = sp.ks[sp.nk - 1] != 1 && sp.ms[sp.nm - 1] == 1;
        if (unsigned short* hit = split_cached(cx, sp, pbytes, tiled)) return hit;
        if (split_planes_only(cx, X.p)) throw std::logic_error("ctr: planes of another layout from planes-only data");
        unsigned short* dst = (unsigned short*)cx.pool.get((pbytes + 15) / 16);
        planes_tmp.push_back((double2*)dst);
        sp.dst = dst;
        launch_split_nd(sp, tiled ? 1 : 0, cx.stream);
        return dst;
      }
      // more than four digits: go through a contiguous copy
      if (split_planes_only(cx, X.p)) throw std::logic_error("ctr: planes of another layout from planes-only data");
      unsigned short* dst = (unsigned short*)cx.pool.get((pbytes + 15) / 16);
      planes_tmp.push_back((double2*)dst);
      double2* t = cx.pool.get(X.size());
      tmps.push_back(t);
      permute_into(cx, X, vx, rl + Ko, false, t, C1(), C0());
      sp.src = t;
      sp.dst = dst;
      sp.nm = 1; sp.md[0] = rows; sp.ms[0] = Kn;
      sp.nk = 1; sp.kd[0] = Kn; sp.ks[0] = 1;
      launch_split_nd(sp, 0, cx.stream);
      return dst;
    };
    unsigned short* Aq = split(A, va, Ml, cA, Mn);
    unsigned short* Bq = split(B, vb, Nl, cB, Nn);
    BfGemm g{};
    g.M = Mn; g.N = Nn; g.Kp = Kp;
    g.A = Aq; g.lda = Mn;
    g.B = Bq; g.ldb = Nn;
    g.alpha = alpha; g.beta = beta;
    int64_t scm = 0, scn = 0;
    OutMap om{};
    if (group_map(vc, Ml, scm, om.nm, om.md, om.ms) && group_map(vc, Nl, scn, om.nn, om.nd, om.ns)) {
      g.C = C.p; g.scm = scm; g.scn = scn; g.om = om;
      g.c32 = C.f32 ? 1 : 0;
      gemm_bf16p(cx, g);
    } else {
      if (C.f32) throw std::logic_error("ctr: complex64 output needs a direct output map");
      double2* t = cx.pool.get(Mn * Nn);
      tmps.push_back(t);
      g.C = t; g.scm = Nn; g.scn = 1; g.alpha = C1(); g.beta = C0();
      gemm_bf16p(cx, g);
      Tensor tt;
      tt.p = t;
      for (char c : Ml + Nl) tt.d.push_back(vc.size.at(c));
      std::string tl = Ml + Nl;
      perm(cx, alpha, tt, tl.c_str(), false, beta, C, lc);
    }
    for (auto* t : planes_tmp) cx.pool.put(t);
    for (auto* t : tmps) cx.pool.put(t);
    return;
  }
  // ---- operand A: need batch, M, K groups fusable
  {
    int64_t sbt = fused_stride(va, bat), sm = fused_stride(va, Ml), sk = fused_stride(va, Kl);
    if (sbt < 0 || sm < 0 || sk < 0) {
      double2* t = cx.pool.get(A.size());
      tmps.push_back(t);
      permute_into(cx, A, va, bat + Ml + Kl, false, t, C1(), C0());
      g.A = t; g.sab = Mn * Kn; g.sam = Kn; g.sak = 1;
    } else {
      g.A = A.p; g.sab = sbt; g.sam = sm; g.sak = sk;
    }
    if (Ml.empty()) g.sam = 0;
    if (Kl.empty()) g.sak = 0;
    if (bat.empty()) g.sab = 0;
  }
  // ---- operand B: batch, K (in A's K order), N
  {
    int64_t sbt = fused_stride(vb, bat), sn = fused_stride(vb, Nl), sk = fused_stride(vb, Kl);
    if (sbt < 0 || sn < 0 || sk < 0) {
      double2* t = cx.pool.get(B.size());
      tmps.push_back(t);
      permute_into(cx, B, vb, bat + Nl + Kl, false, t, C1(), C0());
      g.B = t; g.sbb = Nn * Kn; g.sbn = Kn; g.sbk = 1;
    } else {
      g.B = B.p; g.sbb = sbt; g.sbn = sn; g.sbk = sk;
    }
    if (Nl.empty()) g.sbn = 0;
    if (Kl.empty()) g.sbk = 0;
    if (bat.empty()) g.sbb = 0;
  }
  if (Kn == 0) {
    // empty sum: C = beta C
    if (C.f32) {
      if (beta.re == 1.0 && beta.im == 0.0) {
        // nothing to do
      } else if (beta.re == 0.0 && beta.im == 0.0 && C.st.empty()) {
        launch_fill(C.p, (C.size() + 1) / 2, C0(), cx.stream);
      } else {
        throw std::logic_error("ctr: complex64 output of an empty sum");
      }
    } else if (beta.re != 1.0 || beta.im != 0.0) {
      perm(cx, beta, C, lc, false, C0(), C, lc);
    }
  } else {
    // ---- output
    const int64_t sbt = fused_stride(vc, bat);
    int64_t sm = 0, sn = 0;
    OutMap om{};
    if (sbt >= 0 && group_map(vc, Ml, sm, om.nm, om.md, om.ms) && group_map(vc, Nl, sn, om.nn, om.nd, om.ns)) {
      g.C = C.p; g.scb = bat.empty() ? 0 : sbt; g.scm = sm; g.scn = sn; g.om = om;
      g.c32 = C.f32 ? 1 : 0;
      gemm(cx, g);
    } else {
      if (C.f32) throw std::logic_error("ctr: complex64 output needs a direct output map");
      double2* t = cx.pool.get(Bn * Mn * Nn);
      tmps.push_back(t);
      g.C = t; g.scb = Mn * Nn; g.scm = Nn; g.scn = 1;
      cplx a0 = g.alpha;
      g.alpha = C1(); g.beta = C0();
      gemm(cx, g);
      // t has labels bat+Ml+Nl contiguous
      Tensor tt;
      tt.p = t;
      for (char c : bat + Ml + Nl) tt.d.push_back(vc.size.at(c));
      std::string tl = bat + Ml + Nl;
      perm(cx, a0, tt, tl.c_str(), false, beta, C, lc);
    }
  }
  for (auto* t : tmps) cx.pool.put(t);
}

}  // namespace adc
