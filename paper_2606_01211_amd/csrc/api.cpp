// Host side of liblwe_hip: contexts, device working memory, staging of host buffers,
// launch planning and the C ABI entry points declared in include/lwe.h.
#include <errno.h>
#include <string.h>
#include <sys/random.h>

#include <algorithm>
#include <map>
#include <set>
#include <tuple>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "lwe_internal.h"

using namespace lwe;

namespace {

// batch sizes map to grid.y of the sampling and keygen kernels
constexpr size_t LWE_MAX_BATCH = 65535;
// the AES T-table every context keeps on its device
constexpr size_t T0_BYTES = 1024;

enum BufId {
  B_SEEDA, B_SEEDSK, B_Z, B_RKA, B_RK, B_X, B_E, B_E2, B_COINS, B_KP, B_HCT, B_FLAGS, B_MU2,
  B_ACC, B_PK, B_SK, B_CT, B_MU, B_SS, B_PKH, B_TEST, B_AMAT, B_CHAIN, B_ROWSUM, B_COUNT
};

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
  bool async = false;  // allocated with hipMallocAsync (freed with hipFreeAsync)
};

}  // namespace

struct lwe_ctx;
// Arguments of one host hashing function (host_hash_async).
struct HostHashJob {
  lwe_ctx* c;
  const uint8_t* src;
  size_t len, count;
  uint8_t* out;
  bool lookup, remember;
  bool operator<(const HostHashJob& o) const {
    return std::tie(src, len, count, out, lookup, remember) < std::tie(o.src, o.len, o.count, o.out, o.lookup, o.remember);
  }
};

struct lwe_ctx {
  int device = 0;
  hipStream_t own = nullptr;
  // second stream for work that overlaps the main one inside a call (decaps hashes the
  // received ciphertexts while it decrypts and re-encrypts them); created on first use
  hipStream_t side = nullptr;
  bool use_side = true;
  int hash_lanes = 2;  // lanes per record of the batched SHA3 kernel (2 or 1)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // Calls on one context reuse its buffers.  Every call records ev_done on its stream when it
  // has queued its work; a call on a different stream first waits for that event, so the
  // context's calls execute in the order they were made whatever streams they are given.
  hipEvent_t ev_done = nullptr;
  hipStream_t last = nullptr;  // stream of the previous call (null before the first)
  hipStream_t cur = nullptr;   // stream of the call in progress: orders buffer growth
  bool async_alloc = false;    // the device supports stream-ordered allocation
  size_t budget = 0;  // 0 = unlimited; bounds held
  size_t held = 0;    // device bytes held: the growable buffers plus the AES table (T0_BYTES)
  // Fixed arena (no-allocation calls): when set, buffers are carved from [arena, arena +
  // arena_cap) for the duration of one call and nothing is allocated or freed.
  uint8_t* arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  bool device_hash_only = false;  // never hash on the host (no host staging)
  uint32_t* d_T0 = nullptr;
  Buf bufs[B_COUNT];
  // cache of the last public key hashed on the host; host callbacks of queued calls read and
  // fill it on the runtime's thread, so it is guarded
  std::mutex pk_mu;
  std::vector<uint8_t> pk_cache;
  uint8_t pkh_cache[32];
  // Pinned host staging of the host hashing paths (public keys down, their hashes up), so that
  // those copies are plain asynchronous transfers rather than the runtime's staged pageable
  // copies, which serialise the host threads of concurrent contexts.  Grown on demand.
  uint8_t* hpin = nullptr;
  size_t hpin_cap = 0;
  // arguments of the queued host hashing functions (see host_hash_async)
  std::set<HostHashJob> hash_jobs;
  lwe_tuning tuning[256];
  int host_threads = 1;
  // kernel timing (lwe_prof_*): events bracketing each launch, resolved lazily
  struct ProfRec {
    const char* name;
    hipEvent_t a, b;
  };
  bool prof_on = false;
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> prof_pool;
  std::map<std::string, std::pair<uint64_t, double>> prof_agg;
};

namespace {

struct DevGuard {
  int prev = -1;
  explicit DevGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DevGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

#define HIP_CHECK(x)                          \
  do {                                        \
    hipError_t e_ = (x);                      \
    if (e_ != hipSuccess) return LWE_EDEVICE; \
  } while (0)

#define LWE_CHECK(x)          \
  do {                        \
    int s_ = (x);             \
    if (s_ != LWE_OK) return s_; \
  } while (0)

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.isManaged;
}

// Returns a device buffer of at least `bytes`, growing it when needed.
int ensure(lwe_ctx* c, BufId id, size_t bytes, void** out) {
  Buf& b = c->bufs[id];
  if (bytes == 0) bytes = 16;
  if (c->arena) {
    // carve from the fixed arena; a buffer asked for again in the same call keeps its region
    if (b.cap < bytes) {
      const size_t off = (c->arena_used + 255) & ~(size_t)255;
      if (off > c->arena_cap || bytes > c->arena_cap - off) return LWE_ENOMEM;
      b.p = c->arena + off;
      b.cap = bytes;
      c->arena_used = off + bytes;
    }
    *out = b.p;
    return LWE_OK;
  }
  if (b.cap < bytes) {
    size_t want = std::max(bytes, b.cap + b.cap / 2);
    want = (want + 255) & ~(size_t)255;
    if (c->budget && c->held - b.cap + want > c->budget) {
      want = (bytes + 255) & ~(size_t)255;
      if (c->held - b.cap + want > c->budget) return LWE_ENOMEM;
    }
    if (b.p) {
      // The old buffer may still be read by queued work of this context.  All of it is
      // ordered before the current call's stream (CallScope), so it is freed in that stream's
      // order; without stream-ordered allocation the device is drained first.
      if (b.async && c->cur) {
        if (hipFreeAsync(b.p, c->cur) != hipSuccess) return LWE_EDEVICE;
      } else {
        if (hipDeviceSynchronize() != hipSuccess) return LWE_EDEVICE;
        (void)hipFree(b.p);
      }
      c->held -= b.cap;
      b.p = nullptr;
      b.cap = 0;
    }
    const bool async = c->async_alloc && c->cur;
    if ((async ? hipMallocAsync(&b.p, want, c->cur) : hipMalloc(&b.p, want)) != hipSuccess) {
      (void)hipGetLastError();
      b.p = nullptr;
      return LWE_ENOMEM;
    }
    b.async = async;
    b.cap = want;
    c->held += want;
  }
  *out = b.p;
  return LWE_OK;
}

template <class T>
int ensure_t(lwe_ctx* c, BufId id, size_t bytes, T** out) {
  void* p = nullptr;
  int s = ensure(c, id, bytes, &p);
  *out = (T*)p;
  return s;
}

// Device view of a caller input: the pointer itself if it is device memory, otherwise a
// copy in buffer `id`.
int stage_in(lwe_ctx* c, BufId id, const void* src, size_t bytes, hipStream_t s, const uint8_t** dev) {
  if (is_device_ptr(src)) {
    *dev = (const uint8_t*)src;
    return LWE_OK;
  }
  uint8_t* d = nullptr;
  LWE_CHECK(ensure_t(c, id, bytes, &d));
  HIP_CHECK(hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, s));
  *dev = d;
  return LWE_OK;
}

// Host copies of two caller buffers (either may be on the device) with a single wait.
int host_copy2(const void* a, size_t na, std::vector<uint8_t>& oa, const void* b, size_t nb,
               std::vector<uint8_t>& ob, hipStream_t s) {
  oa.resize(na);
  ob.resize(nb);
  bool wait = false;
  if (is_device_ptr(a)) {
    HIP_CHECK(hipMemcpyAsync(oa.data(), a, na, hipMemcpyDeviceToHost, s));
    wait = true;
  } else {
    memcpy(oa.data(), a, na);
  }
  if (is_device_ptr(b)) {
    HIP_CHECK(hipMemcpyAsync(ob.data(), b, nb, hipMemcpyDeviceToHost, s));
    wait = true;
  } else {
    memcpy(ob.data(), b, nb);
  }
  if (wait) HIP_CHECK(hipStreamSynchronize(s));
  return LWE_OK;
}

// The context's pinned staging, at least `bytes`.  The host writes into it only after a wait
// on the calling stream (which the call scope orders after every earlier call of the
// context), so no queued copy still reads what it overwrites; growing it waits the same way.
int host_pinned(lwe_ctx* c, size_t bytes, hipStream_t s, uint8_t** out) {
  if (c->hpin_cap < bytes) {
    const size_t want = (std::max(bytes, 2 * c->hpin_cap) + 4095) & ~(size_t)4095;
    if (c->hpin) {
      HIP_CHECK(hipStreamSynchronize(s));
      (void)hipHostFree(c->hpin);
      c->hpin = nullptr;
      c->hpin_cap = 0;
    }
    if (hipHostMalloc((void**)&c->hpin, want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      c->hpin = nullptr;
      return LWE_ENOMEM;
    }
    c->hpin_cap = want;
  }
  *out = c->hpin;
  return LWE_OK;
}

// Host copy of a caller buffer (which may be on the device); synchronises when copying.
int host_copy(const void* src, size_t bytes, hipStream_t s, std::vector<uint8_t>& out) {
  out.resize(bytes);
  if (is_device_ptr(src)) {
    HIP_CHECK(hipMemcpyAsync(out.data(), src, bytes, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
  } else {
    memcpy(out.data(), src, bytes);
  }
  return LWE_OK;
}

struct OutStage {
  void* user = nullptr;
  uint8_t* dev = nullptr;
  size_t bytes = 0;
  bool host = false;
};

int stage_out(lwe_ctx* c, BufId id, void* user, size_t bytes, OutStage& o) {
  o.user = user;
  o.bytes = bytes;
  o.host = !is_device_ptr(user);
  if (o.host) {
    LWE_CHECK(ensure_t(c, id, bytes, &o.dev));
  } else {
    o.dev = (uint8_t*)user;
  }
  return LWE_OK;
}

int finish_out(const OutStage& o, hipStream_t s) {
  if (o.host && o.bytes) HIP_CHECK(hipMemcpyAsync(o.user, o.dev, o.bytes, hipMemcpyDeviceToHost, s));
  return LWE_OK;
}

hipStream_t pick_stream(lwe_ctx* c, void* user) { return user ? (hipStream_t)user : c->own; }

// Brackets one entry point: orders it after the context's previous call when that call used
// another stream, and marks the end of its work on its own stream for the next call.
struct CallScope {
  lwe_ctx* c;
  hipStream_t s;
  hipStream_t outer;
  int status = LWE_OK;
  CallScope(lwe_ctx* c_, hipStream_t s_) : c(c_), s(s_), outer(c_->cur) {
    if (c->last && c->last != s && hipStreamWaitEvent(s, c->ev_done, 0) != hipSuccess) status = LWE_EDEVICE;
    c->cur = s;
  }
  ~CallScope() {
    if (c->ev_done && hipEventRecord(c->ev_done, s) == hipSuccess) c->last = s;
    c->cur = outer;
  }
};

#define CALL_SCOPE(c, s)                 \
  CallScope call_scope_(c, s);           \
  LWE_CHECK(call_scope_.status)

hipEvent_t prof_event(lwe_ctx* c) {
  if (!c->prof_pool.empty()) {
    hipEvent_t e = c->prof_pool.back();
    c->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one kernel launch with events when profiling is on.
struct ProfScope {
  lwe_ctx* c;
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(lwe_ctx* c_, const char* n, hipStream_t s_) : c(c_), name(n), s(s_) {
    if (c->prof_on && (a = prof_event(c)) != nullptr) (void)hipEventRecord(a, s);
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = prof_event(c);
    if (!b) return;
    (void)hipEventRecord(b, s);
    c->prof_pending.push_back({name, a, b});
  }
};

int prof_resolve(lwe_ctx* c) {
  for (auto& r : c->prof_pending) {
    if (hipEventSynchronize(r.b) != hipSuccess) return LWE_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return LWE_EDEVICE;
    auto& agg = c->prof_agg[r.name];
    agg.first += 1;
    agg.second += ms;
    c->prof_pool.push_back(r.a);
    c->prof_pool.push_back(r.b);
  }
  c->prof_pending.clear();
  return LWE_OK;
}

#define KLAUNCH(name, s, x)          \
  do {                               \
    ProfScope ps_(c, name, s);       \
    HIP_CHECK(x);                    \
  } while (0)

// Parallel loop over [0, count) on host threads (used for host-side hashing).
template <class F>
void host_for(int threads, size_t count, F f) {
  if (threads <= 1 || count < 4) {
    for (size_t i = 0; i < count; ++i) f(i);
    return;
  }
  const int nt = (int)std::min<size_t>((size_t)threads, count);
  std::vector<std::thread> th;
  th.reserve(nt);
  for (int t = 0; t < nt; ++t)
    th.emplace_back([=, &f]() {
      for (size_t i = t; i < count; i += nt) f(i);
    });
  for (auto& x : th) x.join();
}

const lwe_tuning& tuning_of(lwe_ctx* c, int pid) { return c->tuning[pid & 255]; }

bool use_host_hash(lwe_ctx* c, int pid, size_t count) {
  if (c->device_hash_only) return false;
  const lwe_tuning& t = tuning_of(c, pid);
  const size_t lim = t.host_hash_max ? t.host_hash_max : 16;
  return count <= lim;
}

// ------------------------------------------------------------------------------------
// Product launch planning
// ------------------------------------------------------------------------------------
// The strip product (large row counts) reads S' in fragment order; the streaming one row-major.
bool uses_strip(int M, bool trans, bool per_inst_A) { return !trans && !per_inst_A && M >= 256; }

// Launch shape of one product.  plan_product fills the tiling fields of ProdArgs (K chunks,
// column and row tiles); exec_product launches it.  A contraction split into K chunks needs a
// zeroed int32 accumulator of acc_bytes, given in a.acc32 before exec_product.
struct ProdPlan {
  bool strip = false;
  int CG = 1, RG = 1, W = 1, KS = 1, unr = 3;
  size_t acc_bytes = 0;
};

ProdPlan plan_product(lwe_ctx* c, int pid, const Params& p, ProdArgs& a, bool trans) {
  ProdPlan pl;
  const int ksteps = (p.n + 63) / 64;
  const lwe_tuning& tu = tuning_of(c, pid);
  // the paper's sets (prime q) run on the streaming kernel only
  pl.strip = !p.paper && uses_strip(a.M, trans, a.per_inst_A != 0);
  if (!pl.strip) {
    int RG = 1;
    if (!a.per_inst_A) RG = a.M <= 16 ? 1 : (a.M <= 32 ? 2 : 4);
    const int CG = 1;
    a.m_tile = a.per_inst_A ? p.nbar : 16 * RG;
    a.n_mt = a.per_inst_A ? a.M / p.nbar : (a.M + a.m_tile - 1) / a.m_tile;
    a.n_jt = (a.ncols + 16 * CG - 1) / (16 * CG);
    const long long units = (long long)a.n_jt * a.n_mt * ksteps;
    int KS = (int)std::max<long long>(1, (units + 65535) / 65536);
    int W = std::min(16, (ksteps + KS - 1) / KS);
    a.n_kc = (ksteps + W * KS - 1) / (W * KS);
    W = (ksteps + a.n_kc * KS - 1) / (a.n_kc * KS);
    a.kc_len = W * KS * 64;
    pl.CG = CG;
    pl.RG = RG;
    pl.W = W;
    pl.KS = KS;
  } else {
    // Default tile: the widest strip of A that fits LDS over the whole contraction (fewer
    // re-reads of the S' stack), and one row chunk per XCD so that all workgroups of an XCD
    // stream the same rows of S' through that XCD's L2.
    int CG = (int)tu.col_groups;
    if (!CG) {
      CG = 1;
      for (int cg = 3; cg >= 1; --cg)
        if (product_strip_lds_bytes(cg, ksteps * 64, 3) <= 160 * 1024) {
          CG = cg;
          break;
        }
    }
    int RG = tu.row_groups ? (int)tu.row_groups : (CG >= 3 ? 2 : 4);
    if (!product_strip_shape_ok(CG, RG)) {  // a shape the library does not build
      CG = CG >= 3 ? 3 : CG;
      RG = CG >= 2 ? 2 : 4;
    }
    // longest K chunk whose padded strip fits LDS (a multiple of three 64-row steps)
    const int max_rows = (int)(((160 * 1024 - 4096) / (32 * CG)) / 192 * 192);
    a.kc_len = std::min(ksteps * 64, max_rows);
    a.n_kc = (p.n + a.kc_len - 1) / a.kc_len;
    // a deeper loop unroll (longer X prefetch) when it adds no padding and still fits LDS
    int unr = a.n_kc == 1 ? product_strip_unroll(CG, RG, a.kc_len) : 3;
    if (product_strip_lds_bytes(CG, a.kc_len, unr) > 160 * 1024) unr = 3;
    a.n_jt = (a.ncols + 16 * CG - 1) / (16 * CG);
    int mch = tu.m_chunks ? (int)tu.m_chunks : 8;
    const int unit = 16 * RG;
    const int m_units = (a.M + unit - 1) / unit;
    mch = std::min(mch, m_units);
    a.m_tile = ((m_units + mch - 1) / mch) * unit;
    a.n_mt = (a.M + a.m_tile - 1) / a.m_tile;
    pl.CG = CG;
    pl.RG = RG;
    pl.unr = unr;
  }
  if (a.n_kc > 1) {
    a.acc_ld = a.ncols;
    pl.acc_bytes = (size_t)a.M * a.acc_ld * 4;
  }
  return pl;
}

int exec_product(lwe_ctx* c, const ProdPlan& pl, const ProdArgs& a, bool trans, hipStream_t s) {
  if (a.n_kc > 1) KLAUNCH("fill", s, launch_fill_u32((uint32_t*)a.acc32, (size_t)a.M * a.acc_ld, 0, s));
  if (!pl.strip) {
    KLAUNCH("prod_stream", s, launch_product_stream(a, pl.CG, pl.RG, pl.W, trans, a.n_mt, pl.KS, s));
  } else {
    // timed under separate names: the compare launch of a decapsulation shares the GPU with its
    // concurrent hash
    KLAUNCH(a.mode == PM_COMPARE ? "prod_strip_cmp" : "prod_strip", s,
            launch_product_strip(a, pl.CG, pl.RG, pl.unr, s));
  }
  if (a.n_kc > 1) KLAUNCH("finalize", s, launch_finalize(a, s));
  return LWE_OK;
}

int run_product(lwe_ctx* c, int pid, const Params& p, ProdArgs a, bool trans, hipStream_t s) {
  // a: operands, epilogue fields, M and ncols are filled in by the caller
  const lwe_tuning& tu = tuning_of(c, pid);
  // Unfused variant: expand A once into device memory and let the product read it (one A per
  // call, so not for key-generation batches, where every instance has its own A).
  if (tu.a_source == 1 && !p.paper && (!a.per_inst_A || a.M == 8)) {
    uint16_t* Am;
    LWE_CHECK(ensure_t(c, B_AMAT, (size_t)p.n * p.n * 2, &Am));
    KLAUNCH("expand_A", s, launch_expand_A(p, a.rkA, a.T0, 0, (uint32_t)p.n, Am, s));
    a.Amat = Am;
  }
  const ProdPlan pl = plan_product(c, pid, p, a, trans);
  if (pl.acc_bytes) LWE_CHECK(ensure_t(c, B_ACC, pl.acc_bytes, &a.acc32));
  return exec_product(c, pl, a, trans, s);
}

// ------------------------------------------------------------------------------------
// Core operations on device-resident data
// ------------------------------------------------------------------------------------

// Encrypt `count` messages under one public key with per-instance coins already expanded
// into round keys at d_rk.  Writes ct records (or, in compare mode, sets flags).
int encrypt_core(lwe_ctx* c, int pid, const Params& p, size_t count, const uint8_t* pk_dev,
                 const uint32_t* d_rk, const uint8_t* mu_dev, size_t mu_stride, uint8_t* ct_out,
                 const uint8_t* ct_cmp, uint32_t* flags, hipStream_t s) {
  const int n = p.n;
  int8_t *X, *E, *E2;
  uint32_t* rkA;
  const bool frag = uses_strip((int)(count * 8), false, false);
  // fragment order covers whole 16-row groups
  LWE_CHECK(ensure_t(c, B_X, (count * 8 + 15) / 16 * 16 * (size_t)p.ldx, &X));
  LWE_CHECK(ensure_t(c, B_E, count * 8 * (size_t)n, &E));
  LWE_CHECK(ensure_t(c, B_E2, count * 64, &E2));
  LWE_CHECK(ensure_t(c, B_RKA, 44 * 4, &rkA));
  KLAUNCH("expand_keys", s, launch_expand_keys(pk_dev, 0, 1, c->d_T0, rkA, s));
  SampleArgs sa;
  memset(&sa, 0, sizeof(sa));
  sa.rk = d_rk;
  sa.T0 = c->d_T0;
  sa.n = n;
  sa.K = p.K;
  sa.ldx = p.ldx;
  sa.nseg = 3;
  for (int k = 0; k < MAX_K; ++k) sa.T2[k] = (uint32_t)p.T[k] * 0x10001u;
  sa.X = X;
  sa.x_frag = frag ? 1 : 0;
  sa.E = E;
  sa.E2 = E2;
  KLAUNCH("sample", s, launch_sample(sa, (int)count, s));
  ProdArgs a;
  memset(&a, 0, sizeof(a));
  a.rkA = rkA;
  a.T0 = c->d_T0;
  a.X = X;
  a.ldx = p.ldx;
  a.M = (int)(count * 8);
  a.n = n;
  a.logq = p.logq;
  a.B = p.B;
  a.ncols = n + 8;
  a.Bt = pk_dev + 16;
  a.mode = ct_cmp ? PM_COMPARE : PM_ENCRYPT;
  a.E = E;
  a.E2 = E2;
  a.mu = mu_dev;
  a.mu_stride = mu_stride;
  a.out = ct_out;
  a.out_stride = p.ct_bytes;
  a.out_off = 0;
  a.cmp = ct_cmp;
  a.cmp_stride = p.ct_bytes;
  a.flags = flags;
  return run_product(c, pid, p, a, false, s);
}

int check_pid(int pid, const Params** pp) {
  const Params* p = get_params(pid);
  if (!p) return LWE_EINVAL;
  *pp = p;
  return LWE_OK;
}

void host_pkh(lwe_ctx* c, const uint8_t* pk, size_t len, uint8_t out[32]) {
  std::lock_guard<std::mutex> lk(c->pk_mu);
  if (c->pk_cache.size() == len && memcmp(c->pk_cache.data(), pk, len) == 0) {
    memcpy(out, c->pkh_cache, 32);
    return;
  }
  sha3_256(pk, len, out);
  c->pk_cache.assign(pk, pk + len);
  memcpy(c->pkh_cache, out, 32);
}

// Host hashing in stream order: a host function queued on the stream hashes `count` records of
// `len` bytes at `src` (pinned staging, filled by a copy queued before it) into `out` (pinned
// staging, read by a copy queued after it).  The calling thread does not wait for the device:
// under load a small copy can take milliseconds to be scheduled, and a caller blocked on it
// cannot queue its next work meanwhile.  `lookup`: one public key, hashed through the cache;
// `remember`: the last record becomes the cached key.  The function runs on the runtime's
// thread and makes no runtime calls.  Its arguments are a job owned by the context, one per
// distinct set of arguments, never changed and kept until the context is destroyed: a call
// captured into a graph runs the same job at every replay.
void host_hash_cb(void* arg) {
  const HostHashJob* j = (const HostHashJob*)arg;
  if (j->lookup) {
    host_pkh(j->c, j->src, j->len, j->out);
  } else {
    host_for(j->c->host_threads, j->count, [&](size_t i) { sha3_256(j->src + i * j->len, j->len, j->out + i * 32); });
    if (j->remember) {
      std::lock_guard<std::mutex> lk(j->c->pk_mu);
      j->c->pk_cache.assign(j->src + (j->count - 1) * j->len, j->src + j->count * j->len);
      memcpy(j->c->pkh_cache, j->out + (j->count - 1) * 32, 32);
    }
  }
}

int host_hash_async(lwe_ctx* c, const uint8_t* src, size_t len, size_t count, uint8_t* out, bool lookup,
                    bool remember, hipStream_t s) {
  const HostHashJob key{c, src, len, count, out, lookup, remember};
  const HostHashJob* j = &*c->hash_jobs.insert(key).first;
  HIP_CHECK(hipLaunchHostFunc(s, host_hash_cb, (void*)j));
  return LWE_OK;
}

// ------------------------------------------------------------------------------------
// The paper's own sets (Table 1): one encryption per message bit, prime q, noise from the
// AES-256 CTR_DRBG.  Hashing (H(pk), coins, K', H(ct), K) stays on the host: a ciphertext is
// 256 (n + 1) coefficients (0.26 to 32 MB), a single sponge chain too long for one device lane.
// ------------------------------------------------------------------------------------
constexpr size_t DRBG_REQ_BYTES = (size_t)DRBG_REQ_BLOCKS * 16;

// Generate requests of one noise stream of `words` 16-bit words
int drbg_requests(size_t words) { return (int)((2 * words + DRBG_REQ_BYTES - 1) / DRBG_REQ_BYTES); }

// Runs the DRBG chains of `count` instances (keys [count][16] on the device) for `nseg`
// streams of the given word counts, then samples them into the destinations of `sa`
// (dist, rowlen, dst8, inst_stride8, ld8, dst16 filled in by the caller).
int pb_noise(lwe_ctx* c, const Params& p, size_t count, const uint8_t* dkeys, int nseg, const size_t words[3],
             PbSampleArgs& sa, hipStream_t s) {
  PbChainArgs ca;
  memset(&ca, 0, sizeof(ca));
  ca.nseg = nseg;
  int rmax = 1;
  for (int k = 0; k < nseg; ++k) {
    ca.domain[k] = (uint32_t)(k + 1);
    ca.requests[k] = drbg_requests(words[k]);
    rmax = std::max(rmax, ca.requests[k]);
  }
  ca.rmax = rmax;
  uint32_t* chain;
  LWE_CHECK(ensure_t(c, B_CHAIN, count * nseg * (size_t)rmax * 64 * 4, &chain));
  KLAUNCH("drbg_chain", s, launch_drbg_chain(dkeys, 16, (int)count, ca, c->d_T0, chain, s));
  sa.count = (int)count;
  sa.nseg = nseg;
  sa.rmax = rmax;
  for (int k = 0; k < nseg; ++k) sa.blocks[k] = (uint32_t)(words[k] / 8);
  sa.eta = p.eta;
  sa.ku = p.ku;
  sa.K = p.K;
  for (int k = 0; k <= MAX_K; ++k) sa.T[k] = p.T[k];
  KLAUNCH("pb_sample", s, launch_pb_sample(sa, c->d_T0, chain, s));
  return LWE_OK;
}

ProdArgs pb_prod_args(lwe_ctx* c, const Params& p) {
  ProdArgs a;
  memset(&a, 0, sizeof(a));
  a.T0 = c->d_T0;
  a.ldx = p.ldx;
  a.n = p.n;
  a.logq = p.logq;
  a.B = p.B;
  a.qp = p.q;
  a.qp_magic = p.q < 65536 ? (uint32_t)((1ull << 32) / p.q + 1) : 0u;
  a.coef_bytes = p.coef_bytes;
  return a;
}

// Encryption of count messages under one public key (device pk record) with per-instance
// coins [count][16] on the device: u_r = A^T r_r + e1_r and v_r = t^T r_r + e2_r + m_r
// round(q/2) for r < 256 (Alg. 2 once per bit).  Writes ct records, or in compare mode sets
// flags for records that differ from ct_cmp.
int pb_encrypt_core(lwe_ctx* c, int pid, const Params& p, size_t count, const uint8_t* pk_dev, const uint8_t* dcoins,
                    const uint8_t* mu_dev, size_t mu_stride, uint8_t* ct_out, const uint8_t* ct_cmp, uint32_t* flags,
                    hipStream_t s) {
  const size_t n = (size_t)p.n, rows = count * PB_BITS;
  int8_t *X, *E, *E2;
  int32_t* rowsum;
  uint32_t* rkA;
  LWE_CHECK(ensure_t(c, B_X, rows * p.ldx, &X));
  LWE_CHECK(ensure_t(c, B_E, rows * n, &E));
  LWE_CHECK(ensure_t(c, B_E2, count * PB_BITS, &E2));
  LWE_CHECK(ensure_t(c, B_ROWSUM, rows * 4, &rowsum));
  LWE_CHECK(ensure_t(c, B_RKA, 44 * 4, &rkA));
  KLAUNCH("expand_keys", s, launch_expand_keys(pk_dev, 0, 1, c->d_T0, rkA, s));
  // r_r (domain 1, Gaussian), e1_r (domain 2, Gaussian), e2 (domain 3, uniform)
  PbSampleArgs sa;
  memset(&sa, 0, sizeof(sa));
  const size_t words[3] = {rows * n, rows * n, count * PB_BITS};
  sa.dist[0] = 1;
  sa.dist[1] = 1;
  sa.dist[2] = 2;
  sa.rowlen[0] = sa.rowlen[1] = p.n;
  sa.rowlen[2] = PB_BITS;
  sa.dst8[0] = X;
  sa.inst_stride8[0] = (size_t)PB_BITS * p.ldx;
  sa.ld8[0] = p.ldx;
  sa.dst8[1] = E;
  sa.inst_stride8[1] = (size_t)PB_BITS * n;
  sa.ld8[1] = p.n;
  sa.dst8[2] = E2;
  sa.inst_stride8[2] = PB_BITS;
  sa.ld8[2] = PB_BITS;
  const size_t per_inst[3] = {words[0] / count, words[1] / count, words[2] / count};
  LWE_CHECK(pb_noise(c, p, count, dcoins, 3, per_inst, sa, s));
  // row sums of r (limb correction) and v_r
  PbRowsArgs ra;
  memset(&ra, 0, sizeof(ra));
  ra.X = X;
  ra.ldx = p.ldx;
  ra.n = p.n;
  ra.rows = (int)rows;
  ra.rows_per_inst = PB_BITS;
  ra.rowsum = rowsum;
  ra.mode = ct_cmp ? 2 : 1;
  ra.t = pk_dev + 16;
  ra.coef_bytes = p.coef_bytes;
  ra.e2 = E2;
  ra.mu = mu_dev;
  ra.mu_stride = mu_stride;
  ra.q = p.q;
  ra.out = ct_out;
  ra.out_stride = p.ct_bytes;
  ra.v_off = (size_t)p.coef_bytes * PB_BITS * n;
  ra.cmp = ct_cmp;
  ra.cmp_stride = p.ct_bytes;
  ra.flags = flags;
  KLAUNCH("pb_rows", s, launch_pb_rows(ra, s));
  ProdArgs a = pb_prod_args(c, p);
  a.rkA = rkA;
  a.X = X;
  a.M = (int)rows;
  a.ncols = p.n;
  a.mode = ct_cmp ? PM_COMPARE : PM_ENCRYPT;
  a.E = E;
  a.out = ct_out;
  a.out_stride = p.ct_bytes;
  a.cmp = ct_cmp;
  a.cmp_stride = p.ct_bytes;
  a.flags = flags;
  a.rowsum = rowsum;
  a.rows_per_inst = PB_BITS;
  return run_product(c, pid, p, a, false, s);
}

int pb_keygen(lwe_ctx* c, int pid, const Params& p, size_t count, const uint8_t* seedA, const uint8_t* seedSK,
              const uint8_t* z, uint8_t* pk, uint8_t* sk, void* stream) {
  DevGuard g(c->device);
  hipStream_t s = pick_stream(c, stream);
  CALL_SCOPE(c, s);
  const size_t n = (size_t)p.n;
  const uint8_t *dA, *dS, *dZ;
  LWE_CHECK(stage_in(c, B_SEEDA, seedA, count * 16, s, &dA));
  LWE_CHECK(stage_in(c, B_SEEDSK, seedSK, count * 16, s, &dS));
  LWE_CHECK(stage_in(c, B_Z, z, count * 32, s, &dZ));
  OutStage opk, osk;
  LWE_CHECK(stage_out(c, B_PK, pk, count * p.pk_bytes, opk));
  LWE_CHECK(stage_out(c, B_SK, sk, count * p.sk_bytes, osk));
  uint32_t* rkA;
  int8_t *X, *E;
  int32_t* rowsum;
  LWE_CHECK(ensure_t(c, B_RKA, count * 44 * 4, &rkA));
  LWE_CHECK(ensure_t(c, B_X, count * (size_t)p.ldx, &X));
  LWE_CHECK(ensure_t(c, B_E, count * n, &E));
  LWE_CHECK(ensure_t(c, B_ROWSUM, count * 4, &rowsum));
  KLAUNCH("expand_keys", s, launch_expand_keys(dA, 16, (int)count, c->d_T0, rkA, s));
  // s (domain 1, binomial; also as int16 at the start of sk), e (domain 2, Gaussian)
  PbSampleArgs sa;
  memset(&sa, 0, sizeof(sa));
  const size_t words[3] = {n, n, 0};
  sa.dist[0] = 0;
  sa.dist[1] = 1;
  sa.rowlen[0] = sa.rowlen[1] = p.n;
  sa.dst8[0] = X;
  sa.inst_stride8[0] = (size_t)p.ldx;
  sa.ld8[0] = p.ldx;
  sa.dst8[1] = E;
  sa.inst_stride8[1] = n;
  sa.ld8[1] = p.n;
  sa.dst16 = osk.dev;
  sa.dst16_stride = p.sk_bytes;
  LWE_CHECK(pb_noise(c, p, count, dS, 2, words, sa, s));
  PbRowsArgs ra;
  memset(&ra, 0, sizeof(ra));
  ra.X = X;
  ra.ldx = p.ldx;
  ra.n = p.n;
  ra.rows = (int)count;
  ra.rows_per_inst = 1;
  ra.rowsum = rowsum;
  KLAUNCH("pb_rows", s, launch_pb_rows(ra, s));
  // t = A s + e mod q (every instance its own A)
  ProdArgs a = pb_prod_args(c, p);
  a.rkA = rkA;
  a.X = X;
  a.M = (int)count;
  a.ncols = p.n;
  a.per_inst_A = 1;
  a.mode = PM_KEYGEN;
  a.E = E;
  a.out = opk.dev;
  a.out_stride = p.pk_bytes;
  a.out_off = 16;
  a.rowsum = rowsum;
  a.rows_per_inst = 1;
  LWE_CHECK(run_product(c, pid, p, a, true, s));
  // pk = seedA || t ; sk = s || pk || H(pk) || z
  HIP_CHECK(hipMemcpy2DAsync(opk.dev, p.pk_bytes, dA, 16, 16, count, hipMemcpyDeviceToDevice, s));
  const size_t off_pk = 2 * n, off_pkh = off_pk + p.pk_bytes, off_z = off_pkh + 32;
  HIP_CHECK(hipMemcpy2DAsync(osk.dev + off_pk, p.sk_bytes, opk.dev, p.pk_bytes, p.pk_bytes, count,
                             hipMemcpyDeviceToDevice, s));
  HIP_CHECK(hipMemcpy2DAsync(osk.dev + off_z, p.sk_bytes, dZ, 32, 32, count, hipMemcpyDeviceToDevice, s));
  std::vector<uint8_t> hpk(count * p.pk_bytes), hh(count * 32);
  HIP_CHECK(hipMemcpyAsync(hpk.data(), opk.dev, hpk.size(), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  host_for(c->host_threads, count,
           [&](size_t i) { sha3_256(hpk.data() + i * p.pk_bytes, p.pk_bytes, hh.data() + i * 32); });
  uint8_t* dh;
  LWE_CHECK(ensure_t(c, B_HCT, count * 32, &dh));
  HIP_CHECK(hipMemcpyAsync(dh, hh.data(), hh.size(), hipMemcpyHostToDevice, s));
  HIP_CHECK(hipMemcpy2DAsync(osk.dev + off_pkh, p.sk_bytes, dh, 32, 32, count, hipMemcpyDeviceToDevice, s));
  LWE_CHECK(finish_out(opk, s));
  LWE_CHECK(finish_out(osk, s));
  HIP_CHECK(hipStreamSynchronize(s));  // hh must outlive the copy
  return LWE_OK;
}

int pb_encaps(lwe_ctx* c, int pid, const Params& p, size_t count, const uint8_t* pk, const uint8_t* mu, uint8_t* ct,
              uint8_t* ss, void* stream) {
  DevGuard g(c->device);
  hipStream_t s = pick_stream(c, stream);
  CALL_SCOPE(c, s);
  const size_t mb = p.mu_bytes;
  std::vector<uint8_t> hpk, hmu;
  LWE_CHECK(host_copy2(pk, p.pk_bytes, hpk, mu, count * mb, hmu, s));
  uint8_t pkh[32];
  host_pkh(c, hpk.data(), p.pk_bytes, pkh);
  const uint8_t *dpk, *dmu;
  LWE_CHECK(stage_in(c, B_PK, pk, p.pk_bytes, s, &dpk));
  LWE_CHECK(stage_in(c, B_MU, mu, count * mb, s, &dmu));
  OutStage oct;
  LWE_CHECK(stage_out(c, B_CT, ct, count * p.ct_bytes, oct));
  uint8_t* dcoins;
  LWE_CHECK(ensure_t(c, B_COINS, count * 16, &dcoins));
  std::vector<uint8_t> hcoins(count * 16), hkp(count * 32);
  const uint8_t one = 1;
  host_for(c->host_threads, count, [&](size_t i) {
    uint8_t h[32];
    sha3_256_3(&one, 1, pkh, 32, hmu.data() + i * mb, mb, h);
    memcpy(hcoins.data() + i * 16, h, 16);
    sha3_256_3(pkh, 32, hmu.data() + i * mb, mb, nullptr, 0, hkp.data() + i * 32);
  });
  HIP_CHECK(hipMemcpyAsync(dcoins, hcoins.data(), count * 16, hipMemcpyHostToDevice, s));
  LWE_CHECK(pb_encrypt_core(c, pid, p, count, dpk, dcoins, dmu, mb, oct.dev, nullptr, nullptr, s));
  std::vector<uint8_t> hct(count * p.ct_bytes), hss(count * 32);
  HIP_CHECK(hipMemcpyAsync(hct.data(), oct.dev, hct.size(), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  host_for(c->host_threads, count, [&](size_t i) {
    uint8_t h[32];
    sha3_256(hct.data() + i * p.ct_bytes, p.ct_bytes, h);
    sha3_256_3(hkp.data() + i * 32, 32, h, 32, nullptr, 0, hss.data() + i * 32);
  });
  if (oct.host) {
    memcpy(ct, hct.data(), hct.size());
    oct.bytes = 0;
  }
  if (is_device_ptr(ss)) {
    HIP_CHECK(hipMemcpyAsync(ss, hss.data(), hss.size(), hipMemcpyHostToDevice, s));
    HIP_CHECK(hipStreamSynchronize(s));
  } else {
    memcpy(ss, hss.data(), hss.size());
  }
  return LWE_OK;
}

int pb_decaps(lwe_ctx* c, int pid, const Params& p, size_t count, const uint8_t* sk, const uint8_t* ct, uint8_t* ss,
              void* stream) {
  DevGuard g(c->device);
  hipStream_t s = pick_stream(c, stream);
  CALL_SCOPE(c, s);
  const size_t n = (size_t)p.n, mb = p.mu_bytes;
  const size_t off_pk = 2 * n, off_pkh = off_pk + p.pk_bytes;
  const uint8_t *dsk, *dct;
  LWE_CHECK(stage_in(c, B_SK, sk, p.sk_bytes, s, &dsk));
  LWE_CHECK(stage_in(c, B_CT, ct, count * p.ct_bytes, s, &dct));
  uint8_t *dmu2, *dcoins;
  uint32_t* dflags;
  LWE_CHECK(ensure_t(c, B_MU2, count * mb, &dmu2));
  LWE_CHECK(ensure_t(c, B_COINS, count * 16, &dcoins));
  LWE_CHECK(ensure_t(c, B_FLAGS, count * 4, &dflags));
  // m' = Decrypt(sk, ct) (Alg. 3)
  PbDecArgs da;
  da.ct = dct;
  da.ct_stride = p.ct_bytes;
  da.sk = dsk;
  da.n = p.n;
  da.q = p.q;
  da.coef_bytes = p.coef_bytes;
  da.count = (int)count;
  da.mu_out = dmu2;
  KLAUNCH("pb_decrypt", s, launch_pb_decrypt(da, s));
  // coins' and K'' of m' on the host; the received ciphertexts come back in the same wait
  std::vector<uint8_t> hmu(count * mb), tail(64), hct(count * p.ct_bytes);
  HIP_CHECK(hipMemcpyAsync(hmu.data(), dmu2, hmu.size(), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(tail.data(), dsk + off_pkh, 64, hipMemcpyDeviceToHost, s));
  if (is_device_ptr(ct))
    HIP_CHECK(hipMemcpyAsync(hct.data(), ct, hct.size(), hipMemcpyDeviceToHost, s));
  else
    memcpy(hct.data(), ct, hct.size());
  HIP_CHECK(hipStreamSynchronize(s));
  std::vector<uint8_t> hcoins(count * 16), hkp(count * 32), hhct(count * 32);
  const uint8_t one = 1;
  const uint8_t* pkh = tail.data();
  host_for(c->host_threads, count, [&](size_t i) {
    uint8_t h[32];
    sha3_256_3(&one, 1, pkh, 32, hmu.data() + i * mb, mb, h);
    memcpy(hcoins.data() + i * 16, h, 16);
    sha3_256_3(pkh, 32, hmu.data() + i * mb, mb, nullptr, 0, hkp.data() + i * 32);
  });
  HIP_CHECK(hipMemcpyAsync(dcoins, hcoins.data(), count * 16, hipMemcpyHostToDevice, s));
  KLAUNCH("fill", s, launch_fill_u32(dflags, count, 0, s));
  // c' = Encrypt(pk, m'; coins') compared with c on the device
  LWE_CHECK(pb_encrypt_core(c, pid, p, count, dsk + off_pk, dcoins, dmu2, mb, nullptr, dct, dflags, s));
  std::vector<uint32_t> hflags(count);
  HIP_CHECK(hipMemcpyAsync(hflags.data(), dflags, count * 4, hipMemcpyDeviceToHost, s));
  // H(ct) on the host while the device re-encrypts
  host_for(c->host_threads, count,
           [&](size_t i) { sha3_256(hct.data() + i * p.ct_bytes, p.ct_bytes, hhct.data() + i * 32); });
  HIP_CHECK(hipStreamSynchronize(s));
  std::vector<uint8_t> hss(count * 32);
  const uint8_t* zz = tail.data() + 32;
  for (size_t i = 0; i < count; ++i) {
    uint8_t buf[64];
    const uint8_t rej = (uint8_t)(0u - (uint32_t)(hflags[i] != 0));
    for (int k = 0; k < 32; ++k) buf[k] = (uint8_t)((hkp[i * 32 + k] & (uint8_t)~rej) | (zz[k] & rej));
    memcpy(buf + 32, hhct.data() + i * 32, 32);
    sha3_256(buf, 64, hss.data() + i * 32);
  }
  if (is_device_ptr(ss)) {
    HIP_CHECK(hipMemcpyAsync(ss, hss.data(), hss.size(), hipMemcpyHostToDevice, s));
    HIP_CHECK(hipStreamSynchronize(s));
  } else {
    memcpy(ss, hss.data(), hss.size());
  }
  return LWE_OK;
}

}  // namespace

// =====================================================================================
// C ABI
// =====================================================================================
extern "C" {

const char* lwe_strerror(int status) {
  switch (status) {
    case LWE_OK: return "ok";
    case LWE_EINVAL: return "invalid argument";
    case LWE_ENOMEM: return "out of device memory or over the context budget";
    case LWE_EDEVICE: return "HIP runtime error";
    case LWE_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

int lwe_ctx_create(lwe_ctx** out, int device, size_t hbm_budget_bytes) {
  if (!out) return LWE_EINVAL;
  *out = nullptr;
  if (hbm_budget_bytes && hbm_budget_bytes < T0_BYTES) return LWE_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return LWE_EDEVICE;
  }
  DevGuard g(device);
  lwe_ctx* c = new lwe_ctx();
  c->device = device;
  c->budget = hbm_budget_bytes;
  c->held = T0_BYTES;
  memset(c->tuning, 0, sizeof(c->tuning));
  unsigned hc = std::thread::hardware_concurrency();
  c->host_threads = (int)std::max(1u, std::min(hc, 16u));
  if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_done, hipEventDisableTiming) != hipSuccess ||
      hipMalloc(&c->d_T0, T0_BYTES) != hipSuccess ||
      hipMemcpy(c->d_T0, aes_T0(), T0_BYTES, hipMemcpyHostToDevice) != hipSuccess ||
      init_kernels() != hipSuccess) {
    (void)hipGetLastError();
    lwe_ctx_destroy(c);
    return LWE_EDEVICE;
  }
  int pools = 0;
  c->async_alloc = hipDeviceGetAttribute(&pools, hipDeviceAttributeMemoryPoolsSupported, device) == hipSuccess &&
                   pools != 0;
  (void)hipGetLastError();
  *out = c;
  return LWE_OK;
}

void lwe_ctx_destroy(lwe_ctx* c) {
  if (!c) return;
  DevGuard g(c->device);
  (void)hipDeviceSynchronize();
  for (auto& b : c->bufs) {
    if (!b.p) continue;
    if (b.async)
      (void)hipFreeAsync(b.p, c->own);
    else
      (void)hipFree(b.p);
  }
  if (c->own) (void)hipStreamSynchronize(c->own);
  if (c->d_T0) (void)hipFree(c->d_T0);
  if (c->hpin) (void)hipHostFree(c->hpin);
  for (auto& r : c->prof_pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->prof_pool) (void)hipEventDestroy(e);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->ev_done) (void)hipEventDestroy(c->ev_done);
  if (c->side) (void)hipStreamDestroy(c->side);
  if (c->own) (void)hipStreamDestroy(c->own);
  delete c;
}

size_t lwe_ctx_device_bytes(const lwe_ctx* c) { return c ? c->held : 0; }

int lwe_ctx_set_budget(lwe_ctx* c, size_t hbm_budget_bytes) {
  if (!c || (hbm_budget_bytes && hbm_budget_bytes < T0_BYTES)) return LWE_EINVAL;
  c->budget = hbm_budget_bytes;
  return LWE_OK;
}

int lwe_ctx_trim(lwe_ctx* c) {
  if (!c) return LWE_EINVAL;
  DevGuard g(c->device);
  // every queued use of the buffers is ordered before the end of the last call's stream
  hipStream_t s = c->last ? c->last : c->own;
  for (auto& b : c->bufs) {
    if (!b.p) continue;
    if (b.async) {
      HIP_CHECK(hipFreeAsync(b.p, s));
    } else {
      HIP_CHECK(hipStreamSynchronize(s));
      HIP_CHECK(hipFree(b.p));
    }
    c->held -= b.cap;
    b.p = nullptr;
    b.cap = 0;
    b.async = false;
  }
  return LWE_OK;
}

size_t lwe_ctx_call_bytes(lwe_ctx* c, int pid, int op, size_t count) {
  const Params* p = get_params(pid);
  if (!c || !p || op < 0 || op > 2 || count == 0 || count > LWE_MAX_BATCH) return 0;
  auto r = [](size_t b) { return ((b ? b : 16) + 255) & ~(size_t)255; };  // as ensure() rounds
  const size_t n = (size_t)p->n, ldx = (size_t)p->ldx, mb = p->mu_bytes;
  const lwe_tuning& tu = tuning_of(c, pid);
  // product split-K accumulator and, for the unfused variant, the expanded A
  auto product = [&](int M, int ncols, bool trans, bool per_inst_A) {
    ProdArgs a;
    memset(&a, 0, sizeof(a));
    a.M = M;
    a.ncols = ncols;
    a.per_inst_A = per_inst_A ? 1 : 0;
    size_t b = 0;
    if (tu.a_source == 1 && (!per_inst_A || M == 8)) b += r(n * n * 2);
    const ProdPlan pl = plan_product(c, pid, *p, a, trans);
    if (pl.acc_bytes) b += r(pl.acc_bytes);
    return b;
  };
  if (p->paper) {
    // the paper's sets: stream product (split-K accumulator via product()), DRBG chains,
    // operands of 256 rows per instance, row sums
    const size_t rows = count * PB_BITS, n = (size_t)p->n;
    const size_t req = (size_t)drbg_requests(rows / count * n);
    const size_t enc = r(rows * p->ldx) + r(rows * n) + r(count * PB_BITS) + r(rows * 4) + r(44 * 4) +
                       r(count * 3 * req * 256) + product((int)rows, p->n, false, false);
    size_t b = 0;
    if (op == 0)
      b = r(count * 16) * 2 + r(count * 32) + r(count * p->pk_bytes) + r(count * p->sk_bytes) + r(count * 44 * 4) +
          r(count * p->ldx) + r(count * n) + r(count * 4) + r(count * 2 * 256) + product((int)count, p->n, true, true) +
          r(count * 32);
    else if (op == 1)
      b = r(p->pk_bytes) + r(count * mb) + r(count * p->ct_bytes) + r(count * 16) + enc;
    else
      b = r(p->sk_bytes) + r(count * p->ct_bytes) + r(count * mb) + r(count * 16) + r(count * 4) + enc;
    return b + T0_BYTES;
  }
  const size_t M = count * 8;
  // encrypt_core: S' (whole 16-row groups), E', E'', round keys of seedA
  const size_t enc = r((M + 15) / 16 * 16 * ldx) + r(M * n) + r(count * 64) + r(44 * 4) +
                     product((int)M, (int)(n + 8), false, false);
  size_t b = 0;
  if (op == 0) {
    b = r(count * 16) * 2 + r(count * 32) + r(count * p->pk_bytes) + r(count * p->sk_bytes) + r(count * 44 * 4) * 2 +
        r(M * ldx) + r(M * n) + product((int)M, (int)n, true, true) + r(count * 32);
  } else if (op == 1) {
    b = r(p->pk_bytes) + r(count * mb) + r(count * p->ct_bytes) + r(count * 32) + r(count * 16) + r(count * 32) +
        r(count * 44 * 4) + r(32) + enc + r(count * 32);
  } else {
    b = r(p->sk_bytes) + r(count * p->ct_bytes) + r(count * 32) + r(count * mb) + r(count * 16) + r(count * 32) +
        r(count * 44 * 4) + r(count * 4) + enc + r(count * 32);
  }
  return b + T0_BYTES;
}
void* lwe_ctx_stream(lwe_ctx* c) { return c ? (void*)c->own : nullptr; }

int lwe_ctx_set_hash_lanes(lwe_ctx* c, int lanes) {
  if (!c || (lanes != 1 && lanes != 2)) return LWE_EINVAL;
  c->hash_lanes = lanes;
  return LWE_OK;
}

int lwe_ctx_set_side_stream(lwe_ctx* c, int enable) {
  if (!c || (enable != 0 && enable != 1)) return LWE_EINVAL;
  c->use_side = enable != 0;
  return LWE_OK;
}

int lwe_prof_enable(lwe_ctx* c, int on) {
  if (!c) return LWE_EINVAL;
  DevGuard g(c->device);
  LWE_CHECK(prof_resolve(c));
  c->prof_on = on != 0;
  return LWE_OK;
}

int lwe_prof_reset(lwe_ctx* c) {
  if (!c) return LWE_EINVAL;
  DevGuard g(c->device);
  LWE_CHECK(prof_resolve(c));
  c->prof_agg.clear();
  return LWE_OK;
}

int lwe_prof_read(lwe_ctx* c, const char* kernel, uint64_t* launches, double* total_ms) {
  if (!c || !kernel || !launches || !total_ms) return LWE_EINVAL;
  DevGuard g(c->device);
  LWE_CHECK(prof_resolve(c));
  auto it = c->prof_agg.find(kernel);
  *launches = it == c->prof_agg.end() ? 0 : it->second.first;
  *total_ms = it == c->prof_agg.end() ? 0.0 : it->second.second;
  return LWE_OK;
}

int lwe_param_id(uint32_t n) { return find_param(n); }
int lwe_param_id_paper(uint32_t n) { return find_param_paper(n); }

int lwe_param_register(uint32_t n, uint32_t logq, uint32_t B, uint32_t K, double sigma) {
  return register_param(n, logq, B, K, sigma);
}

int lwe_param_get(int pid, lwe_param_info* out) {
  const Params* p = get_params(pid);
  if (!p || !out) return LWE_EINVAL;
  out->n = (uint32_t)p->n;
  out->logq = (uint32_t)p->logq;
  out->B = (uint32_t)p->B;
  out->K = (uint32_t)p->K;
  out->sigma = p->sigma;
  out->pk_bytes = p->pk_bytes;
  out->sk_bytes = p->sk_bytes;
  out->ct_bytes = p->ct_bytes;
  out->mu_bytes = p->mu_bytes;
  out->paper = (uint32_t)p->paper;
  out->q = p->q;
  out->nbar = (uint32_t)p->nbar;
  out->mbar = (uint32_t)p->mbar;
  out->coef_bytes = (uint32_t)p->coef_bytes;
  out->eta = (uint32_t)p->eta;
  out->k = (uint32_t)p->ku;
  return LWE_OK;
}

size_t lwe_pk_bytes(int pid) {
  const Params* p = get_params(pid);
  return p ? p->pk_bytes : 0;
}
size_t lwe_sk_bytes(int pid) {
  const Params* p = get_params(pid);
  return p ? p->sk_bytes : 0;
}
size_t lwe_ct_bytes(int pid) {
  const Params* p = get_params(pid);
  return p ? p->ct_bytes : 0;
}
size_t lwe_mu_bytes(int pid) {
  const Params* p = get_params(pid);
  return p ? p->mu_bytes : 0;
}

int lwe_cdf_table(int pid, uint16_t* T_out, size_t capacity) {
  const Params* p = get_params(pid);
  if (!p || !T_out || capacity < (size_t)p->K + 1) return LWE_EINVAL;
  for (int k = 0; k <= p->K; ++k) T_out[k] = p->T[k];
  return LWE_OK;
}

int lwe_set_tuning(lwe_ctx* c, int pid, const lwe_tuning* t) {
  if (!c || !t || !get_params(pid)) return LWE_EINVAL;
  // both knobs zero (default) or both set to a built pair; one alone pairs with the default
  if (t->col_groups && t->row_groups && !product_strip_shape_ok((int)t->col_groups, (int)t->row_groups))
    return LWE_EINVAL;
  if ((t->col_groups && t->col_groups > 3) || (t->row_groups && t->row_groups != 2 && t->row_groups != 4))
    return LWE_EINVAL;
  if (t->a_source > 1) return LWE_EINVAL;
  c->tuning[pid & 255] = *t;
  return LWE_OK;
}

int lwe_get_tuning(lwe_ctx* c, int pid, lwe_tuning* t) {
  if (!c || !t || !get_params(pid)) return LWE_EINVAL;
  *t = c->tuning[pid & 255];
  return LWE_OK;
}

// ---------------------------------------------------------------------------------------
// KeyGen (Alg. 1): B^T = S^T A^T + E^T; pk = seedA || B^T; sk = S^T || pk || H(pk) || z
// ---------------------------------------------------------------------------------------
int lwe_keygen_batch(lwe_ctx* c, int pid, size_t count, const uint8_t* seedA, const uint8_t* seedSK,
                     const uint8_t* z, uint8_t* pk, uint8_t* sk, void* stream) {
  const Params* pp;
  if (!c) return LWE_EINVAL;
  LWE_CHECK(check_pid(pid, &pp));
  if (count == 0) return LWE_OK;
  if (!seedA || !seedSK || !z || !pk || !sk || count > LWE_MAX_BATCH) return LWE_EINVAL;
  const Params& p = *pp;
  if (p.paper) return pb_keygen(c, pid, p, count, seedA, seedSK, z, pk, sk, stream);
  DevGuard g(c->device);
  hipStream_t s = pick_stream(c, stream);
  CALL_SCOPE(c, s);
  const int n = p.n;
  const uint8_t *dA, *dS, *dZ;
  LWE_CHECK(stage_in(c, B_SEEDA, seedA, count * 16, s, &dA));
  LWE_CHECK(stage_in(c, B_SEEDSK, seedSK, count * 16, s, &dS));
  LWE_CHECK(stage_in(c, B_Z, z, count * 32, s, &dZ));
  OutStage opk, osk;
  LWE_CHECK(stage_out(c, B_PK, pk, count * p.pk_bytes, opk));
  LWE_CHECK(stage_out(c, B_SK, sk, count * p.sk_bytes, osk));
  uint32_t *rkA, *rkS;
  int8_t *X, *E;
  LWE_CHECK(ensure_t(c, B_RKA, count * 44 * 4, &rkA));
  LWE_CHECK(ensure_t(c, B_RK, count * 44 * 4, &rkS));
  LWE_CHECK(ensure_t(c, B_X, count * 8 * (size_t)p.ldx, &X));
  LWE_CHECK(ensure_t(c, B_E, count * 8 * (size_t)n, &E));
  KLAUNCH("expand_keys", s, launch_expand_keys(dA, 16, (int)count, c->d_T0, rkA, s));
  KLAUNCH("expand_keys", s, launch_expand_keys(dS, 16, (int)count, c->d_T0, rkS, s));
  SampleArgs sa;
  memset(&sa, 0, sizeof(sa));
  sa.rk = rkS;
  sa.T0 = c->d_T0;
  sa.n = n;
  sa.K = p.K;
  sa.ldx = p.ldx;
  sa.nseg = 2;
  for (int k = 0; k < MAX_K; ++k) sa.T2[k] = (uint32_t)p.T[k] * 0x10001u;
  sa.X = X;
  sa.X16 = osk.dev;  // S^T int16 at the start of each sk record
  sa.x16_stride = p.sk_bytes;
  sa.E = E;
  KLAUNCH("sample", s, launch_sample(sa, (int)count, s));
  ProdArgs a;
  memset(&a, 0, sizeof(a));
  a.rkA = rkA;
  a.T0 = c->d_T0;
  a.X = X;
  a.ldx = p.ldx;
  a.M = (int)(count * 8);
  a.n = n;
  a.logq = p.logq;
  a.B = p.B;
  a.ncols = n;
  a.per_inst_A = 1;
  a.mode = PM_KEYGEN;
  a.E = E;
  a.out = opk.dev;
  a.out_stride = p.pk_bytes;
  a.out_off = 16;
  LWE_CHECK(run_product(c, pid, p, a, true, s));
  // pk = seedA || B^T ; sk = S^T || pk || H(pk) || z
  HIP_CHECK(hipMemcpy2DAsync(opk.dev, p.pk_bytes, dA, 16, 16, count, hipMemcpyDeviceToDevice, s));
  const size_t off_pk = (size_t)16 * n, off_pkh = off_pk + p.pk_bytes, off_z = off_pkh + 32;
  HIP_CHECK(hipMemcpy2DAsync(osk.dev + off_pk, p.sk_bytes, opk.dev, p.pk_bytes, p.pk_bytes, count,
                             hipMemcpyDeviceToDevice, s));
  HIP_CHECK(hipMemcpy2DAsync(osk.dev + off_z, p.sk_bytes, dZ, 32, 32, count, hipMemcpyDeviceToDevice, s));
  if (use_host_hash(c, pid, count)) {
    // public keys down, hashed on the host in stream order, hashes up, all through the pinned
    // staging (every use of it is ordered on the context's calls); the newest key's hash is
    // left in the cache for an encapsulation against it
    uint8_t* hpk;
    LWE_CHECK(host_pinned(c, count * (p.pk_bytes + 32), s, &hpk));
    uint8_t* hh = hpk + count * p.pk_bytes;
    HIP_CHECK(hipMemcpyAsync(hpk, opk.dev, count * p.pk_bytes, hipMemcpyDeviceToHost, s));
    LWE_CHECK(host_hash_async(c, hpk, p.pk_bytes, count, hh, false, true, s));
    uint8_t* dh;
    LWE_CHECK(ensure_t(c, B_HCT, count * 32, &dh));
    HIP_CHECK(hipMemcpyAsync(dh, hh, count * 32, hipMemcpyHostToDevice, s));
    HIP_CHECK(hipMemcpy2DAsync(osk.dev + off_pkh, p.sk_bytes, dh, 32, 32, count, hipMemcpyDeviceToDevice, s));
  } else {
    uint8_t* dh;
    LWE_CHECK(ensure_t(c, B_HCT, count * 32, &dh));
    KLAUNCH("hash_records", s, launch_hash_records((int)count, opk.dev, p.pk_bytes, p.pk_bytes, dh, c->hash_lanes, s));
    HIP_CHECK(hipMemcpy2DAsync(osk.dev + off_pkh, p.sk_bytes, dh, 32, 32, count, hipMemcpyDeviceToDevice, s));
  }
  LWE_CHECK(finish_out(opk, s));
  LWE_CHECK(finish_out(osk, s));
  if (opk.host || osk.host || !stream) HIP_CHECK(hipStreamSynchronize(s));
  return LWE_OK;
}

int lwe_keygen(lwe_ctx* c, int pid, const uint8_t* seedA, const uint8_t* seedSK, const uint8_t* z,
               uint8_t* pk, uint8_t* sk, void* stream) {
  return lwe_keygen_batch(c, pid, 1, seedA, seedSK, z, pk, sk, stream);
}

// ---------------------------------------------------------------------------------------
// Encaps (Alg. 4): coins = H(0x01 || H(pk) || mu)[0:16], K' = H(H(pk) || mu),
// ct = Encrypt(pk, mu; coins), K = H(K' || H(ct))
// ---------------------------------------------------------------------------------------
int lwe_encaps_batch(lwe_ctx* c, int pid, size_t count, const uint8_t* pk, const uint8_t* mu,
                     uint8_t* ct, uint8_t* ss, void* stream) {
  const Params* pp;
  if (!c) return LWE_EINVAL;
  LWE_CHECK(check_pid(pid, &pp));
  if (count == 0) return LWE_OK;
  if (!pk || !mu || !ct || !ss || count > LWE_MAX_BATCH) return LWE_EINVAL;
  const Params& p = *pp;
  if (p.paper) return pb_encaps(c, pid, p, count, pk, mu, ct, ss, stream);
  DevGuard g(c->device);
  hipStream_t s = pick_stream(c, stream);
  CALL_SCOPE(c, s);
  const size_t mb = p.mu_bytes;
  // H(pk) on the host (cached per public key); with host hashing the messages come back in the
  // same wait
  const bool hh = use_host_hash(c, pid, count);
  std::vector<uint8_t> hpk, hmu;
  uint8_t pkh[32];
  const uint8_t* pkh_src = pkh;  // host source of the H(pk) upload (device hashing only)
  if (hh) {
    LWE_CHECK(host_copy2(pk, p.pk_bytes, hpk, mu, count * mb, hmu, s));
    host_pkh(c, hpk.data(), p.pk_bytes, pkh);
  } else if (is_device_ptr(pk)) {
    // the key down, hashed (or found in the cache) on the host in stream order, its hash up:
    // through the pinned staging, without waiting here
    uint8_t* st;
    LWE_CHECK(host_pinned(c, p.pk_bytes + 32, s, &st));
    HIP_CHECK(hipMemcpyAsync(st, pk, p.pk_bytes, hipMemcpyDeviceToHost, s));
    LWE_CHECK(host_hash_async(c, st, p.pk_bytes, 1, st + p.pk_bytes, true, false, s));
    pkh_src = st + p.pk_bytes;
  } else {
    host_pkh(c, pk, p.pk_bytes, pkh);
  }
  const uint8_t *dpk, *dmu;
  LWE_CHECK(stage_in(c, B_PK, pk, p.pk_bytes, s, &dpk));
  LWE_CHECK(stage_in(c, B_MU, mu, count * mb, s, &dmu));
  OutStage oct, oss;
  LWE_CHECK(stage_out(c, B_CT, ct, count * p.ct_bytes, oct));
  LWE_CHECK(stage_out(c, B_SS, ss, count * 32, oss));
  uint8_t *dcoins, *dkp;
  uint32_t* drk;
  LWE_CHECK(ensure_t(c, B_COINS, count * 16, &dcoins));
  LWE_CHECK(ensure_t(c, B_KP, count * 32, &dkp));
  LWE_CHECK(ensure_t(c, B_RK, count * 44 * 4, &drk));
  std::vector<uint8_t> hcoins, hkp;
  if (hh) {
    hcoins.resize(count * 16);
    hkp.resize(count * 32);
    const uint8_t one = 1;
    host_for(c->host_threads, count, [&](size_t i) {
      uint8_t h[32];
      sha3_256_3(&one, 1, pkh, 32, hmu.data() + i * mb, mb, h);
      memcpy(hcoins.data() + i * 16, h, 16);
      sha3_256_3(pkh, 32, hmu.data() + i * mb, mb, nullptr, 0, hkp.data() + i * 32);
    });
    HIP_CHECK(hipMemcpyAsync(dcoins, hcoins.data(), count * 16, hipMemcpyHostToDevice, s));
  } else {
    uint8_t* dpkh;
    LWE_CHECK(ensure_t(c, B_PKH, 32, &dpkh));
    HIP_CHECK(hipMemcpyAsync(dpkh, pkh_src, 32, hipMemcpyHostToDevice, s));
    KLAUNCH("fo_coins", s, launch_fo_coins((int)count, dpkh, dmu, mb, (int)mb, dcoins, dkp, s));
  }
  KLAUNCH("expand_keys", s, launch_expand_keys(dcoins, 16, (int)count, c->d_T0, drk, s));
  LWE_CHECK(encrypt_core(c, pid, p, count, dpk, drk, dmu, mb, oct.dev, nullptr, nullptr, s));
  if (hh) {
    std::vector<uint8_t> hct(count * p.ct_bytes), hss(count * 32);
    HIP_CHECK(hipMemcpyAsync(hct.data(), oct.dev, hct.size(), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    host_for(c->host_threads, count, [&](size_t i) {
      uint8_t h[32];
      sha3_256(hct.data() + i * p.ct_bytes, p.ct_bytes, h);
      sha3_256_3(hkp.data() + i * 32, 32, h, 32, nullptr, 0, hss.data() + i * 32);
    });
    if (oss.host) {
      memcpy(ss, hss.data(), hss.size());
      oss.bytes = 0;
    } else {
      HIP_CHECK(hipMemcpyAsync(oss.dev, hss.data(), hss.size(), hipMemcpyHostToDevice, s));
      HIP_CHECK(hipStreamSynchronize(s));
    }
  } else {
    uint8_t* dhct;
    LWE_CHECK(ensure_t(c, B_HCT, count * 32, &dhct));
    KLAUNCH("hash_records", s, launch_hash_records((int)count, oct.dev, p.ct_bytes, p.ct_bytes, dhct, c->hash_lanes, s));
    KLAUNCH("final_ss", s, launch_final_ss((int)count, nullptr, dkp, nullptr, dhct, oss.dev, s));
  }
  LWE_CHECK(finish_out(oct, s));
  LWE_CHECK(finish_out(oss, s));
  if (oct.host || oss.host || !stream) HIP_CHECK(hipStreamSynchronize(s));
  return LWE_OK;
}

int lwe_encaps(lwe_ctx* c, int pid, const uint8_t* pk, const uint8_t* mu, uint8_t* ct, uint8_t* ss,
               void* stream) {
  return lwe_encaps_batch(c, pid, 1, pk, mu, ct, ss, stream);
}

// ---------------------------------------------------------------------------------------
// Decaps (Alg. 5): mu' = Decrypt(sk, ct); coins', K'' from mu'; ct' = Encrypt(pk, mu'; coins');
// K = H(K'' || H(ct)) if ct' == ct else H(z || H(ct)), selected in constant time.
// ---------------------------------------------------------------------------------------
int lwe_decaps_batch(lwe_ctx* c, int pid, size_t count, const uint8_t* sk, const uint8_t* ct,
                     uint8_t* ss, void* stream) {
  const Params* pp;
  if (!c) return LWE_EINVAL;
  LWE_CHECK(check_pid(pid, &pp));
  if (count == 0) return LWE_OK;
  if (!sk || !ct || !ss || count > LWE_MAX_BATCH) return LWE_EINVAL;
  const Params& p = *pp;
  if (p.paper) return pb_decaps(c, pid, p, count, sk, ct, ss, stream);
  DevGuard g(c->device);
  hipStream_t s = pick_stream(c, stream);
  CALL_SCOPE(c, s);
  const int n = p.n;
  const size_t mb = p.mu_bytes;
  const size_t off_pk = (size_t)16 * n, off_pkh = off_pk + p.pk_bytes, off_z = off_pkh + 32;
  const uint8_t *dsk, *dct;
  LWE_CHECK(stage_in(c, B_SK, sk, p.sk_bytes, s, &dsk));
  LWE_CHECK(stage_in(c, B_CT, ct, count * p.ct_bytes, s, &dct));
  OutStage oss;
  LWE_CHECK(stage_out(c, B_SS, ss, count * 32, oss));
  uint8_t *dmu2, *dcoins, *dkp;
  uint32_t *drk, *dflags;
  LWE_CHECK(ensure_t(c, B_MU2, count * mb, &dmu2));
  LWE_CHECK(ensure_t(c, B_COINS, count * 16, &dcoins));
  LWE_CHECK(ensure_t(c, B_KP, count * 32, &dkp));
  LWE_CHECK(ensure_t(c, B_RK, count * 44 * 4, &drk));
  LWE_CHECK(ensure_t(c, B_FLAGS, count * 4, &dflags));
  // mu' = Decrypt(sk, ct)
  DecArgs da;
  da.ct = dct;
  da.ct_stride = p.ct_bytes;
  da.St16 = dsk;
  da.n = n;
  da.logq = p.logq;
  da.B = p.B;
  da.count = (int)count;
  da.mu_bytes = (int)mb;
  da.mu_out = dmu2;
  KLAUNCH("decrypt", s, launch_decrypt(da, s));
  const bool hh = use_host_hash(c, pid, count);
  std::vector<uint8_t> hsk_tail, hkp, hct, hhct;
  if (hh) {
    // pkh and z from the secret key, mu' to the host, coins' and K'' on the host.  The received
    // ciphertexts come back in the same wait, so that their hashing on the host overlaps the
    // re-encryption below.
    std::vector<uint8_t> hmu(count * mb), hcoins(count * 16);
    hsk_tail.resize(64);
    HIP_CHECK(hipMemcpyAsync(hsk_tail.data(), dsk + off_pkh, 64, hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(hmu.data(), dmu2, hmu.size(), hipMemcpyDeviceToHost, s));
    hct.resize(count * p.ct_bytes);
    if (is_device_ptr(ct))
      HIP_CHECK(hipMemcpyAsync(hct.data(), ct, hct.size(), hipMemcpyDeviceToHost, s));
    else
      memcpy(hct.data(), ct, hct.size());
    HIP_CHECK(hipStreamSynchronize(s));
    hkp.resize(count * 32);
    const uint8_t one = 1;
    const uint8_t* pkh = hsk_tail.data();
    host_for(c->host_threads, count, [&](size_t i) {
      uint8_t h[32];
      sha3_256_3(&one, 1, pkh, 32, hmu.data() + i * mb, mb, h);
      memcpy(hcoins.data() + i * 16, h, 16);
      sha3_256_3(pkh, 32, hmu.data() + i * mb, mb, nullptr, 0, hkp.data() + i * 32);
    });
    HIP_CHECK(hipMemcpyAsync(dcoins, hcoins.data(), count * 16, hipMemcpyHostToDevice, s));
    KLAUNCH("expand_keys", s, launch_expand_keys(dcoins, 16, (int)count, c->d_T0, drk, s));
    KLAUNCH("fill", s, launch_fill_u32(dflags, count, 0, s));
    LWE_CHECK(encrypt_core(c, pid, p, count, dsk + off_pk, drk, dmu2, mb, nullptr, dct, dflags, s));
    std::vector<uint32_t> hflags(count);
    HIP_CHECK(hipMemcpyAsync(hflags.data(), dflags, count * 4, hipMemcpyDeviceToHost, s));
    // H(ct) on the host while the device re-encrypts
    hhct.resize(count * 32);
    host_for(c->host_threads, count,
             [&](size_t i) { sha3_256(hct.data() + i * p.ct_bytes, p.ct_bytes, hhct.data() + i * 32); });
    HIP_CHECK(hipStreamSynchronize(s));
    std::vector<uint8_t> hss(count * 32);
    const uint8_t* zz = hsk_tail.data() + 32;
    for (size_t i = 0; i < count; ++i) {
      uint8_t buf[64];
      const uint8_t rej = (uint8_t)(0u - (uint32_t)(hflags[i] != 0));
      for (int k = 0; k < 32; ++k)
        buf[k] = (uint8_t)((hkp[i * 32 + k] & (uint8_t)~rej) | (zz[k] & rej));
      memcpy(buf + 32, hhct.data() + i * 32, 32);
      sha3_256(buf, 64, hss.data() + i * 32);
    }
    if (oss.host) {
      memcpy(ss, hss.data(), hss.size());
      oss.bytes = 0;
    } else {
      HIP_CHECK(hipMemcpyAsync(oss.dev, hss.data(), hss.size(), hipMemcpyHostToDevice, s));
      HIP_CHECK(hipStreamSynchronize(s));
    }
  } else {
    // H(ct) of the received ciphertexts does not depend on the decryption: it runs on the
    // side stream while the main stream decrypts and re-encrypts (or first, on the main
    // stream, when the context keeps all of its work on one stream).
    uint8_t* dhct;
    LWE_CHECK(ensure_t(c, B_HCT, count * 32, &dhct));
    if (c->use_side && !c->side && hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
      c->side = nullptr;
      (void)hipGetLastError();
      return LWE_EDEVICE;
    }
    hipStream_t hs = c->use_side ? c->side : s;
    if (c->use_side) {
      HIP_CHECK(hipEventRecord(c->ev_fork, s));
      HIP_CHECK(hipStreamWaitEvent(c->side, c->ev_fork, 0));
    }
    KLAUNCH("hash_records", hs, launch_hash_records((int)count, dct, p.ct_bytes, p.ct_bytes, dhct, c->hash_lanes, hs));
    if (c->use_side) HIP_CHECK(hipEventRecord(c->ev_join, c->side));
    KLAUNCH("fo_coins", s, launch_fo_coins((int)count, dsk + off_pkh, dmu2, mb, (int)mb, dcoins, dkp, s));
    KLAUNCH("expand_keys", s, launch_expand_keys(dcoins, 16, (int)count, c->d_T0, drk, s));
    KLAUNCH("fill", s, launch_fill_u32(dflags, count, 0, s));
    LWE_CHECK(encrypt_core(c, pid, p, count, dsk + off_pk, drk, dmu2, mb, nullptr, dct, dflags, s));
    if (c->use_side) HIP_CHECK(hipStreamWaitEvent(s, c->ev_join, 0));
    KLAUNCH("final_ss", s, launch_final_ss((int)count, dflags, dkp, dsk + off_z, dhct, oss.dev, s));
  }
  LWE_CHECK(finish_out(oss, s));
  if (oss.host || !stream) HIP_CHECK(hipStreamSynchronize(s));
  return LWE_OK;
}

int lwe_decaps(lwe_ctx* c, int pid, const uint8_t* sk, const uint8_t* ct, uint8_t* ss, void* stream) {
  return lwe_decaps_batch(c, pid, 1, sk, ct, ss, stream);
}

// ---------------------------------------------------------------------------------------
// Test hooks
// ---------------------------------------------------------------------------------------
int lwe_test_expand_A(lwe_ctx* c, int pid, const uint8_t* seedA, uint32_t col0, uint32_t ncols,
                      uint16_t* out, void* stream) {
  const Params* pp;
  if (!c || !seedA || !out) return LWE_EINVAL;
  LWE_CHECK(check_pid(pid, &pp));
  if (pp->paper) return LWE_EUNSUPPORTED;
  const Params& p = *pp;
  if ((uint64_t)col0 + ncols > (uint64_t)p.n) return LWE_EINVAL;
  DevGuard g(c->device);
  hipStream_t s = pick_stream(c, stream);
  CALL_SCOPE(c, s);
  const uint8_t* dA;
  LWE_CHECK(stage_in(c, B_SEEDA, seedA, 16, s, &dA));
  uint32_t* rk;
  LWE_CHECK(ensure_t(c, B_RKA, 44 * 4, &rk));
  KLAUNCH("expand_keys", s, launch_expand_keys(dA, 16, 1, c->d_T0, rk, s));
  OutStage o;
  LWE_CHECK(stage_out(c, B_TEST, out, (size_t)ncols * p.n * 2, o));
  HIP_CHECK(launch_expand_A(p, rk, c->d_T0, col0, ncols, (uint16_t*)o.dev, s));
  LWE_CHECK(finish_out(o, s));
  HIP_CHECK(hipStreamSynchronize(s));
  return LWE_OK;
}

int lwe_test_keystream(lwe_ctx* c, const uint8_t* key, uint32_t domain, uint64_t block0, size_t nblocks,
                       uint8_t* out, void* stream) {
  if (!c || !key || !out) return LWE_EINVAL;
  DevGuard g(c->device);
  hipStream_t s = pick_stream(c, stream);
  CALL_SCOPE(c, s);
  const uint8_t* dk;
  LWE_CHECK(stage_in(c, B_SEEDA, key, 16, s, &dk));
  uint32_t* rk;
  LWE_CHECK(ensure_t(c, B_RKA, 44 * 4, &rk));
  KLAUNCH("expand_keys", s, launch_expand_keys(dk, 16, 1, c->d_T0, rk, s));
  OutStage o;
  LWE_CHECK(stage_out(c, B_TEST, out, nblocks * 16, o));
  KLAUNCH("keystream", s, launch_keystream(rk, c->d_T0, domain, block0, nblocks, o.dev, s));
  LWE_CHECK(finish_out(o, s));
  HIP_CHECK(hipStreamSynchronize(s));
  return LWE_OK;
}

int lwe_test_sample(lwe_ctx* c, int pid, const uint8_t* key, uint32_t domain, uint64_t word0, size_t count,
                    int16_t* out, void* stream) {
  const Params* pp;
  if (!c || !key || !out) return LWE_EINVAL;
  LWE_CHECK(check_pid(pid, &pp));
  if (pp->paper) return LWE_EUNSUPPORTED;
  DevGuard g(c->device);
  hipStream_t s = pick_stream(c, stream);
  CALL_SCOPE(c, s);
  const uint8_t* dk;
  LWE_CHECK(stage_in(c, B_SEEDA, key, 16, s, &dk));
  uint32_t* rk;
  LWE_CHECK(ensure_t(c, B_RKA, 44 * 4, &rk));
  KLAUNCH("expand_keys", s, launch_expand_keys(dk, 16, 1, c->d_T0, rk, s));
  OutStage o;
  LWE_CHECK(stage_out(c, B_TEST, out, count * 2, o));
  KLAUNCH("sample_stream", s, launch_sample_stream(*pp, rk, c->d_T0, domain, word0, count, (int16_t*)o.dev, s));
  LWE_CHECK(finish_out(o, s));
  HIP_CHECK(hipStreamSynchronize(s));
  return LWE_OK;
}

int lwe_test_encrypt(lwe_ctx* c, int pid, size_t count, const uint8_t* pk, const uint8_t* coins,
                     const uint8_t* mu, uint8_t* ct, void* stream) {
  const Params* pp;
  if (!c || !pk || !coins || !mu || !ct || count > LWE_MAX_BATCH) return LWE_EINVAL;
  LWE_CHECK(check_pid(pid, &pp));
  if (pp->paper) return LWE_EUNSUPPORTED;
  if (count == 0) return LWE_OK;
  const Params& p = *pp;
  DevGuard g(c->device);
  hipStream_t s = pick_stream(c, stream);
  CALL_SCOPE(c, s);
  const uint8_t *dpk, *dco, *dmu;
  LWE_CHECK(stage_in(c, B_PK, pk, p.pk_bytes, s, &dpk));
  LWE_CHECK(stage_in(c, B_SEEDSK, coins, count * 16, s, &dco));
  LWE_CHECK(stage_in(c, B_MU, mu, count * p.mu_bytes, s, &dmu));
  OutStage o;
  LWE_CHECK(stage_out(c, B_CT, ct, count * p.ct_bytes, o));
  uint32_t* drk;
  LWE_CHECK(ensure_t(c, B_RK, count * 44 * 4, &drk));
  KLAUNCH("expand_keys", s, launch_expand_keys(dco, 16, (int)count, c->d_T0, drk, s));
  LWE_CHECK(encrypt_core(c, pid, p, count, dpk, drk, dmu, p.mu_bytes, o.dev, nullptr, nullptr, s));
  LWE_CHECK(finish_out(o, s));
  HIP_CHECK(hipStreamSynchronize(s));
  return LWE_OK;
}

int lwe_test_decrypt(lwe_ctx* c, int pid, size_t count, const uint8_t* sk, const uint8_t* ct, uint8_t* mu,
                     void* stream) {
  const Params* pp;
  if (!c || !sk || !ct || !mu || count > LWE_MAX_BATCH) return LWE_EINVAL;
  LWE_CHECK(check_pid(pid, &pp));
  if (pp->paper) return LWE_EUNSUPPORTED;
  if (count == 0) return LWE_OK;
  const Params& p = *pp;
  DevGuard g(c->device);
  hipStream_t s = pick_stream(c, stream);
  CALL_SCOPE(c, s);
  const uint8_t *dsk, *dct;
  LWE_CHECK(stage_in(c, B_SK, sk, p.sk_bytes, s, &dsk));
  LWE_CHECK(stage_in(c, B_CT, ct, count * p.ct_bytes, s, &dct));
  OutStage o;
  LWE_CHECK(stage_out(c, B_MU2, mu, count * p.mu_bytes, o));
  DecArgs da;
  da.ct = dct;
  da.ct_stride = p.ct_bytes;
  da.St16 = dsk;
  da.n = p.n;
  da.logq = p.logq;
  da.B = p.B;
  da.count = (int)count;
  da.mu_bytes = (int)p.mu_bytes;
  da.mu_out = o.dev;
  KLAUNCH("decrypt", s, launch_decrypt(da, s));
  LWE_CHECK(finish_out(o, s));
  HIP_CHECK(hipStreamSynchronize(s));
  return LWE_OK;
}

int lwe_test_sha3(lwe_ctx* c, size_t count, size_t len, const uint8_t* in, uint8_t* out, void* stream) {
  if (!c || !in || !out || count > ((size_t)1 << 24)) return LWE_EINVAL;
  if (count == 0) return LWE_OK;
  DevGuard g(c->device);
  hipStream_t s = pick_stream(c, stream);
  CALL_SCOPE(c, s);
  const uint8_t* din;
  LWE_CHECK(stage_in(c, B_CT, in, count * len, s, &din));
  OutStage o;
  LWE_CHECK(stage_out(c, B_TEST, out, count * 32, o));
  KLAUNCH("hash_records", s, launch_hash_records((int)count, din, len, len, o.dev, c->hash_lanes, s));
  LWE_CHECK(finish_out(o, s));
  HIP_CHECK(hipStreamSynchronize(s));
  return LWE_OK;
}


int lwe_test_sample_batch(lwe_ctx* c, int pid, size_t count, int mode, int layout, const uint8_t* keys,
                          int8_t* X_out, int8_t* E_out, int8_t* E2_out, uint8_t* X16_out, void* stream) {
  const Params* pp;
  if (!c || !keys || !X_out || !E_out || count == 0 || count > LWE_MAX_BATCH) return LWE_EINVAL;
  if ((mode != 0 && mode != 1) || (layout != 0 && layout != 1)) return LWE_EINVAL;
  if ((mode == 1) != (E2_out != nullptr) || (mode == 1 && X16_out)) return LWE_EINVAL;
  LWE_CHECK(check_pid(pid, &pp));
  if (pp->paper) return LWE_EUNSUPPORTED;
  const Params& p = *pp;
  DevGuard g(c->device);
  hipStream_t s = pick_stream(c, stream);
  CALL_SCOPE(c, s);
  const int n = p.n;
  const uint8_t* dk;
  LWE_CHECK(stage_in(c, B_SEEDSK, keys, count * 16, s, &dk));
  uint32_t* rk;
  LWE_CHECK(ensure_t(c, B_RK, count * 44 * 4, &rk));
  KLAUNCH("expand_keys", s, launch_expand_keys(dk, 16, (int)count, c->d_T0, rk, s));
  const size_t x_bytes = (layout ? (count * 8 + 15) / 16 * 16 : count * 8) * (size_t)p.ldx;
  OutStage ox, oe, oe2, o16;
  LWE_CHECK(stage_out(c, B_X, X_out, x_bytes, ox));
  LWE_CHECK(stage_out(c, B_E, E_out, count * 8 * (size_t)n, oe));
  if (E2_out) LWE_CHECK(stage_out(c, B_E2, E2_out, count * 64, oe2));
  if (X16_out) LWE_CHECK(stage_out(c, B_SK, X16_out, count * 16 * (size_t)n, o16));
  // bytes the sampler does not own (unwritten rows of the last fragment group) stay 0x5a
  KLAUNCH("fill", s, launch_fill_u32((uint32_t*)ox.dev, x_bytes / 4, 0x5a5a5a5au, s));
  SampleArgs sa;
  memset(&sa, 0, sizeof(sa));
  sa.rk = rk;
  sa.T0 = c->d_T0;
  sa.n = n;
  sa.K = p.K;
  sa.ldx = p.ldx;
  sa.nseg = mode ? 3 : 2;
  for (int k = 0; k < MAX_K; ++k) sa.T2[k] = (uint32_t)p.T[k] * 0x10001u;
  sa.X = (int8_t*)ox.dev;
  sa.x_frag = layout;
  sa.X16 = X16_out ? o16.dev : nullptr;
  sa.x16_stride = 16 * (size_t)n;
  sa.E = (int8_t*)oe.dev;
  sa.E2 = E2_out ? (int8_t*)oe2.dev : nullptr;
  KLAUNCH("sample", s, launch_sample(sa, (int)count, s));
  LWE_CHECK(finish_out(ox, s));
  LWE_CHECK(finish_out(oe, s));
  if (E2_out) LWE_CHECK(finish_out(oe2, s));
  if (X16_out) LWE_CHECK(finish_out(o16, s));
  HIP_CHECK(hipStreamSynchronize(s));
  return LWE_OK;
}

int lwe_test_product(lwe_ctx* c, int pid, size_t count, const uint8_t* seedA, const uint8_t* Bt, const int8_t* S,
                     const int8_t* E, const int8_t* E2, const uint8_t* mu, uint8_t* ct, void* stream) {
  const Params* pp;
  if (!c || !seedA || !Bt || !S || !E || !E2 || !mu || !ct || count == 0 || count > LWE_MAX_BATCH)
    return LWE_EINVAL;
  LWE_CHECK(check_pid(pid, &pp));
  if (pp->paper) return LWE_EUNSUPPORTED;
  const Params& p = *pp;
  DevGuard g(c->device);
  hipStream_t s = pick_stream(c, stream);
  CALL_SCOPE(c, s);
  const int n = p.n;
  const size_t rows = count * 8;
  const uint8_t *dA, *dBt, *dS, *dE, *dE2, *dmu;
  LWE_CHECK(stage_in(c, B_SEEDA, seedA, 16, s, &dA));
  LWE_CHECK(stage_in(c, B_PK, Bt, 16 * (size_t)n, s, &dBt));
  LWE_CHECK(stage_in(c, B_TEST, S, rows * n, s, &dS));
  LWE_CHECK(stage_in(c, B_E, E, rows * n, s, &dE));
  LWE_CHECK(stage_in(c, B_E2, E2, count * 64, s, &dE2));
  LWE_CHECK(stage_in(c, B_MU, mu, count * p.mu_bytes, s, &dmu));
  OutStage o;
  LWE_CHECK(stage_out(c, B_CT, ct, count * p.ct_bytes, o));
  uint32_t* rkA;
  LWE_CHECK(ensure_t(c, B_RKA, 44 * 4, &rkA));
  KLAUNCH("expand_keys", s, launch_expand_keys(dA, 16, 1, c->d_T0, rkA, s));
  // S' into the operand layout of the product this batch size selects
  const bool frag = uses_strip((int)rows, false, false);
  int8_t* X;
  LWE_CHECK(ensure_t(c, B_X, (rows + 15) / 16 * 16 * (size_t)p.ldx, &X));
  HIP_CHECK(launch_pack_x((const int8_t*)dS, (int)rows, n, p.ldx, frag ? 1 : 0, X, s));
  ProdArgs a;
  memset(&a, 0, sizeof(a));
  a.rkA = rkA;
  a.T0 = c->d_T0;
  a.X = X;
  a.ldx = p.ldx;
  a.M = (int)rows;
  a.n = n;
  a.logq = p.logq;
  a.B = p.B;
  a.ncols = n + 8;
  a.Bt = dBt;
  a.mode = PM_ENCRYPT;
  a.E = (const int8_t*)dE;
  a.E2 = (const int8_t*)dE2;
  a.mu = dmu;
  a.mu_stride = p.mu_bytes;
  a.out = o.dev;
  a.out_stride = p.ct_bytes;
  LWE_CHECK(run_product(c, pid, p, a, false, s));
  LWE_CHECK(finish_out(o, s));
  HIP_CHECK(hipStreamSynchronize(s));
  return LWE_OK;
}

}  // extern "C"

namespace {
// Fills buf with bytes from the operating system's random source (getrandom(2)).
int os_random(uint8_t* buf, size_t len) {
  size_t got = 0;
  while (got < len) {
    const ssize_t r = getrandom(buf + got, len - got, 0);
    if (r < 0) {
      if (errno == EINTR) continue;
      return LWE_EDEVICE;
    }
    got += (size_t)r;
  }
  return LWE_OK;
}

void wipe(std::vector<uint8_t>& v) {
  volatile uint8_t* p = v.data();
  for (size_t i = 0; i < v.size(); ++i) p[i] = 0;
}
}  // namespace

extern "C" {

int lwe_keygen_rand(lwe_ctx* c, int pid, size_t count, uint8_t* pk, uint8_t* sk, void* stream) {
  const Params* pp;
  if (!c) return LWE_EINVAL;
  LWE_CHECK(check_pid(pid, &pp));
  if (count == 0) return LWE_OK;
  if (!pk || !sk || count > LWE_MAX_BATCH) return LWE_EINVAL;
  std::vector<uint8_t> seeds(count * 64);  // seedA (16) | seedSK (16) | z (32) blocks
  int st = os_random(seeds.data(), seeds.size());
  if (st == LWE_OK)
    st = lwe_keygen_batch(c, pid, count, seeds.data(), seeds.data() + count * 16, seeds.data() + count * 32, pk, sk,
                          stream);
  // the staged seeds must have left host memory before it is wiped
  if (st == LWE_OK && stream && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) st = LWE_EDEVICE;
  wipe(seeds);
  return st;
}

int lwe_encaps_rand(lwe_ctx* c, int pid, size_t count, const uint8_t* pk, uint8_t* ct, uint8_t* ss, void* stream) {
  const Params* pp;
  if (!c) return LWE_EINVAL;
  LWE_CHECK(check_pid(pid, &pp));
  if (count == 0) return LWE_OK;
  if (!pk || !ct || !ss || count > LWE_MAX_BATCH) return LWE_EINVAL;
  std::vector<uint8_t> mu(count * pp->mu_bytes);
  int st = os_random(mu.data(), mu.size());
  if (st == LWE_OK) st = lwe_encaps_batch(c, pid, count, pk, mu.data(), ct, ss, stream);
  if (st == LWE_OK && stream && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) st = LWE_EDEVICE;
  wipe(mu);
  return st;
}

}  // extern "C"

// =====================================================================================
// No-allocation decapsulation: the working memory of lwe_decaps_batch taken from a fixed
// device array instead of a context's growable buffers.
// =====================================================================================
static __device__ __align__(256) uint8_t scratch[LWE_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
uint8_t* g_noalloc_ptr[NOALLOC_MAX_DEVICES];

// Device address of the current device's copy of `scratch`, set up once per device: the
// address comes from hipGetSymbolAddress (the array's name is only a host-side stand-in), and
// the first T0_BYTES receive the AES table.  The rest is the per-call arena.
int noalloc_base(int dev, uint8_t** out) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr ||
        hipMemcpy(ptr, aes_T0(), T0_BYTES, hipMemcpyHostToDevice) != hipSuccess || init_kernels() != hipSuccess) {
      (void)hipGetLastError();
      return LWE_EDEVICE;
    }
    g_noalloc_ptr[dev] = (uint8_t*)ptr;
  }
  *out = g_noalloc_ptr[dev];
  return LWE_OK;
}

}  // namespace

extern "C" int lwe_decaps_batch_noalloc(int pid, size_t count, const uint8_t* sk, const uint8_t* ct,
                                        uint8_t* ss, void* stream) {
  const Params* pp;
  LWE_CHECK(check_pid(pid, &pp));
  if (count == 0) return LWE_OK;
  if (!sk || !ct || !ss || count > LWE_MAX_BATCH) return LWE_EINVAL;
  if (!is_device_ptr(sk) || !is_device_ptr(ct) || !is_device_ptr(ss)) return LWE_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
    (void)hipGetLastError();
    return LWE_EDEVICE;
  }
  if (pp->paper) return LWE_EUNSUPPORTED;
  uint8_t* base = nullptr;
  LWE_CHECK(noalloc_base(dev, &base));
  // A transient context over the arena: device hashing on the caller's stream only (no host
  // staging, no second stream), default tuning, no profiling.
  lwe_ctx c;
  memset(c.tuning, 0, sizeof(c.tuning));
  c.device = dev;
  c.use_side = false;
  c.device_hash_only = true;
  c.d_T0 = (uint32_t*)base;
  c.arena = base + T0_BYTES;
  c.arena_cap = LWE_NOALLOC_SCRATCH_BYTES - T0_BYTES;
  // The arena holds what lwe_decaps_batch needs beyond its (device) inputs and output; the
  // same sizes as lwe_ctx_call_bytes less the staging of sk, ct and ss.
  auto r = [](size_t b) { return ((b ? b : 16) + 255) & ~(size_t)255; };
  const size_t need = lwe_ctx_call_bytes(&c, pid, 2, count) - T0_BYTES - r(pp->sk_bytes) -
                      r(count * pp->ct_bytes) - r(count * 32);
  if (need > c.arena_cap) return LWE_ENOMEM;
  return lwe_decaps_batch(&c, pid, count, sk, ct, ss, stream);
}
