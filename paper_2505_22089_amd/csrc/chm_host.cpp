// Host side of libchm: the C-ABI entry points for stores, hashing and
// matching plans.  Device memory comes only from the caller's arena.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "chm.h"
#include "chm_internal.h"
#include "chm_host.h"

using namespace chm;

static thread_local std::string g_err;

chm_status chm::fail(chm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

void chm::clear_error() { g_err.clear(); }

// Test hook (chm_debug_fail_hip): checked HIP calls of this thread left
// before the one that reports a failure without being made (0: none).
static thread_local int g_hip_fault_in = 0;

bool chm::hip_fault_due() {
  if (g_hip_fault_in <= 0) return false;
  return --g_hip_fault_in == 0;
}

extern "C" void chm_debug_fail_hip(int32_t n) { g_hip_fault_in = n > 0 ? n : 0; }

#define HIPCHK(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = chm::hip_fault_due() ? hipErrorUnknown : (call);                     \
    if (e_ != hipSuccess)                                                                \
      return chm::fail(CHM_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));        \
  } while (0)

extern "C" const char* chm_last_error(void) { return g_err.c_str(); }
extern "C" int32_t chm_abi_version(void) { return CHM_ABI_VERSION; }

extern "C" void chm_config_default(chm_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof *cfg);
  cfg->abi_version = CHM_ABI_VERSION;
  cfg->num_tables = 6;
  cfg->bucket_bits = 8;
  cfg->top_k = 8;
  cfg->ratio_num = 4;
  cfg->ratio_den = 5;
  cfg->proj_precision = CHM_PROJ_BF16;
  cfg->fixup_rel = 1e-4;
}

static chm_status check_config(const chm_config* c) {
  if (!c) return fail(CHM_E_INVALID_ARG, "config is NULL");
  if (c->abi_version != CHM_ABI_VERSION)
    return fail(CHM_E_INVALID_ARG, "config abi_version %u != %d", c->abi_version, CHM_ABI_VERSION);
  if (c->num_tables < 1 || c->num_tables > 8) return fail(CHM_E_INVALID_ARG, "num_tables must be 1..8");
  if (c->bucket_bits < 0 || c->bucket_bits > 8) return fail(CHM_E_INVALID_ARG, "bucket_bits must be 0..8");
  if (c->top_k < 1 || c->top_k > 32) return fail(CHM_E_INVALID_ARG, "top_k must be 1..32");
  if (c->ratio_num <= 0 || c->ratio_den <= 0 || c->ratio_num > c->ratio_den || c->ratio_den > 46340)
    return fail(CHM_E_INVALID_ARG, "ratio must satisfy 0 < num <= den <= 46340");
  if (c->proj_precision != CHM_PROJ_BF16 && c->proj_precision != CHM_PROJ_FP32)
    return fail(CHM_E_INVALID_ARG, "proj_precision must be CHM_PROJ_BF16 or CHM_PROJ_FP32");
  if (c->flags & ~(CHM_ACCEPT_SINGLE | CHM_WHOLE_LAST_BUCKET))
    return fail(CHM_E_INVALID_ARG, "unknown config flags 0x%x", c->flags);
  if (!(c->fixup_rel >= 1e-4 && c->fixup_rel <= 0.5))
    return fail(CHM_E_INVALID_ARG, "fixup_rel must lie in [1e-4, 0.5]");
  return CHM_OK;
}

static inline uint64_t round_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }


// ------------------------------------------------------------------ arena

bool Arena::alloc(uint64_t bytes, uint64_t* off) {
  bytes = round_up(bytes ? bytes : 1, 256);
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      const uint64_t rest = it->second - bytes;
      const uint64_t start = it->first + bytes;
      free_.erase(it);
      if (rest) free_[start] = rest;
      return true;
    }
  }
  return false;
}

void Arena::release(uint64_t off, uint64_t bytes) {
  bytes = round_up(bytes ? bytes : 1, 256);
  auto it = free_.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != free_.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    free_.erase(nx);
  }
  if (it != free_.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      free_.erase(it);
    }
  }
}

// ------------------------------------------------------------------ store

static const uint64_t kHdrW = 0;
static const uint64_t kHdrTau = round_up((uint64_t)kRowsPad * kDim * 2, 256);
static const uint64_t kHdrCmu = kHdrTau + round_up(3 * kRowsPad * 4, 256);
static const uint64_t kHdrMu = kHdrCmu + round_up(kRowsPad * 8, 256);
static const uint64_t kHdrFix = kHdrMu + 256;
static const uint64_t kHdrFixList = kHdrFix + 256;
// fix-up list: one region per projection wavefront
static const uint64_t kHdrBytes = kHdrFixList + round_up((uint64_t)kFixListCap * 4, 256);

extern "C" chm_status chm_store_overhead_bytes(const chm_config* cfg, uint64_t* out) {
  clear_error();
  chm_status st = check_config(cfg);
  if (st) return st;
  if (!out) return fail(CHM_E_INVALID_ARG, "out is NULL");
  *out = kHdrBytes;
  return CHM_OK;
}

extern "C" chm_status chm_image_bytes(const chm_config* cfg, int32_t n, uint64_t* out) {
  clear_error();
  chm_status st = check_config(cfg);
  if (st) return st;
  if (!out) return fail(CHM_E_INVALID_ARG, "out is NULL");
  if (n < 0 || n > CHM_MAX_FEATS) return fail(CHM_E_INVALID_ARG, "n_feats must be 0..%d", CHM_MAX_FEATS);
  *out = image_layout(cfg->num_tables, cfg->bucket_bits, n).total;
  return CHM_OK;
}

static bool bf16_ok(uint16_t b) {
  const int e = (b >> 7) & 0xFF;
  if ((b & 0x7FFF) == 0) return true;  // +-0
  if (e == 0xFF) return false;         // inf / nan
  // magnitude in [2^-16, 32): biased exponent 111 .. 131
  return e >= 127 - 16 && e <= 127 + 4;
}

extern "C" chm_status chm_store_create(const chm_config* cfg, const uint16_t* h_W, const uint8_t* h_mu,
                                       void* d_arena, uint64_t arena_bytes, chm_store** out) {
  clear_error();
  chm_status st = check_config(cfg);
  if (st) return st;
  if (!h_W || !h_mu || !d_arena || !out) return fail(CHM_E_INVALID_ARG, "NULL argument");
  if (((uintptr_t)d_arena) % 256) return fail(CHM_E_INVALID_ARG, "arena must be 256-byte aligned");
  if (arena_bytes < kHdrBytes) return fail(CHM_E_CAPACITY, "arena smaller than the store header");
  if (arena_bytes > (256ull << 32)) return fail(CHM_E_INVALID_ARG, "arena larger than 1 TiB");
  const int R = CHM_CODE_BITS + cfg->num_tables * cfg->bucket_bits;
  for (int i = 0; i < R * kDim; ++i)
    if (!bf16_ok(h_W[i]))
      return fail(CHM_E_INVALID_ARG, "W[%d] = 0x%04x is not 0 or of magnitude in [2^-16, 32)", i, h_W[i]);

  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  int ncu = 0;
  HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));

  std::vector<uint16_t> W(kRowsPad * kDim, 0);
  std::memcpy(W.data(), h_W, sizeof(uint16_t) * R * kDim);
  // per row: tau_r = fixup_rel ||W_r||, kappa_r = fixup_rel |c_r| (both
  // rounded up) and c_r rounded to fp32
  std::vector<float> tau(3 * kRowsPad, 0.f);
  std::vector<double> cmu(kRowsPad, 0.0);
  for (int r = 0; r < R; ++r) {
    double s = 0, c = 0;
    for (int d = 0; d < kDim; ++d) {
      uint32_t u = (uint32_t)W[r * kDim + d] << 16;
      float f;
      std::memcpy(&f, &u, 4);
      s += (double)f * (double)f;
      c += (double)f * (double)h_mu[d];  // exact: multiples of 2^-23 below 2^21
    }
    cmu[r] = c;
    auto up = [](double t) {
      float tf = (float)t;
      if ((double)tf < t) tf = std::nextafter(tf, INFINITY);
      return std::nextafter(tf, INFINITY);
    };
    tau[r] = up(cfg->fixup_rel * std::sqrt(s));
    tau[kRowsPad + r] = up(cfg->fixup_rel * std::fabs(c));
    tau[2 * kRowsPad + r] = (float)c;
  }

  chm_store* S = new chm_store();
  S->cfg = *cfg;
  S->R = R;
  S->nb = 1 << cfg->bucket_bits;
  S->base = (uint8_t*)d_arena;
  S->size = arena_bytes;
  S->n_cu = ncu;
  {
    int nx = 1;
    if (hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, dev) != hipSuccess || nx < 1) nx = 1;
    S->n_xcd = std::min(nx, kMaxBins);
    // the match kernel's LDS stage takes what one work-group may have
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) lds = 0;
    lds = std::min<int>(lds, (int)kLdsTotal);
    S->lds_top = std::max(0, lds - (int)kLdsTop) & ~15;
  }
  S->device = dev;
  S->arena.free_[kHdrBytes] = arena_bytes - kHdrBytes;
  if (arena_bytes == kHdrBytes) S->arena.free_.clear();
  S->dW = (uint16_t*)(S->base + kHdrW);
  S->dTau = (float*)(S->base + kHdrTau);
  S->dCmu = (double*)(S->base + kHdrCmu);
  S->dMu = S->base + kHdrMu;
  S->dFix = (unsigned long long*)(S->base + kHdrFix);
  S->dFixList = (uint32_t*)(S->base + kHdrFixList);
  std::memset(&S->stats, 0, sizeof S->stats);
  S->tuning.queries_per_item = 2048;
  S->tuning.wg_threads = 1024;
  S->tuning.lds_codes = 1;
  S->tuning.grid_per_cu = 1;
  S->tuning.match_kernel = CHM_KERNEL_BUCKET_MAJOR;
  S->tuning.bm_min_db_feats = lds_code_cap() + 1;
  S->tuning.group_queries = 98304;
  S->tuning.tail_percent = 8;
  S->tuning.hbm_item_queries = 512;
  hipError_t e = hipMemcpy(S->dW, W.data(), W.size() * 2, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(S->dTau, tau.data(), tau.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(S->dCmu, cmu.data(), cmu.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(S->dMu, h_mu, kDim, hipMemcpyHostToDevice);
  unsigned long long zero[2] = {0, 0};  // fix-ups, flips
  if (e == hipSuccess) e = hipMemcpy(S->dFix, zero, sizeof zero, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete S;
    return fail(CHM_E_HIP, "store setup failed: %s", hipGetErrorString(e));
  }
  *out = S;
  return CHM_OK;
}

extern "C" void chm_store_destroy(chm_store* S) {
  if (!S) return;
  (void)hipDeviceSynchronize();
  if (S->cap_stream) (void)hipStreamDestroy(S->cap_stream);
  delete S;
}

HashImage chm::hash_image_of(const chm_store* S, const ImageSlot& sl) {
  return hash_image_at(S->base + sl.off, sl.n, S->cfg.num_tables, S->cfg.bucket_bits);
}

chm_status chm::hash_images(chm_store* S, const std::vector<const ImageSlot*>& slots, hipStream_t s) {
  ProjConsts pc;
  pc.W = S->dW;
  pc.tau = S->dTau;
  pc.cmu = S->dCmu;
  pc.mu = S->dMu;
  pc.fixups = S->dFix;
  pc.fixlist = S->dFixList;
  pc.fix_cap = kFixListCap;
  pc.R = S->R;
  // descriptors per batch: the expected fix-up list (about 2800 fixup_rel
  // entries per descriptor) at most half the list
  const double per_desc = 2800.0 * S->cfg.fixup_rel;
  const int budget = (int)std::max(65536.0, std::min((double)kHashBatchDescs, kFixListCap / (2.0 * per_desc)));
  for (size_t i0 = 0; i0 < slots.size();) {
    HashBatch hb;
    std::memset(&hb, 0, sizeof hb);
    hb.arena = S->base;
    hb.L = S->cfg.num_tables;
    hb.m = S->cfg.bucket_bits;
    int cnt = 0, tiles = 0;
    int descs = 0;
    for (size_t i = i0; i < slots.size() && cnt < kHashBatch; ++i, ++cnt) {
      if (cnt > 0 && descs + slots[i]->n > budget) break;
      hb.img[cnt].off256 = (uint32_t)(slots[i]->off / 256);
      hb.img[cnt].n = slots[i]->n;
      hb.tile_prefix[cnt] = tiles;
      tiles += (slots[i]->n + 31) / 32;
      descs += slots[i]->n;
    }
    hb.tile_prefix[cnt] = tiles;
    for (int k = cnt + 1; k <= kHashBatch; ++k) hb.tile_prefix[k] = tiles;
    hb.count = cnt;
    HIPCHK(launch_project(hb, pc, S->cfg.proj_precision == CHM_PROJ_FP32, S->n_cu, s));
    HIPCHK(launch_buckets(hb, S->n_xcd, s));
    i0 += cnt;
  }
  return CHM_OK;
}

chm_status chm::load_check(const chm_store* S, int32_t count, const int32_t* ids, const void* const* descs,
                           const int32_t* n_feats) {
  if (!S) return fail(CHM_E_INVALID_ARG, "store is NULL");
  if (count < 0) return fail(CHM_E_INVALID_ARG, "count < 0");
  if (count == 0) return CHM_OK;
  if (!ids || !descs || !n_feats) return fail(CHM_E_INVALID_ARG, "NULL argument");
  std::unordered_set<int32_t> seen;
  for (int i = 0; i < count; ++i) {
    if (ids[i] < 0) return fail(CHM_E_INVALID_ARG, "image id %d < 0", ids[i]);
    if (S->images.count(ids[i])) return fail(CHM_E_INVALID_ARG, "image %d already resident", ids[i]);
    if (!seen.insert(ids[i]).second) return fail(CHM_E_INVALID_ARG, "image %d listed twice", ids[i]);
    if (n_feats[i] < 0 || n_feats[i] > CHM_MAX_FEATS)
      return fail(CHM_E_INVALID_ARG, "image %d: n_feats %d outside 0..%d", ids[i], n_feats[i], CHM_MAX_FEATS);
    if (n_feats[i] > 0 && !descs[i]) return fail(CHM_E_INVALID_ARG, "image %d: descriptors NULL", ids[i]);
  }
  return CHM_OK;
}

chm_status chm::load_alloc(chm_store* S, int32_t count, const int32_t* ids, const int32_t* n_feats,
                           std::vector<ImageSlot>* slots) {
  slots->assign((size_t)count, ImageSlot());
  for (int i = 0; i < count; ++i) {
    const ImageLayout l = image_layout(S->cfg.num_tables, S->cfg.bucket_bits, n_feats[i]);
    ImageSlot& sl = (*slots)[(size_t)i];
    sl.n = n_feats[i];
    sl.bytes = l.total;
    if (!S->arena.alloc(l.total, &sl.off)) {
      for (int k = 0; k < i; ++k) S->arena.release((*slots)[(size_t)k].off, (*slots)[(size_t)k].bytes);
      slots->clear();
      return fail(CHM_E_CAPACITY, "arena cannot hold image %d (%llu bytes)", ids[i],
                  (unsigned long long)l.total);
    }
  }
  return CHM_OK;
}

chm_status chm::load_commit(chm_store* S, int32_t count, const int32_t* ids, const void* const* descs,
                            std::vector<ImageSlot>& slots, bool on_device, hipStream_t s,
                            std::vector<const ImageSlot*>* ptrs) {
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  for (int i = 0; i < count; ++i) {
    if (slots[(size_t)i].n > 0) {
      hipError_t e = hipMemcpyAsync(S->base + slots[(size_t)i].off, descs[i], (size_t)slots[(size_t)i].n * kDim,
                                    kind, s);
      if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        for (int k = 0; k < count; ++k) S->arena.release(slots[(size_t)k].off, slots[(size_t)k].bytes);
        return fail(CHM_E_HIP, "descriptor copy failed: %s", hipGetErrorString(e));
      }
    }
  }
  for (int i = 0; i < count; ++i) {
    slots[(size_t)i].gen = ++S->gen_counter;
    auto& ref = S->images[ids[i]] = slots[(size_t)i];
    ptrs->push_back(&ref);
    S->stats.resident_bytes += ref.bytes;
    (on_device ? S->stats.d2d_bytes : S->stats.h2d_bytes) += (uint64_t)ref.n * kDim;
    S->stats.images_loaded += 1;
  }
  S->stats.resident_images = (int32_t)S->images.size();
  S->stats.resident_peak = std::max(S->stats.resident_peak, S->stats.resident_bytes);
  return CHM_OK;
}

extern "C" chm_status chm_store_load(chm_store* S, int32_t count, const int32_t* ids,
                                     const void* const* descs, const int32_t* n_feats,
                                     int32_t on_device, void* stream) {
  clear_error();
  chm_status st = load_check(S, count, ids, descs, n_feats);
  if (st || count == 0) return st;
  std::vector<ImageSlot> slots;
  st = load_alloc(S, count, ids, n_feats, &slots);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  std::vector<const ImageSlot*> ptrs;
  st = load_commit(S, count, ids, descs, slots, on_device != 0, s, &ptrs);
  if (st) return st;
  return hash_images(S, ptrs, s);
}

extern "C" chm_status chm_store_rehash(chm_store* S, int32_t count, const int32_t* ids, void* stream) {
  clear_error();
  if (!S) return fail(CHM_E_INVALID_ARG, "store is NULL");
  if (count < 0 || (count > 0 && !ids)) return fail(CHM_E_INVALID_ARG, "bad image list");
  std::vector<const ImageSlot*> ptrs;
  for (int i = 0; i < count; ++i) {
    auto it = S->images.find(ids[i]);
    if (it == S->images.end()) return fail(CHM_E_NOT_RESIDENT, "image %d is not resident", ids[i]);
    ptrs.push_back(&it->second);
  }
  return hash_images(S, ptrs, (hipStream_t)stream);
}

chm_status chm::evict_hold(chm_store* S, int32_t count, const int32_t* ids,
                           std::vector<std::pair<uint64_t, uint64_t>>* held) {
  if (!S) return fail(CHM_E_INVALID_ARG, "store is NULL");
  if (count < 0 || (count > 0 && !ids)) return fail(CHM_E_INVALID_ARG, "bad image list");
  for (int i = 0; i < count; ++i)
    if (!S->images.count(ids[i])) return fail(CHM_E_NOT_RESIDENT, "image %d is not resident", ids[i]);
  for (int i = 0; i < count; ++i) {
    auto it = S->images.find(ids[i]);
    if (it == S->images.end()) continue;  // listed twice
    if (held)
      held->push_back({it->second.off, it->second.bytes});
    else
      S->arena.release(it->second.off, it->second.bytes);
    S->stats.resident_bytes -= it->second.bytes;
    S->stats.images_evicted += 1;
    S->images.erase(it);
  }
  S->stats.resident_images = (int32_t)S->images.size();
  return CHM_OK;
}

void chm::release_held(chm_store* S, std::vector<std::pair<uint64_t, uint64_t>>* held) {
  for (auto& h : *held) S->arena.release(h.first, h.second);
  held->clear();
}

extern "C" chm_status chm_store_evict(chm_store* S, int32_t count, const int32_t* ids) {
  clear_error();
  return evict_hold(S, count, ids, nullptr);
}

extern "C" chm_status chm_store_image_feats(const chm_store* S, int32_t id, int32_t* out) {
  clear_error();
  if (!S || !out) return fail(CHM_E_INVALID_ARG, "NULL argument");
  auto it = S->images.find(id);
  *out = it == S->images.end() ? -1 : it->second.n;
  return CHM_OK;
}

extern "C" chm_status chm_store_stats(chm_store* S, chm_stats* out) {
  clear_error();
  if (!S || !out) return fail(CHM_E_INVALID_ARG, "NULL argument");
  HIPCHK(hipDeviceSynchronize());
  unsigned long long fl[2] = {0, 0};
  HIPCHK(hipMemcpy(fl, S->dFix, sizeof fl, hipMemcpyDeviceToHost));
  S->stats.fixups = fl[0];
  S->stats.fixup_flips = fl[1];
  *out = S->stats;
  return CHM_OK;
}

extern "C" chm_status chm_debug_image(chm_store* S, int32_t id, uint32_t* d_codes, uint8_t* d_ids,
                                      int32_t* d_offsets, uint16_t* d_members, uint32_t* d_norms,
                                      void* stream) {
  clear_error();
  if (!S) return fail(CHM_E_INVALID_ARG, "store is NULL");
  auto it = S->images.find(id);
  if (it == S->images.end()) return fail(CHM_E_NOT_RESIDENT, "image %d is not resident", id);
  const HashImage h = hash_image_of(S, it->second);
  hipStream_t s = (hipStream_t)stream;
  const int L = S->cfg.num_tables;
  const size_t n = (size_t)h.n;
  if (d_codes && n) HIPCHK(hipMemcpyAsync(d_codes, h.codes, n * 16, hipMemcpyDeviceToDevice, s));
  if (d_ids && n)
    HIPCHK(hipMemcpy2DAsync(d_ids, n, h.ids, (size_t)h.n_pad, n, L, hipMemcpyDeviceToDevice, s));
  if (d_norms && n) HIPCHK(hipMemcpyAsync(d_norms, h.norms, n * 4, hipMemcpyDeviceToDevice, s));
  if (d_offsets || d_members) {
    // The device tables hold padded bucket ranges; hand out the plain tables
    // (each bucket's members only), recovered as the strictly increasing
    // prefix of each padded range.
    const size_t nb1 = (size_t)S->nb + 1;
    std::vector<int32_t> po((size_t)L * nb1), ro((size_t)L * nb1);
    std::vector<uint32_t> pm((size_t)L * h.m_stride + 1);
    std::vector<uint16_t> rm((size_t)L * n + 1);
    HIPCHK(hipMemcpyAsync(po.data(), h.offsets, po.size() * 4, hipMemcpyDeviceToHost, s));
    if (h.m_stride)
      HIPCHK(hipMemcpyAsync(pm.data(), h.members, (size_t)L * h.m_stride * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int t = 0; t < L; ++t) {
      const int32_t* o = po.data() + t * nb1;
      const uint32_t* mm = pm.data() + (size_t)t * h.m_stride;
      size_t pos = 0;
      for (size_t b = 0; b + 1 < nb1; ++b) {
        ro[t * nb1 + b] = (int32_t)pos;
        if (o[b] < 0 || o[b] > o[b + 1] || o[b + 1] > h.m_stride || (o[b] & 7))
          return fail(CHM_E_INTERNAL, "table %d bucket %zu: bad padded range", t, b);
        for (int32_t k = o[b]; k < o[b + 1] && (k == o[b] || mm[k] > mm[k - 1]); ++k) {
          if (pos >= n) return fail(CHM_E_INTERNAL, "table %d holds more than n members", t);
          if ((mm[k] & 15u) || (mm[k] >> 4) >= n)
            return fail(CHM_E_INTERNAL, "table %d: member %u is no code offset", t, mm[k]);
          rm[(size_t)t * n + pos++] = (uint16_t)(mm[k] >> 4);
        }
      }
      ro[t * nb1 + nb1 - 1] = (int32_t)pos;
      if (pos != n) return fail(CHM_E_INTERNAL, "table %d holds %zu members, not %zu", t, pos, n);
    }
    if (d_offsets) HIPCHK(hipMemcpyAsync(d_offsets, ro.data(), ro.size() * 4, hipMemcpyHostToDevice, s));
    if (d_members && n)
      HIPCHK(hipMemcpyAsync(d_members, rm.data(), (size_t)L * n * 2, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  return CHM_OK;
}

extern "C" chm_status chm_store_get_tuning(const chm_store* S, chm_tuning* out) {
  clear_error();
  if (!S || !out) return fail(CHM_E_INVALID_ARG, "NULL argument");
  *out = S->tuning;
  return CHM_OK;
}

extern "C" chm_status chm_store_set_tuning(chm_store* S, const chm_tuning* t) {
  clear_error();
  if (!S || !t) return fail(CHM_E_INVALID_ARG, "NULL argument");
  if (t->queries_per_item < 64 || t->queries_per_item > 8192 || t->queries_per_item % 64)
    return fail(CHM_E_INVALID_ARG, "queries_per_item must be a multiple of 64 in 64..8192");
  if (t->wg_threads != 256 && t->wg_threads != 1024)
    return fail(CHM_E_INVALID_ARG, "wg_threads must be 256 or 1024");
  if (t->lds_codes != 0 && t->lds_codes != 1) return fail(CHM_E_INVALID_ARG, "lds_codes must be 0 or 1");
  if (t->grid_per_cu < 1 || t->grid_per_cu > 8) return fail(CHM_E_INVALID_ARG, "grid_per_cu must be 1..8");
  if (t->match_kernel != CHM_KERNEL_QUERY_MAJOR && t->match_kernel != CHM_KERNEL_BUCKET_MAJOR)
    return fail(CHM_E_INVALID_ARG, "match_kernel must be CHM_KERNEL_QUERY_MAJOR or CHM_KERNEL_BUCKET_MAJOR");
  if (t->bm_min_db_feats < 0 || t->bm_min_db_feats > 65536)
    return fail(CHM_E_INVALID_ARG, "bm_min_db_feats must be 0..65536");
  if (t->group_queries < 1 || t->group_queries > (1 << 20))
    return fail(CHM_E_INVALID_ARG, "group_queries must be 1..1048576");
  if (t->tail_percent < 0 || t->tail_percent > 50) return fail(CHM_E_INVALID_ARG, "tail_percent must be 0..50");
  if (t->hbm_item_queries < 64 || t->hbm_item_queries > 8192 || t->hbm_item_queries % 64)
    return fail(CHM_E_INVALID_ARG, "hbm_item_queries must be a multiple of 64 in 64..8192");
  S->tuning = *t;
  return CHM_OK;
}

// ------------------------------------------------------------------ plans

int chm::lds_max_feats(const chm_store* S) {
  return std::min(lds_code_cap(), S->lds_top / 16);
}

static ImageDev image_dev(const chm_store* S, const ImageSlot& sl) {
  const HashImage h = hash_image_of(S, sl);
  ImageDev d;
  d.desc = h.desc;
  d.codes = h.codes;
  d.ids = h.ids;
  d.norms = h.norms;
  d.offsets = h.offsets;
  d.counts = h.counts;
  d.members = h.members;
  d.tcodes = h.tcodes;
  d.n = h.n;
  d.n_pad = h.n_pad;
  d.m_stride = h.m_stride;
  d.reserved = 0;
  return d;
}

// Query-major batched plans halve the items that end each bin (the tail
// fraction is chm_tuning.tail_percent).
static constexpr int kTailPieces = 2;

// Kept-list state of the bucket-major part of a plan: at most this much
// arena per round.
static constexpr uint64_t kBmStateMax = 512ull << 20;
static constexpr int kBmMaxGroupPairs = 32;

static int kept_slots(int K) { return K <= 2 ? 2 : K <= 4 ? 4 : K <= 8 ? 8 : K <= 16 ? 16 : 32; }

// The bucket-major part of a batched plan, before upload.
struct BmPart {
  std::vector<int> order;        // the part's pairs (indices into pd) in group order
  std::vector<int64_t> st_off;   // state row of each, per order position
  std::vector<int32_t> ints;     // group ranges (absolute pair indices), then the rounds' bin tables
  std::vector<chm_plan::BmRound> rounds;
  int groups = 0;
};

// Groups the pairs idx (into pd) for bucket-major matching: ordered by db
// image, a group holds pairs with one db image whose query images have at
// most tuning.group_queries descriptors together (at most kBmMaxGroupPairs
// pairs).  Groups go into rounds whose kept lists (KT keys per query) fit
// one state block of the arena (allocated here), and inside a round into
// one bin per XCD, most expensive first onto the least loaded bin.  The
// part's pairs will sit at first_pair.. of the plan's pair array.
// CHM_E_CAPACITY when not even one group's lists fit.
static chm_status bm_part(chm_store* S, chm_plan* pl, const std::vector<PairDev>& pd, const std::vector<int>& idx,
                          int first_pair, uint64_t keep_free, BmPart* bp) {
  const int P = (int)idx.size();
  const int L = S->cfg.num_tables;
  const uint64_t row_bytes = 4ull * (uint64_t)kept_slots(S->cfg.top_k);
  const int nbins = std::max(1, S->n_xcd);
  std::vector<int>& ord = bp->order;
  ord = idx;
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
    if (pd[x].d.codes != pd[y].d.codes) return pd[x].d.codes < pd[y].d.codes;
    return pd[x].q.codes < pd[y].q.codes;
  });
  std::vector<int> gstart;
  int64_t gq = 0;
  for (int i = 0; i < P; ++i) {
    const PairDev& x = pd[ord[i]];
    const bool fresh = i == 0 || x.d.codes != pd[ord[i - 1]].d.codes || i - gstart.back() >= kBmMaxGroupPairs ||
                       (gq + x.q.n > pl->tun.group_queries && gq > 0);
    if (fresh) {
      gstart.push_back(i);
      gq = 0;
    }
    gq += x.q.n;
  }
  const int G = (int)gstart.size();
  gstart.push_back(P);
  std::vector<uint64_t> gstate(G, 0);
  std::vector<double> gcost(G, 0.0);
  uint64_t total_state = 0, max_state = 0;
  for (int g = 0; g < G; ++g) {
    for (int i = gstart[g]; i < gstart[g + 1]; ++i) {
      const PairDev& x = pd[ord[i]];
      gstate[g] += row_bytes * (uint64_t)x.q.n;
      gcost[g] += (double)x.q.n * (double)(x.d.n + 64);
    }
    gstate[g] = round_up(gstate[g], 256);
    total_state += gstate[g];
    max_state = std::max(max_state, gstate[g]);
  }
  // the state block: all groups' lists if they fit, else the largest block
  // (halving) that still holds the largest group; L = 1 keeps no lists.
  // keep_free bytes stay free for the rest of the plan (reserved meanwhile).
  uint64_t want = L > 1 ? std::min(total_state, std::max(kBmStateMax, max_state)) : 0;
  if (want > 0) {
    uint64_t keep_off = 0;
    const bool kept = S->arena.alloc(keep_free, &keep_off);
    if (!kept) return fail(CHM_E_CAPACITY, "arena cannot hold the plan");
    bool got = false;
    for (;;) {
      if (S->arena.alloc(want, &pl->state_off)) {
        got = true;
        break;
      }
      if (want / 2 < max_state) break;
      want = std::max(max_state, round_up(want / 2, 256));
    }
    S->arena.release(keep_off, keep_free);
    if (!got) return fail(CHM_E_CAPACITY, "arena cannot hold the kept lists of a group");
    pl->state_bytes = want;
    pl->dState = (uint32_t*)(S->base + pl->state_off);
  }
  std::vector<std::vector<int>> rounds;
  uint64_t used = 0;
  for (int g = 0; g < G; ++g) {
    if (rounds.empty() || (want > 0 && used + gstate[g] > want)) {
      rounds.emplace_back();
      used = 0;
    }
    rounds.back().push_back(g);
    used += gstate[g];
  }
  bp->st_off.assign(P, 0);
  bp->ints.clear();
  for (int g = 0; g <= G; ++g) bp->ints.push_back(first_pair + gstart[g]);
  for (auto& r : rounds) {
    uint64_t row = 0;
    for (int g : r)
      for (int i = gstart[g]; i < gstart[g + 1]; ++i) {
        bp->st_off[i] = (int64_t)row;
        row += (uint64_t)pd[ord[i]].q.n;
      }
    std::vector<int> og(r);
    std::stable_sort(og.begin(), og.end(), [&](int x, int y) { return gcost[x] > gcost[y]; });
    std::vector<std::vector<int>> bins(nbins);
    std::vector<double> load(nbins, 0.0);
    for (int g : og) {
      const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[b] += gcost[g];
      bins[b].push_back(g);
    }
    chm_plan::BmRound br;
    br.begin_off = (int)bp->ints.size();
    br.max_groups = 0;
    int acc = 0;
    for (int b = 0; b < nbins; ++b) {
      bp->ints.push_back(acc);
      acc += (int)bins[b].size();
      br.max_groups = std::max(br.max_groups, (int)bins[b].size());
    }
    bp->ints.push_back(acc);
    br.list_off = (int)bp->ints.size();
    for (int b = 0; b < nbins; ++b) bp->ints.insert(bp->ints.end(), bins[b].begin(), bins[b].end());
    bp->rounds.push_back(br);
  }
  bp->groups = G;
  return CHM_OK;
}

chm_status chm::plan_build(chm_store* S, const int32_t* h_pairs, int32_t P, const int64_t* starts,
                           int32_t* d_out, uint32_t* d_topk, int32_t mode, void* stream,
                           chm_plan** out, bool wait_upload) {
  if (mode != CHM_MATCH_PLAIN && mode != CHM_MATCH_BATCHED) return fail(CHM_E_INVALID_ARG, "bad mode");
  std::vector<PairDev> pd(P);
  std::unordered_map<int32_t, uint64_t> gens;
  int64_t total_out = 0;
  for (int p = 0; p < P; ++p) {
    auto iq = S->images.find(h_pairs[2 * p]);
    auto id = S->images.find(h_pairs[2 * p + 1]);
    if (iq == S->images.end() || id == S->images.end())
      return fail(CHM_E_NOT_RESIDENT, "pair %d names an image that is not resident", p);
    if (starts[p] < 0) return fail(CHM_E_INVALID_ARG, "negative output offset");
    pd[p].q = image_dev(S, iq->second);
    pd[p].d = image_dev(S, id->second);
    pd[p].out_off = starts[p];
    pd[p].st_off = 0;
    total_out += iq->second.n;
    gens[iq->first] = iq->second.gen;
    gens[id->first] = id->second.gen;
  }
  if (total_out > 0 && !d_out) return fail(CHM_E_INVALID_ARG, "d_out is NULL");

  chm_plan* pl = new chm_plan();
  pl->st = S;
  pl->mode = mode;
  pl->n_pairs = P;
  pl->out = d_out;
  pl->topk = d_topk;
  pl->gens.assign(gens.begin(), gens.end());
  pl->tun = S->tuning;
  const int ldsmax = pl->tun.lds_codes ? lds_max_feats(S) : 0;
  pl->lds_max = ldsmax;

  // Batched plans match pairs whose db image has at least
  // tuning.bm_min_db_feats points bucket major, the others query major.
  std::vector<int> qm_idx, bm_idx;
  const bool bm_ok = mode == CHM_MATCH_BATCHED && pl->tun.match_kernel == CHM_KERNEL_BUCKET_MAJOR &&
                     !(S->cfg.flags & CHM_WHOLE_LAST_BUCKET);
  for (int p = 0; p < P; ++p) (bm_ok && pd[p].d.n >= pl->tun.bm_min_db_feats ? bm_idx : qm_idx).push_back(p);
  BmPart bp;
  if (!bm_idx.empty()) {
    // room the rest of the plan may need: all pairs, one query-major item
    // per 64 queries and pair, the queue and bin words, the group tables
    uint64_t items_max = 0;
    for (const PairDev& x : pd) items_max += (uint64_t)(x.q.n + 63) / 64 + 1;
    const uint64_t keep_free = round_up(sizeof(PairDev) * (uint64_t)P, 256) + round_up(sizeof(WorkItem) * items_max, 256) +
                               512 + round_up(4ull * (uint64_t)bm_idx.size() * (uint64_t)(std::max(1, S->n_xcd) + 3) + 4, 256);
    const chm_status bst = bm_part(S, pl, pd, bm_idx, (int)qm_idx.size(), keep_free, &bp);
    if (bst == CHM_E_CAPACITY) {  // the kept lists do not fit the arena: all query major
      clear_error();
      qm_idx.insert(qm_idx.end(), bm_idx.begin(), bm_idx.end());
      std::sort(qm_idx.begin(), qm_idx.end());
      bm_idx.clear();
      bp = BmPart();
    } else if (bst) {
      delete pl;
      return bst;
    }
  }
  // the plan's pair array: the query-major pairs in input order, then the
  // bucket-major ones in group order
  std::vector<PairDev> fp;
  fp.reserve(P);
  for (int p : qm_idx) fp.push_back(pd[p]);
  for (size_t i = 0; i < bp.order.size(); ++i) {
    fp.push_back(pd[bp.order[i]]);
    fp.back().st_off = bp.st_off[i];
  }

  std::vector<WorkItem> items;
  {
    const std::vector<PairDev>& pd = fp;  // the query-major pairs come first
    const int P = (int)qm_idx.size();
    if (mode == CHM_MATCH_PLAIN) {
      const int qp = pl->tun.wg_threads;
      pl->pair_begin.resize(P);
      pl->pair_count.resize(P);
      pl->pair_lds.resize(P);
      for (int p = 0; p < P; ++p) {
        const bool lds = ldsmax > 0 && pd[p].d.n <= ldsmax && pd[p].d.n > 0;
        pl->pair_begin[p] = (int)items.size();
        for (int q0 = 0; q0 < pd[p].q.n; q0 += qp)
          items.push_back({p, q0, std::min(pd[p].q.n, q0 + qp), lds ? 1 : 0});
        pl->pair_count[p] = (int)items.size() - pl->pair_begin[p];
        pl->pair_lds[p] = lds;
      }
    } else {
      // All items go to one persistent launch: the LDS-staging kernel when any
      // db image fits the code stage (it reads larger ones from HBM in the same
      // launch), else the HBM-only kernel.  Items are dealt into one bin per
      // XCD, whole db images at a time (largest total first onto the least
      // loaded bin), so the work-groups of an XCD share the db images' codes,
      // members and descriptors in their L2; inside a bin, a db image's items
      // are consecutive, longest first.
      const int qpi = pl->tun.queries_per_item;
      const int nbins = std::max(1, S->n_xcd);
      std::map<const void*, std::vector<std::pair<double, WorkItem>>> groups;
      for (int p = 0; p < P; ++p) pl->lds_launch |= ldsmax > 0 && pd[p].d.n <= ldsmax && pd[p].d.n > 0;
      for (int p = 0; p < P; ++p) {
        const bool lds = ldsmax > 0 && pd[p].d.n <= ldsmax && pd[p].d.n > 0;
        // Above a large stage an item's sort order may not fit: such pairs
        // take items small enough to sort, down to one query per thread of a
        // 1024-thread work-group; below that they keep full items, unsorted.
        // A launch without any staged pair takes items of at most
        // tuning.hbm_item_queries queries.
        int qp = qpi;
        if (lds) {
          const int room = lds_sort_room(S->lds_top, pd[p].d.n) / 64 * 64;
          if (room < qp && room >= 1024) qp = room;
        } else if (!pl->lds_launch) {
          // the HBM-only kernel ran 512-query items 9% faster than 2048-query
          // ones on 40k-feature images; in the staging kernel's launch the
          // smaller items were slower
          qp = std::min(qp, pl->tun.hbm_item_queries);
        }
        for (int q0 = 0; q0 < pd[p].q.n; q0 += qp) {
          WorkItem w{p, q0, std::min(pd[p].q.n, q0 + qp), lds ? 1 : 0};
          const double cost = (double)(w.q1 - w.q0) * (double)(pd[p].d.n + 64);
          groups[pd[p].d.codes].push_back({cost, w});
        }
      }
      std::vector<std::pair<double, std::vector<std::pair<double, WorkItem>>*>> order;
      for (auto& g : groups) {
        double c = 0;
        for (auto& x : g.second) c += x.first;
        std::sort(g.second.begin(), g.second.end(),
                  [](const std::pair<double, WorkItem>& x, const std::pair<double, WorkItem>& y) {
                    if (x.first != y.first) return x.first > y.first;
                    if (x.second.pair != y.second.pair) return x.second.pair < y.second.pair;
                    return x.second.q0 < y.second.q0;
                  });
        order.push_back({c, &g.second});
      }
      std::stable_sort(order.begin(), order.end(),
                       [](const auto& x, const auto& y) { return x.first > y.first; });
      std::vector<std::vector<WorkItem>> bins(nbins);
      std::vector<double> load(nbins, 0.0);
      for (auto& g : order) {
        const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[b] += g.first;
        for (auto& x : *g.second) bins[b].push_back(x.second);
      }
      // The items that make up the last tail_percent of a bin's cost are cut
      // into kTailPieces pieces (whole wavefront chunks), so that the
      // work-groups draining the bins finish within a smaller item of each
      // other rather than a full one.
      const int tail_pct = pl->tun.tail_percent;
      for (int b = 0; b < nbins && tail_pct > 0; ++b) {
        std::vector<WorkItem>& v = bins[b];
        auto cost = [&](const WorkItem& w) { return (double)(w.q1 - w.q0) * (double)(pd[w.pair].d.n + 64); };
        double total = 0, tail = 0;
        for (const WorkItem& w : v) total += cost(w);
        size_t cut = v.size();
        while (cut > 0 && tail < total * tail_pct / 100.0) tail += cost(v[--cut]);
        std::vector<WorkItem> out(v.begin(), v.begin() + cut);
        for (size_t i = cut; i < v.size(); ++i) {
          const WorkItem& w = v[i];
          const int piece = std::max(64, ((w.q1 - w.q0 + kTailPieces - 1) / kTailPieces + 63) / 64 * 64);
          for (int q0 = w.q0; q0 < w.q1; q0 += piece) out.push_back({w.pair, q0, std::min(w.q1, q0 + piece), w.lds});
        }
        v.swap(out);
      }
      pl->bins[0] = 0;
      for (int b = 0; b < nbins; ++b) {
        items.insert(items.end(), bins[b].begin(), bins[b].end());
        pl->bins[b + 1] = (int32_t)items.size();
      }
      pl->n_bins = nbins;
    }
  }
  pl->n_items = (int)items.size();
  pl->bm = !bm_idx.empty();
  pl->bm_groups = bp.groups;
  pl->bm_rounds = bp.rounds;

  const uint64_t pairs_bytes = round_up(sizeof(PairDev) * (size_t)std::max(P, 1), 256);
  const uint64_t items_bytes = round_up(sizeof(WorkItem) * (size_t)std::max(pl->n_items, 1), 256);
  const uint64_t queue_bytes = 256;  // kMaxBins counters
  const uint64_t bins_bytes = 256;   // kMaxBins + 1 item offsets
  const uint64_t ints_bytes = round_up(4 * std::max<size_t>(bp.ints.size(), 1), 256);
  static_assert(kMaxBins * 4 <= 256 && (kMaxBins + 1) * 4 <= 256, "plan tail");
  pl->mem_bytes = pairs_bytes + items_bytes + queue_bytes + bins_bytes + ints_bytes;
  if (!S->arena.alloc(pl->mem_bytes, &pl->mem_off)) {
    if (pl->state_bytes) S->arena.release(pl->state_off, pl->state_bytes);
    delete pl;
    return fail(CHM_E_CAPACITY, "arena cannot hold the plan's work list (%llu bytes)",
                (unsigned long long)pl->mem_bytes);
  }
  pl->dPairs = (PairDev*)(S->base + pl->mem_off);
  pl->dItems = (WorkItem*)(S->base + pl->mem_off + pairs_bytes);
  pl->dQueue = (uint32_t*)(S->base + pl->mem_off + pairs_bytes + items_bytes);
  pl->dBins = (int32_t*)(S->base + pl->mem_off + pairs_bytes + items_bytes + queue_bytes);
  pl->dBmInts = (int32_t*)(S->base + pl->mem_off + pairs_bytes + items_bytes + queue_bytes + bins_bytes);
  // the plan owns the host sources of its upload (and its bin table), so the
  // copies may still be in flight when this call returns
  pl->h_pairs = std::move(fp);
  pl->h_items = std::move(items);
  pl->h_bm_ints = std::move(bp.ints);
  hipStream_t s = (hipStream_t)stream;
  pl->upload_stream = s;
  pl->upload_pending = true;
  hipError_t e = hipSuccess;
  if (P) e = hipMemcpyAsync(pl->dPairs, pl->h_pairs.data(), sizeof(PairDev) * P, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && pl->n_items)
    e = hipMemcpyAsync(pl->dItems, pl->h_items.data(), sizeof(WorkItem) * pl->n_items, hipMemcpyHostToDevice,
                       s);
  if (e == hipSuccess) e = hipMemcpyAsync(pl->dBins, pl->bins, sizeof pl->bins, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !pl->h_bm_ints.empty())
    e = hipMemcpyAsync(pl->dBmInts, pl->h_bm_ints.data(), 4 * pl->h_bm_ints.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && wait_upload) {
    e = hipStreamSynchronize(s);
    pl->upload_pending = false;
  }
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(s);
    plan_free(pl);
    return fail(CHM_E_HIP, "plan upload failed: %s", hipGetErrorString(e));
  }

  MatchArgs& a = pl->args;
  a.pairs = pl->dPairs;
  a.items = pl->dItems;
  a.n_items = 0;
  a.item_base = 0;
  a.queue = pl->dQueue;
  a.bin_begin = pl->dBins;
  a.n_bins = 1;
  a.out = d_out;
  a.topk = d_topk;
  a.L = S->cfg.num_tables;
  a.nb = S->nb;
  a.K = S->cfg.top_k;
  a.ratio_num = S->cfg.ratio_num;
  a.ratio_den = S->cfg.ratio_den;
  a.accept_single = (S->cfg.flags & CHM_ACCEPT_SINGLE) ? 1 : 0;
  a.whole_bucket = (S->cfg.flags & CHM_WHOLE_LAST_BUCKET) ? 1 : 0;
  a.lds_max_feats = ldsmax;
  a.lds_top = S->lds_top;

  if (mode == CHM_MATCH_BATCHED && (pl->n_items > 0 || pl->bm_groups > 0)) {
    // one graph: the query-major persistent launch (its queue counters reset
    // by a fill kernel), then the bucket-major launches, table by table and
    // round by round
    hipStream_t cs = S->cap_stream;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess && pl->n_items > 0) {
      e = launch_fill_u32(pl->dQueue, 0u, kMaxBins, cs);
      if (e == hipSuccess) {
        MatchArgs x = a;
        x.n_items = pl->n_items;
        x.n_bins = pl->n_bins;
        // the LDS stage allows one work-group per CU
        const int per_cu = pl->lds_launch ? 1 : pl->tun.grid_per_cu;
        if (!pl->lds_launch) x.lds_max_feats = 0;
        const int grid = std::min(pl->n_items, S->n_cu * per_cu);
        e = launch_match(x, a.K, pl->tun.wg_threads, pl->lds_launch, true, grid, cs);
      }
    }
    const int nbins = std::max(1, S->n_xcd);
    for (size_t r = 0; r < pl->bm_rounds.size() && e == hipSuccess; ++r) {
      BmArgs b;
      b.pairs = pl->dPairs;
      b.groups = pl->dBmInts;
      b.bin_begin = pl->dBmInts + pl->bm_rounds[r].begin_off;
      b.bin_groups = pl->dBmInts + pl->bm_rounds[r].list_off;
      b.state = pl->dState;
      b.out = d_out;
      b.topk = d_topk;
      b.n_bins = nbins;
      b.L = a.L;
      b.nb = a.nb;
      b.K = a.K;
      b.ratio_num = a.ratio_num;
      b.ratio_den = a.ratio_den;
      b.accept_single = a.accept_single;
      const int grid = nbins * pl->bm_rounds[r].max_groups * S->nb;
      for (int t = 0; t < a.L && e == hipSuccess; ++t) {
        b.t = t;
        e = launch_match_bm(b, a.K, grid, cs);
      }
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      if (pl->upload_pending) (void)hipStreamSynchronize(s);
      plan_free(pl);
      return fail(CHM_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    }
  }
  *out = pl;
  return CHM_OK;
}

extern "C" chm_status chm_plan_create(chm_store* S, const int32_t* h_pairs, int32_t P,
                                      const int64_t* h_offs, int32_t* d_out, uint32_t* d_topk,
                                      int32_t mode, void* stream, chm_plan** out) {
  clear_error();
  if (!S || !out) return fail(CHM_E_INVALID_ARG, "NULL argument");
  if (P < 0 || (P > 0 && (!h_pairs || !h_offs))) return fail(CHM_E_INVALID_ARG, "bad pair list");
  for (int p = 0; p < P; ++p) {
    auto iq = S->images.find(h_pairs[2 * p]);
    if (iq == S->images.end() || !S->images.count(h_pairs[2 * p + 1]))
      return fail(CHM_E_NOT_RESIDENT, "pair %d names an image that is not resident", p);
    if (h_offs[p + 1] - h_offs[p] != iq->second.n)
      return fail(CHM_E_INVALID_ARG, "pair %d: output range %lld != query features %d", p,
                  (long long)(h_offs[p + 1] - h_offs[p]), iq->second.n);
  }
  return plan_build(S, h_pairs, P, h_offs, d_out, d_topk, mode, stream, out);
}

static bool plan_fresh(const chm_plan* pl) {
  for (auto& g : pl->gens) {
    auto it = pl->st->images.find(g.first);
    if (it == pl->st->images.end() || it->second.gen != g.second) return false;
  }
  return true;
}

extern "C" chm_status chm_plan_execute(chm_plan* pl, void* stream) {
  clear_error();
  if (!pl) return fail(CHM_E_INVALID_ARG, "plan is NULL");
  if (!plan_fresh(pl)) return fail(CHM_E_NOT_RESIDENT, "an image of the plan was evicted or reloaded");
  hipStream_t s = (hipStream_t)stream;
  pl->last_stream = s;
  pl->executed = true;
  if (pl->n_items == 0 && pl->bm_groups == 0) return CHM_OK;
  if (pl->mode == CHM_MATCH_BATCHED) {
    HIPCHK(hipGraphLaunch(pl->exec, s));
    return CHM_OK;
  }
  for (int p = 0; p < pl->n_pairs; ++p) {
    if (pl->pair_count[p] == 0) continue;
    MatchArgs x = pl->args;
    x.n_items = pl->n_items;
    x.item_base = pl->pair_begin[p];
    if (!pl->pair_lds[p]) x.lds_max_feats = 0;
    HIPCHK(launch_match(x, x.K, pl->tun.wg_threads, pl->pair_lds[p] != 0, false, pl->pair_count[p], s));
  }
  return CHM_OK;
}

void chm::plan_free(chm_plan* pl) {
  if (!pl) return;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  pl->st->arena.release(pl->mem_off, pl->mem_bytes);
  if (pl->state_bytes) pl->st->arena.release(pl->state_off, pl->state_bytes);
  delete pl;
}

extern "C" void chm_plan_destroy(chm_plan* pl) {
  if (!pl) return;
  if (pl->upload_pending) (void)hipStreamSynchronize(pl->upload_stream);
  if (pl->executed) (void)hipStreamSynchronize(pl->last_stream);
  plan_free(pl);
}

extern "C" chm_status chm_match_pairs(chm_store* S, const int32_t* h_pairs, int32_t P,
                                      const int64_t* h_offs, int32_t* d_out, int32_t mode,
                                      void* stream) {
  chm_plan* pl = nullptr;
  chm_status st = chm_plan_create(S, h_pairs, P, h_offs, d_out, nullptr, mode, stream, &pl);
  if (st) return st;
  st = chm_plan_execute(pl, stream);
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  chm_plan_destroy(pl);
  if (st) return st;
  if (e != hipSuccess) return fail(CHM_E_HIP, "matching failed: %s", hipGetErrorString(e));
  return CHM_OK;
}
