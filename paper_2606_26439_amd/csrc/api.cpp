// api.cpp -- the C ABI of include/maxsim.h: argument validation (before any
// work is enqueued), kernel selection, workspace sizing, error reporting and
// the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/maxsim.h"
#include "kernels.h"

namespace {

thread_local std::string g_err;

maxsim_status fail(maxsim_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

maxsim_status hip_fail(hipError_t e, const char* what) {
  return fail(MAXSIM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int esize(int dt) { return dt == MAXSIM_F32 ? 4 : (dt == MAXSIM_F8E4M3 ? 1 : 2); }

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

maxsim_status check_csr(const maxsim_csr* c, const char* name, bool is_query) {
  if (!c) return fail(MAXSIM_EINVAL, "%s: descriptor is NULL", name);
  if (c->dtype < MAXSIM_F32 || c->dtype > MAXSIM_F8E4M3)
    return fail(MAXSIM_EINVAL, "%s: unknown dtype %d", name, c->dtype);
  if (c->dim < 16 || c->dim > 1024 || c->dim % 16 != 0)
    return fail(MAXSIM_EUNSUPPORTED, "%s: dim %d must be a multiple of 16 in [16, 1024]", name,
                c->dim);
  if (c->n_sets < 0 || c->n_tokens < 0)
    return fail(MAXSIM_EINVAL, "%s: negative n_sets or n_tokens", name);
  if (c->max_len < 0) return fail(MAXSIM_EINVAL, "%s: negative max_len", name);
  if (is_query && c->max_len > 64)
    return fail(MAXSIM_EUNSUPPORTED, "%s: max_len %d exceeds 64 query tokens", name, c->max_len);
  if (!c->offsets) return fail(MAXSIM_EINVAL, "%s: offsets is NULL", name);
  if (c->n_tokens > 0 && !c->tokens) return fail(MAXSIM_EINVAL, "%s: tokens is NULL", name);
  if (c->tokens && !aligned(c->tokens, 16))
    return fail(MAXSIM_EINVAL, "%s: tokens must be 16-byte aligned", name);
  if (!aligned(c->offsets, 8)) return fail(MAXSIM_EINVAL, "%s: offsets must be 8-byte aligned", name);
  if (c->dtype == MAXSIM_F8E4M3 && c->n_tokens > 0 && !c->scales)
    return fail(MAXSIM_EINVAL, "%s: FP8 tokens need per-token scales", name);
  return MAXSIM_OK;
}

int nqb_for(int max_len) { return max_len <= 16 ? 1 : (max_len <= 32 ? 2 : 4); }

struct DevInfo {
  int cus = 0;
  size_t max_lds = 0;
};

DevInfo device_info() {
  static std::mutex mu;
  static std::map<int, DevInfo> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  DevInfo d;
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) d.cus = v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
          hipSuccess && v > 0)
    d.max_lds = (size_t)v;
  else
    d.max_lds = 160 * 1024;
  if (d.cus <= 0) d.cus = 256;
  cache[dev] = d;
  return d;
}

// ---------------------------------------------------------------- tuning --

struct TuneKey {
  int dt, dim, nqb;
  bool operator<(const TuneKey& o) const {
    return std::tie(dt, dim, nqb) < std::tie(o.dt, o.dim, o.nqb);
  }
};
struct FusedCfg {
  int pf = 4;
  int nw = 4;
  int wg_per_cu = 0;  // 0: as many as fit
  int stage = 0;      // 1: document tiles staged through LDS
  int rows = 16;      // document rows per step (32: FP8, staged, Q in VGPRs)
};

std::mutex g_tune_mu;
std::map<TuneKey, FusedCfg> g_tuned;

// PQ scorer choice: the table kernel (variant 0) or decode-into-MFMA
// (variant 1, with nqb query blocks per wave; 0 = automatic).
struct PqKey {
  int M, dsub, bpq, cand;
  bool operator<(const PqKey& o) const {
    return std::tie(M, dsub, bpq, cand) < std::tie(o.M, o.dsub, o.bpq, o.cand);
  }
};
struct PqCfg {
  int variant = -1;  // -1: automatic
  int nqb = 0;
};
std::map<PqKey, PqCfg> g_pq_tuned;

// Residual scorer: load-pipeline variant per (nbits, dim, query blocks,
// candidates or not).
struct ResKey {
  int nbits, dim, nqb, cand;
  bool operator<(const ResKey& o) const {
    return std::tie(nbits, dim, nqb, cand) < std::tie(o.nbits, o.dim, o.nqb, o.cand);
  }
};
struct ResCfg {
  int pipe = -1;  // -1: automatic
};
std::map<ResKey, ResCfg> g_res_tuned;

// Untuned keys: document tiles staged through LDS (the faster form measured on
// MI355X for every element type but FP32) when the ring fits beside the query
// block, else register-direct.
FusedCfg default_cfg(int dt, size_t q_lds, int dch) {
  FusedCfg c;
  c.nw = 4;
  c.wg_per_cu = 0;
  if (dt == MAXSIM_F32) {
    c.pf = 2;
    c.stage = 0;
    return c;
  }
  c.pf = 3;
  c.stage = 1;
  if (q_lds + (size_t)c.nw * c.pf * 16 * dch * esize(dt) > device_info().max_lds) {
    c.pf = 4;
    c.stage = 0;
  }
  return c;
}

FusedCfg lookup_cfg(const TuneKey& k, size_t q_lds, int dch) {
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(k);
    if (it != g_tuned.end()) return it->second;
  }
  return default_cfg(k.dt, q_lds, dch);
}

// ------------------------------------------------------------ fused plan --

struct FusedPlan {
  FusedParams P{};
  int dt = 0, nqb = 1, dch = 128;
  bool qreg = false;
  size_t lds = 0;
  int64_t n_pairs = 0;
};

maxsim_status plan_fused(const maxsim_csr* q, const maxsim_csr* d, const maxsim_candidates* cand,
                         float* scores, FusedPlan& pl, bool group_queries = true,
                         bool need_scores = true) {
  maxsim_status st = check_csr(q, "queries", true);
  if (st) return st;
  if ((st = check_csr(d, "docs", false))) return st;
  if (q->dtype != d->dtype) return fail(MAXSIM_EINVAL, "queries and docs differ in dtype");
  if (q->dim != d->dim) return fail(MAXSIM_EINVAL, "queries and docs differ in dim");
  if (d->n_sets > 0x7fffffffLL) return fail(MAXSIM_EUNSUPPORTED, "more than 2^31-1 documents");
  int64_t n_pairs;
  if (cand) {
    if (cand->n_total < 0) return fail(MAXSIM_EINVAL, "candidates: negative n_total");
    if (!cand->offsets) return fail(MAXSIM_EINVAL, "candidates: offsets is NULL");
    if (cand->n_total > 0 && !cand->doc_ids) return fail(MAXSIM_EINVAL, "candidates: doc_ids is NULL");
    n_pairs = cand->n_total;
  } else {
    n_pairs = q->n_sets * d->n_sets;
  }
  if (n_pairs > 0 && !scores && need_scores) return fail(MAXSIM_EINVAL, "scores is NULL");
  pl.dt = q->dtype;
  // d-chunk width: 128 (the paper's dimension tiling), 64 when d > 128 is not
  // a multiple of 128, and 256 for 1- and 2-byte rows of d >= 256 (same k
  // order, so the same bits; each row read becomes 512 contiguous bytes). A d
  // that is not a multiple of the chunk is zero-extended to whole chunks
  // inside the kernel: the query operand's columns past d are zero and the
  // document columns past d are read from inside the row, so they add exact
  // zeros. d <= 128 takes one chunk (64 wide up to 64, else 128).
  if (q->dim <= 128)
    pl.dch = q->dim <= 64 ? 64 : 128;
  else
    pl.dch = (q->dim % 128 == 0) ? 128 : 64;
  if (esize(q->dtype) <= 2 && q->dim >= 256 && q->dim % 256 == 0) pl.dch = 256;
  const int nch = (q->dim + pl.dch - 1) / pl.dch;
  // the query operand sits in VGPRs when d fits one chunk of at most 128
  // (a 256-wide chunk's query blocks live in LDS)
  pl.qreg = nch == 1 && pl.dch <= 128;
  // Query units: without candidate lists, queries are grouped so one read of
  // a document tile serves several of them (up to 8 blocks of 16 query tokens
  // in VGPRs for 1- and 2-byte types, 4 otherwise).
  const int bpq = nqb_for(q->max_len);
  const int row_bytes = q->dim * esize(q->dtype);
  // the query operand's row in LDS spans whole chunks
  const int qrow_bytes = nch * pl.dch * esize(q->dtype);
  int group = 1;
  if (!cand && group_queries) {
    // in LDS (d beyond one chunk) the grouped query blocks leave at least
    // half of it to the staging ring
    const int cap = (pl.qreg && esize(q->dtype) <= 2) ? 8 : 4;
    auto fits = [&](int gr) {
      return pl.qreg || (size_t)gr * bpq * 16 * qrow_bytes <= device_info().max_lds / 2;
    };
    while (group * 2 * bpq <= cap && group * 2 <= q->n_sets && fits(group * 2)) group *= 2;
  }
  pl.nqb = group * bpq;
  pl.lds = (size_t)pl.nqb * 16 * qrow_bytes;
  if (pl.lds > device_info().max_lds)
    return fail(MAXSIM_EUNSUPPORTED, "query block of %zu bytes exceeds LDS", pl.lds);
  FusedParams& P = pl.P;
  P.q_tok = (const char*)q->tokens;
  P.q_off = q->offsets;
  P.q_scales = q->scales;
  P.n_q = q->n_sets;
  P.d_tok = (const char*)d->tokens;
  P.d_off = d->offsets;
  P.d_scales = d->scales;
  P.n_docs = d->n_sets;
  P.cand_off = cand ? cand->offsets : nullptr;
  P.cand_ids = cand ? cand->doc_ids : nullptr;
  P.scores = scores;
  P.n_pairs = n_pairs;
  P.tokens_per_query = d->n_tokens;
  P.dim = q->dim;
  P.nch = nch;
  P.row_bytes = row_bytes;
  P.ncg = qrow_bytes / 64;
  P.group = group;
  P.bpq = bpq;
  P.n_units = (q->n_sets + group - 1) / group;
  P.n_upairs = cand ? n_pairs : P.n_units * d->n_sets;
  pl.n_pairs = n_pairs;
  return MAXSIM_OK;
}

// A fused launch ready to go: kernel, parameters, dynamic LDS and grid.
struct FusedLaunch {
  FusedFns fns{};
  FusedParams P{};
  size_t lds = 0;
  int64_t grid = 0;
};

int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Kernel choice, LDS layout and grid of a fused launch (topk_k > 0: with the
// top-k epilogue, whose key slots take the LDS the tuned occupancy leaves).
maxsim_status prepare_fused(const FusedPlan& pl, const FusedCfg& cfg, int topk_k, FusedLaunch& L) {
  DevInfo di = device_info();
  // 256-wide chunks exist only with LDS-staged tiles, and only where their
  // ring fits beside one copy of the query blocks; else 128-wide
  FusedParams P = pl.P;
  int dch = pl.dch;
  if (dch == 256 && (!cfg.stage || pl.lds + (size_t)cfg.nw * cfg.pf * 16 * 256 * esize(pl.dt) >
                                       di.max_lds)) {
    dch = 128;  // d is a multiple of 256 here: the same padded row
    P.nch = P.dim / dch;
  }
  // 32-row steps only where they exist (FP8, staged, one chunk)
  const int rt = (cfg.rows == 32 && cfg.stage && pl.qreg && pl.dt == MAXSIM_F8E4M3) ? 32 : 16;
  // query operand: VGPRs when d fits one chunk, else one LDS copy per wave
  // when that fits beside the staging ring, else one per workgroup
  const size_t ring = cfg.stage ? (size_t)cfg.nw * cfg.pf * rt * dch * esize(pl.dt) : 0;
  int qm;
  size_t lds;
  if (pl.qreg) {
    qm = 1;
    lds = ring;
  } else if ((size_t)cfg.nw * pl.lds + ring <= di.max_lds) {
    qm = 2;
    lds = (size_t)cfg.nw * pl.lds + ring;
  } else {
    qm = 0;
    lds = pl.lds + ring;
  }
  if (lds > di.max_lds) return fail(MAXSIM_EUNSUPPORTED, "staged tiles need %zu bytes of LDS", lds);
  FusedFns fns = fused_kernel_fns(pl.dt, pl.nqb, dch, cfg.pf, cfg.nw, qm, cfg.stage != 0, rt);
  if (!fns.launch) return fail(MAXSIM_EUNSUPPORTED, "no fused kernel for %d query blocks here", pl.nqb);
  int occ = fns.occupancy(lds);
  if (occ <= 0) return fail(MAXSIM_EHIP, "fused kernel does not fit on a compute unit");
  int per_cu = cfg.wg_per_cu > 0 ? std::min(cfg.wg_per_cu, occ) : occ;
  P.topk_k = 0;
  P.key_cap = 0;
  P.lds_keys_off = 0;
  P.sel_cap = 0;
  if (topk_k > 0) {
    // selection scratch (reusing the query/ring area), then the key slots and
    // the wave ranges; the slots get what the tuned occupancy leaves of LDS
    P.topk_k = topk_k;
    P.sel_cap = std::min(2048, std::max(256, pow2_at_least(2 * topk_k)));
    const size_t head = (std::max(lds, fused_topk_scratch_bytes(P.sel_cap)) + 15) & ~(size_t)15;
    const size_t ranges = (size_t)cfg.nw * 16;
    const size_t share = di.max_lds / (size_t)per_cu;
    int64_t slots = share > head + ranges ? (int64_t)((share - head - ranges) / 4) : 0;
    slots = std::min<int64_t>(slots, 65536);
    slots -= slots % cfg.nw;
    P.key_cap = (int32_t)slots;
    P.lds_keys_off = (int32_t)head;
    lds = head + (size_t)slots * 4 + ranges;
    if (lds > di.max_lds) return fail(MAXSIM_EUNSUPPORTED, "top-k epilogue needs %zu bytes of LDS", lds);
    occ = fns.occupancy(lds);
    if (occ <= 0) return fail(MAXSIM_EHIP, "fused top-k kernel does not fit on a compute unit");
    per_cu = std::min(per_cu, occ);
  }
  int64_t grid = (int64_t)per_cu * di.cus;
  int64_t need = (pl.P.n_upairs + cfg.nw - 1) / cfg.nw;  // at least one work pair per wave
  if (grid > need) grid = need;
  if (grid < 1) grid = 1;
  if (topk_k > 0 && grid > MERGE_MAX_GRID) grid = MERGE_MAX_GRID;
  L.fns = fns;
  L.P = P;
  L.lds = lds;
  L.grid = grid;
  return MAXSIM_OK;
}

maxsim_status run_fused(const FusedPlan& pl, const FusedCfg& cfg, hipStream_t s) {
  if (pl.n_pairs == 0) return MAXSIM_OK;
  FusedLaunch L;
  maxsim_status st = prepare_fused(pl, cfg, 0, L);
  if (st) return st;
  hipError_t e = L.fns.launch(L.P, (int)L.grid, L.lds, s);
  if (e != hipSuccess) return hip_fail(e, "fused MaxSim launch");
  return MAXSIM_OK;
}

// Workspace of the fused top-k: workgroup starts, part counts, part keys and
// the key spill array, each 256-byte aligned.
struct TopkLayout {
  size_t wg_lo = 0, cnt = 0, keys = 0, spill = 0, total = 0;
};

bool topk_layout(const FusedLaunch& L, int k, TopkLayout& T) {
  const FusedParams& P = L.P;
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t n_slots = (size_t)(L.grid + P.n_units) * (size_t)P.group;
  size_t keys_b = 0, spill_b = 0;
  if (__builtin_mul_overflow(n_slots, (size_t)k * 8, &keys_b)) return false;
  if (__builtin_mul_overflow((size_t)P.n_upairs, (size_t)P.group * 4, &spill_b)) return false;
  T.wg_lo = 0;
  T.cnt = up((size_t)L.grid * 8);
  T.keys = T.cnt + up(n_slots * 4);
  T.spill = T.keys + up(keys_b);
  if (__builtin_add_overflow(T.spill, up(spill_b), &T.total)) return false;
  return true;
}

// ------------------------------------------------------------- JSON cache --

std::string cfg_json_all() {
  std::string out = "{\"version\":1,\"entries\":[";
  bool first = true;
  for (auto& kv : g_tuned) {
    char b[192];
    snprintf(b, sizeof b,
             "%s{\"dtype\":%d,\"dim\":%d,\"nqb\":%d,\"pf\":%d,\"nw\":%d,\"wg_per_cu\":%d,"
             "\"stage\":%d,\"rows\":%d}",
             first ? "" : ",", kv.first.dt, kv.first.dim, kv.first.nqb, kv.second.pf, kv.second.nw,
             kv.second.wg_per_cu, kv.second.stage, kv.second.rows);
    out += b;
    first = false;
  }
  for (auto& kv : g_res_tuned) {
    char b[160];
    snprintf(b, sizeof b, "%s{\"residual\":1,\"nbits\":%d,\"dim\":%d,\"nqb\":%d,\"cand\":%d,"
             "\"pipe\":%d}",
             first ? "" : ",", kv.first.nbits, kv.first.dim, kv.first.nqb, kv.first.cand,
             kv.second.pipe);
    out += b;
    first = false;
  }
  for (auto& kv : g_pq_tuned) {
    char b[192];
    snprintf(b, sizeof b,
             "%s{\"pq\":1,\"M\":%d,\"dsub\":%d,\"bpq\":%d,\"cand\":%d,\"variant\":%d,"
             "\"nqb\":%d}",
             first ? "" : ",", kv.first.M, kv.first.dsub, kv.first.bpq, kv.first.cand,
             kv.second.variant, kv.second.nqb);
    out += b;
    first = false;
  }
  out += "]}";
  return out;
}

bool json_int(const char* obj, const char* key, int& v) {
  char pat[32];
  snprintf(pat, sizeof pat, "\"%s\":", key);
  const char* p = strstr(obj, pat);
  if (!p) return false;
  v = atoi(p + strlen(pat));
  return true;
}

}  // namespace

// =================================================================== ABI ==
// Every exported function is declared in maxsim.h inside extern "C", so its
// definition below has C linkage; the helpers in the anonymous namespaces
// between them are internal C++.

int maxsim_abi_version(void) { return MAXSIM_ABI_VERSION; }

const char* maxsim_last_error(void) { return g_err.c_str(); }

maxsim_status maxsim_quantize(const float* src, int64_t n_tokens, int32_t dim, int32_t dtype,
                              void* dst, float* scales, maxsim_stream_t stream) {
  if (n_tokens < 0) return fail(MAXSIM_EINVAL, "quantize: negative n_tokens");
  if (dim < 16 || dim > 1024 || dim % 16 != 0)
    return fail(MAXSIM_EUNSUPPORTED, "quantize: dim %d must be a multiple of 16 in [16, 1024]", dim);
  if (dtype < MAXSIM_F32 || dtype > MAXSIM_F8E4M3)
    return fail(MAXSIM_EINVAL, "quantize: unknown dtype %d", dtype);
  if (n_tokens == 0) return MAXSIM_OK;
  if (!src || !dst) return fail(MAXSIM_EINVAL, "quantize: NULL src or dst");
  if (!aligned(src, 16) || !aligned(dst, 16))
    return fail(MAXSIM_EINVAL, "quantize: src and dst must be 16-byte aligned");
  if (dtype == MAXSIM_F8E4M3 && !scales) return fail(MAXSIM_EINVAL, "quantize: FP8 needs scales");
  if (dtype != MAXSIM_F8E4M3 && scales)
    return fail(MAXSIM_EINVAL, "quantize: scales only apply to FP8");
  hipError_t e = launch_quantize(src, n_tokens, dim, dtype, dst, scales, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "quantize launch");
  return MAXSIM_OK;
}

size_t maxsim_score_workspace_size(const maxsim_csr*, const maxsim_csr*, const maxsim_candidates*) {
  return 0;  // the fused scorer keeps everything on chip
}

maxsim_status maxsim_score(const maxsim_csr* queries, const maxsim_csr* docs,
                           const maxsim_candidates* cand, float* scores, void* workspace,
                           size_t ws_bytes, maxsim_stream_t stream) {
  (void)workspace;
  (void)ws_bytes;
  FusedPlan pl;
  maxsim_status st = plan_fused(queries, docs, cand, scores, pl);
  if (st) return st;
  FusedCfg cfg = lookup_cfg({pl.dt, queries->dim, pl.nqb}, pl.qreg ? 0 : pl.lds, pl.dch);
  return run_fused(pl, cfg, (hipStream_t)stream);
}

namespace {

// Plan of a fused score + top-k call: the scoring launch (when there are work
// pairs) and its workspace layout.
maxsim_status plan_score_topk(const maxsim_csr* q, const maxsim_csr* d,
                              const maxsim_candidates* cand, int32_t k, FusedPlan& pl,
                              FusedLaunch& L, TopkLayout& T, bool* overflow = nullptr) {
  if (k < 1 || k > 1024) return fail(MAXSIM_EINVAL, "score_topk: k=%d must be in [1, 1024]", k);
  maxsim_status st = plan_fused(q, d, cand, nullptr, pl, true, /*need_scores=*/false);
  if (st) return st;
  if (pl.n_pairs > 0) {
    FusedCfg cfg = lookup_cfg({pl.dt, q->dim, pl.nqb}, pl.qreg ? 0 : pl.lds, pl.dch);
    if ((st = prepare_fused(pl, cfg, k, L))) return st;
  } else {
    L.P = pl.P;
    L.grid = 0;
  }
  if (!topk_layout(L, k, T)) {
    if (overflow) *overflow = true;
    return fail(MAXSIM_EUNSUPPORTED, "score_topk: workspace exceeds the address space");
  }
  return MAXSIM_OK;
}

}  // namespace

size_t maxsim_score_topk_workspace_size(const maxsim_csr* q, const maxsim_csr* d,
                                        const maxsim_candidates* cand, int32_t k) {
  FusedPlan pl;
  FusedLaunch L;
  TopkLayout T;
  bool overflow = false;
  const std::string saved = g_err;
  maxsim_status st = plan_score_topk(q, d, cand, k, pl, L, T, &overflow);
  g_err = saved;
  if (overflow) return SIZE_MAX;
  return st ? 0 : T.total;
}

namespace {

// Enqueues a planned fused score + top-k (both launches) with the workspace
// at ws (at least T.total bytes, 16-byte aligned).
maxsim_status launch_score_topk(const FusedPlan& pl, FusedLaunch& L, const TopkLayout& T,
                                int64_t n_q, int32_t k, float* out_scores, int32_t* out_ids,
                                char* ws, hipStream_t s) {
  if (L.grid > 0) {
    FusedParams& P = L.P;
    P.scores = nullptr;
    P.wg_lo = (int64_t*)(ws + T.wg_lo);
    P.part_cnt = (uint32_t*)(ws + T.cnt);
    P.part_keys = (uint64_t*)(ws + T.keys);
    P.key_spill = (uint32_t*)(ws + T.spill);
    hipError_t e = L.fns.launch(P, (int)L.grid, L.lds, s);
    if (e != hipSuccess) return hip_fail(e, "fused score_topk launch");
  }
  MergeParams M{};
  M.cand_off = pl.P.cand_off;
  M.n_q = n_q;
  M.n_docs = pl.P.n_docs;
  M.n_upairs = pl.P.n_upairs;
  M.group = pl.P.group;
  M.grid = (int32_t)L.grid;
  M.k = k;
  M.wg_lo = (const int64_t*)(ws + T.wg_lo);
  M.part_keys = (const uint64_t*)(ws + T.keys);
  M.part_cnt = (const uint32_t*)(ws + T.cnt);
  M.out_scores = out_scores;
  M.out_ids = out_ids;
  hipError_t e = launch_topk_merge(M, s);
  if (e != hipSuccess) return hip_fail(e, "top-k merge launch");
  return MAXSIM_OK;
}

}  // namespace

maxsim_status maxsim_score_topk(const maxsim_csr* queries, const maxsim_csr* docs,
                                const maxsim_candidates* cand, int32_t k, float* out_scores,
                                int32_t* out_ids, void* workspace, size_t ws_bytes,
                                maxsim_stream_t stream) {
  FusedPlan pl;
  FusedLaunch L;
  TopkLayout T;
  maxsim_status st = plan_score_topk(queries, docs, cand, k, pl, L, T);
  if (st) return st;
  if (queries->n_sets == 0) return MAXSIM_OK;
  if (!out_scores || !out_ids) return fail(MAXSIM_EINVAL, "score_topk: NULL output");
  if (!workspace || ws_bytes < T.total)
    return fail(MAXSIM_EWORKSPACE, "score_topk: workspace needs %zu bytes", T.total);
  if (!aligned(workspace, 16))
    return fail(MAXSIM_EINVAL, "score_topk: workspace must be 16-byte aligned");
  return launch_score_topk(pl, L, T, queries->n_sets, k, out_scores, out_ids, (char*)workspace,
                           (hipStream_t)stream);
}

// ------------------------------------------------- allocation-free top-k --
// The workspace of maxsim_score_topk_noalloc: a file-scope device array, one
// copy on every GPU the library runs on, held until the process ends. In host
// code `scratch` names the symbol only, not device memory: its address on a
// device comes from hipGetSymbolAddress with that device current, looked up
// once per device and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[MAXSIM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// The current device's copy of `scratch` (no allocation: the array is part of
// the library's code object on that device).
maxsim_status scratch_on_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "score_topk_noalloc: hipGetDevice");
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
    return fail(MAXSIM_EUNSUPPORTED, "score_topk_noalloc: device %d beyond the first %d", dev,
                SCRATCH_MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "score_topk_noalloc: scratch address lookup");
    if (!p) return fail(MAXSIM_EHIP, "score_topk_noalloc: scratch address lookup gave NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MAXSIM_OK;
}

}  // namespace

maxsim_status maxsim_score_topk_noalloc(const maxsim_csr* queries, const maxsim_csr* docs,
                                        const maxsim_candidates* cand, int32_t k,
                                        float* out_scores, int32_t* out_ids,
                                        maxsim_stream_t stream) {
  FusedPlan pl;
  FusedLaunch L;
  TopkLayout T;
  maxsim_status st = plan_score_topk(queries, docs, cand, k, pl, L, T);
  if (st) return st;
  if (queries->n_sets == 0) return MAXSIM_OK;
  if (!out_scores || !out_ids) return fail(MAXSIM_EINVAL, "score_topk_noalloc: NULL output");
  if (T.total > (size_t)MAXSIM_NOALLOC_SCRATCH_BYTES)
    return fail(MAXSIM_EWORKSPACE,
                "score_topk_noalloc: this problem needs %zu bytes of workspace, above the fixed "
                "%zu-byte scratch (use maxsim_score_topk with a caller workspace)",
                T.total, (size_t)MAXSIM_NOALLOC_SCRATCH_BYTES);
  void* p = nullptr;
  if ((st = scratch_on_current_device(&p))) return st;
  return launch_score_topk(pl, L, T, queries->n_sets, k, out_scores, out_ids, (char*)p,
                           (hipStream_t)stream);
}

size_t maxsim_score_unfused_workspace_size(const maxsim_csr* q, const maxsim_csr* d) {
  if (!q || !d || q->n_sets < 0 || d->n_tokens < 0) return 0;
  // S holds n_q x n_tokens rows of the query-capacity columns, FP32
  const size_t cols = (size_t)nqb_for(q->max_len) * 16 * 4;
  size_t n = 0;
  if (__builtin_mul_overflow((size_t)q->n_sets, (size_t)d->n_tokens, &n) ||
      __builtin_mul_overflow(n, cols, &n))
    return SIZE_MAX;
  return n;
}

maxsim_status maxsim_score_unfused(const maxsim_csr* queries, const maxsim_csr* docs,
                                   float* scores, void* workspace, size_t ws_bytes,
                                   maxsim_stream_t stream) {
  FusedPlan pl;
  maxsim_status st = plan_fused(queries, docs, nullptr, scores, pl, /*group_queries=*/false);
  if (st) return st;
  if (pl.dch == 256) {  // the comparator's tiles are 128 wide at most (d % 256 == 0 here)
    pl.dch = 128;
    pl.P.nch = queries->dim / 128;
  }
  size_t need = maxsim_score_unfused_workspace_size(queries, docs);
  if (need == SIZE_MAX) return fail(MAXSIM_EUNSUPPORTED, "unfused: S exceeds the address space");
  if (need > 0 && (!workspace || ws_bytes < need))
    return fail(MAXSIM_EWORKSPACE, "unfused: workspace needs %zu bytes", need);
  if (pl.n_pairs == 0) return MAXSIM_OK;
  if (queries->n_sets > 65535) return fail(MAXSIM_EUNSUPPORTED, "unfused: at most 65535 queries");
  DevInfo di = device_info();
  // the launcher sizes the grid from the CU count and the kernel's occupancy
  hipError_t e = launch_unfused(pl.dt, pl.nqb, pl.dch, pl.P, (float*)workspace, di.cus, pl.lds,
                                (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "unfused launch");
  return MAXSIM_OK;
}

// ------------------------------------------------------------------ PQ --

namespace {
struct PqPlan {
  PqParams P{};
  size_t lds = 0;
  size_t ws = 0;
  int variant = 0;
};


PqKey pq_key(const maxsim_csr* q, const maxsim_pq_docs* d, const maxsim_candidates* cand) {
  return {d->M, d->dsub, pow2_at_least(std::max(1, (q->max_len + 15) / 16)), cand ? 1 : 0};
}

PqCfg lookup_pq(const PqKey& k) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_pq_tuned.find(k);
  return it == g_pq_tuned.end() ? PqCfg{} : it->second;
}

// Decode-into-MFMA plan; returns false when the problem is outside what that
// kernel handles (the table kernel is used then).
bool plan_pq_mfma(const maxsim_csr* q, const maxsim_pq_docs* d, const maxsim_candidates* cand,
                  int want_nqb, PqPlan& pl) {
  if (q->dtype != MAXSIM_F16 || d->cb_dtype != MAXSIM_F16) return false;
  if (d->dsub != 8 && d->dsub != 16 && d->dsub != 32) return false;
  const size_t lds = (size_t)d->M * d->K * d->dsub * 2;
  if (lds > device_info().max_lds) return false;
  if (!aligned(d->codebooks, 16) || (q->n_tokens > 0 && !aligned(q->tokens, 16))) return false;
  const int dim = d->M * d->dsub;
  const int bpq = pow2_at_least(std::max(1, (q->max_len + 15) / 16));
  if (bpq * dim > 1024) return false;  // query operand registers
  int nqb = bpq;
  if (!cand) {
    const int cap = want_nqb > 0 ? want_nqb : 8;
    nqb = 8;
    while (nqb > bpq && (nqb > cap || nqb * dim > 1024)) nqb >>= 1;
  } else if (want_nqb > 0 && want_nqb != bpq) {
    return false;  // one query per group with candidate lists
  }
  PqParams& P = pl.P;
  P.bpq = bpq;
  P.nqb = nqb;
  P.group = nqb / bpq;
  P.nw = 8;
  const int64_t n_groups = (q->n_sets + P.group - 1) / P.group;
  const int64_t per_group_docs =
      cand ? (q->n_sets > 0 ? cand->n_total / q->n_sets : 0) : d->n_docs;
  // about eight resident workgroups per CU over the whole launch, chunks of
  // at least 64 documents
  const int64_t want = (int64_t)device_info().cus * 8;
  int64_t n_chunks = std::max<int64_t>(1, (want + n_groups - 1) / std::max<int64_t>(1, n_groups));
  n_chunks = std::min<int64_t>(n_chunks, std::max<int64_t>(1, per_group_docs / 64));
  if (n_chunks * std::max<int64_t>(1, n_groups) > 0x7fffffffLL) return false;
  P.n_chunks = (int)n_chunks;
  pl.lds = lds;
  pl.ws = 0;
  pl.variant = 1;
  return true;
}

maxsim_status plan_pq(const maxsim_csr* q, const maxsim_pq_docs* d, const maxsim_candidates* cand,
                      float* scores, PqPlan& pl, const PqCfg* force = nullptr) {
  if (!q || !d) return fail(MAXSIM_EINVAL, "pq: NULL descriptor");
  if (q->dtype != MAXSIM_F16 && q->dtype != MAXSIM_F32)
    return fail(MAXSIM_EUNSUPPORTED, "pq: queries must be F16 or F32");
  if (q->n_sets < 0 || q->max_len < 0) return fail(MAXSIM_EINVAL, "pq: negative query sizes");
  if (q->max_len > 64) return fail(MAXSIM_EUNSUPPORTED, "pq: max_len exceeds 64 query tokens");
  if (!q->offsets || (q->n_tokens > 0 && !q->tokens)) return fail(MAXSIM_EINVAL, "pq: NULL query arrays");
  if (d->M != 4 && d->M != 8 && d->M != 16) return fail(MAXSIM_EUNSUPPORTED, "pq: M must be 4, 8 or 16");
  if (d->K < 1 || d->K > 256) return fail(MAXSIM_EUNSUPPORTED, "pq: K must be in [1, 256]");
  if (d->dsub < 1 || d->dsub > 32 || d->M * d->dsub > 1024)
    return fail(MAXSIM_EUNSUPPORTED, "pq: dsub must be in [1, 32]");
  if (q->dim != d->M * d->dsub) return fail(MAXSIM_EINVAL, "pq: query dim != M * dsub");
  if (d->cb_dtype != MAXSIM_F16 && d->cb_dtype != MAXSIM_F32)
    return fail(MAXSIM_EUNSUPPORTED, "pq: codebooks must be F16 or F32");
  if (!d->codebooks || !d->offsets || (d->n_tokens > 0 && !d->codes))
    return fail(MAXSIM_EINVAL, "pq: NULL document arrays");
  if (d->codes && !aligned(d->codes, d->M)) return fail(MAXSIM_EINVAL, "pq: codes must be M-byte aligned");
  if (d->n_docs < 0 || d->n_tokens < 0) return fail(MAXSIM_EINVAL, "pq: negative document sizes");
  int64_t n_pairs;
  if (cand) {
    if (!cand->offsets || cand->n_total < 0 || (cand->n_total > 0 && !cand->doc_ids))
      return fail(MAXSIM_EINVAL, "pq: bad candidates");
    n_pairs = cand->n_total;
  } else {
    n_pairs = q->n_sets * d->n_docs;
  }
  if (n_pairs > 0 && !scores) return fail(MAXSIM_EINVAL, "pq: scores is NULL");
  const size_t lut_row = (size_t)d->M * d->K * 4;  // bytes per query token of table
  const size_t budget = device_info().max_lds - 4096;
  int qt = 64;
  while (qt > 8 && ((size_t)qt * lut_row + (size_t)qt * q->dim * 4 > budget || qt / 2 >= q->max_len))
    qt /= 2;
  if ((size_t)qt * lut_row + (size_t)qt * q->dim * 4 > device_info().max_lds)
    return fail(MAXSIM_EUNSUPPORTED, "pq: table for M=%d K=%d does not fit LDS", d->M, d->K);
  int n_slices = std::max(1, (q->max_len + qt - 1) / qt);
  PqParams& P = pl.P;
  P.q_tok = (const char*)q->tokens;
  P.q_off = q->offsets;
  P.n_q = q->n_sets;
  P.q_f32 = q->dtype == MAXSIM_F32;
  P.cb_f32 = d->cb_dtype == MAXSIM_F32;
  P.codebooks = d->codebooks;
  P.codes = d->codes;
  P.d_off = d->offsets;
  P.n_docs = d->n_docs;
  P.cand_off = cand ? cand->offsets : nullptr;
  P.cand_ids = cand ? cand->doc_ids : nullptr;
  P.scores = scores;
  P.n_pairs = n_pairs;
  P.tokens_per_query = d->n_tokens;
  P.M = d->M;
  P.K = d->K;
  P.dsub = d->dsub;
  P.dim = q->dim;
  P.qt = qt;
  P.n_slices = n_slices;
  {
    const PqCfg cfg = force ? *force : lookup_pq(pq_key(q, d, cand));
    if (cfg.variant != 0 && plan_pq_mfma(q, d, cand, cfg.nqb, pl)) return MAXSIM_OK;
    if (force && force->variant == 1)
      return fail(MAXSIM_EUNSUPPORTED, "pq: decode-into-MFMA variant does not apply");
  }
  // enough items to balance ~4 waves of workgroups over the CUs, but chunks
  // of at least ~512 pairs so the table build stays amortised
  int64_t base_items = std::max<int64_t>(1, q->n_sets * n_slices);
  int64_t want = (int64_t)device_info().cus * 4;
  int64_t per_query_pairs = q->n_sets > 0 ? n_pairs / q->n_sets : 0;
  int64_t n_chunks = std::max<int64_t>(1, (want + base_items - 1) / base_items);
  n_chunks = std::min<int64_t>(n_chunks, std::max<int64_t>(1, per_query_pairs / 512));
  if ((int64_t)n_chunks * base_items > 0x7fffffffLL)
    return fail(MAXSIM_EUNSUPPORTED, "pq: too many work items");
  P.n_chunks = (int)n_chunks;
  // The table fills most of the LDS, so one workgroup runs per CU: 16 waves
  // keep the LDS and VALU pipes busy (8 waves measured 1.7x slower).
  P.nw = 16;
  pl.lds = ((size_t)d->M * d->K * qt + (size_t)qt * q->dim) * 4;
  // per-slice partial scores; a size past the address space is refused, not
  // wrapped
  if (n_slices > 1 && (size_t)n_pairs > SIZE_MAX / 4 / (size_t)n_slices)
    return fail(MAXSIM_EUNSUPPORTED, "pq: partial scores exceed the address space");
  pl.ws = n_slices > 1 ? (size_t)n_slices * (size_t)n_pairs * 4 : 0;
  pl.variant = 0;
  return MAXSIM_OK;
}

hipError_t run_pq(const PqPlan& pl, int max_len, hipStream_t s) {
  return pl.variant == 1 ? launch_pq_mfma(pl.P, pl.lds, s) : launch_pq(pl.P, max_len, s);
}
}  // namespace

size_t maxsim_pq_score_workspace_size(const maxsim_csr* queries, const maxsim_pq_docs* docs,
                                      const maxsim_candidates* cand) {
  PqPlan pl;
  std::string saved = g_err;
  if (plan_pq(queries, docs, cand, (float*)1, pl)) {
    g_err = saved;
    return 0;
  }
  return pl.ws;
}

maxsim_status maxsim_pq_score(const maxsim_csr* queries, const maxsim_pq_docs* docs,
                              const maxsim_candidates* cand, float* scores, void* workspace,
                              size_t ws_bytes, maxsim_stream_t stream) {
  PqPlan pl;
  maxsim_status st = plan_pq(queries, docs, cand, scores, pl);
  if (st) return st;
  if (pl.ws > 0 && (!workspace || ws_bytes < pl.ws))
    return fail(MAXSIM_EWORKSPACE, "pq: workspace needs %zu bytes", pl.ws);
  if (pl.P.n_pairs == 0) return MAXSIM_OK;
  pl.P.partial = (float*)workspace;
  hipError_t e = run_pq(pl, queries->max_len, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "pq launch");
  return MAXSIM_OK;
}

maxsim_status maxsim_pq_autotune(const maxsim_csr* queries, const maxsim_pq_docs* docs,
                                 const maxsim_candidates* cand, float* scores, void* workspace,
                                 size_t ws_bytes, maxsim_stream_t stream, int32_t reps,
                                 const char* cache_path, char* report, size_t report_len) {
  PqPlan probe;
  maxsim_status st = plan_pq(queries, docs, cand, scores, probe);
  if (st) return st;
  if (reps < 1) reps = 1;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(MAXSIM_EHIP, "pq autotune: event creation failed");
  std::vector<PqCfg> space;
  space.push_back({0, 0});
  for (int nqb : {1, 2, 4, 8}) space.push_back({1, nqb});
  const PqKey key = pq_key(queries, docs, cand);
  std::string rep = "{\"pq\":1,\"M\":" + std::to_string(key.M) + ",\"dsub\":" +
                    std::to_string(key.dsub) + ",\"bpq\":" + std::to_string(key.bpq) +
                    ",\"cand\":" + std::to_string(key.cand) + ",\"trials\":[";
  float best_ms = 1e30f;
  PqCfg best{0, 0};
  bool first = true;
  for (const PqCfg& c : space) {
    PqPlan pl;
    if (plan_pq(queries, docs, cand, scores, pl, &c)) continue;  // does not apply
    if (c.variant == 1 && pl.P.nqb != c.nqb) continue;          // same shape as another trial
    if (pl.ws > 0 && (!workspace || ws_bytes < pl.ws)) continue;
    pl.P.partial = (float*)workspace;
    if (pl.P.n_pairs == 0) break;
    if (run_pq(pl, queries->max_len, s) != hipSuccess) continue;
    (void)hipEventRecord(e0, s);
    bool ok = true;
    for (int r = 0; r < reps && ok; ++r) ok = run_pq(pl, queries->max_len, s) == hipSuccess;
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess || !ok) continue;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= reps;
    char b[128];
    snprintf(b, sizeof b, "%s{\"variant\":%d,\"nqb\":%d,\"ms\":%.5f}", first ? "" : ",",
             c.variant, c.variant ? pl.P.nqb : 0, ms);
    rep += b;
    first = false;
    if (ms < best_ms) {
      best_ms = ms;
      best = {c.variant, c.variant ? pl.P.nqb : 0};
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  char b[128];
  snprintf(b, sizeof b, "],\"best\":{\"variant\":%d,\"nqb\":%d,\"ms\":%.5f}}", best.variant,
           best.nqb, best_ms);
  rep += b;
  std::string all;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_pq_tuned[key] = best;
    all = cfg_json_all();
  }
  if (cache_path) {
    FILE* f = fopen(cache_path, "wb");
    if (!f) return fail(MAXSIM_EINVAL, "pq autotune: cannot write %s", cache_path);
    fputs(all.c_str(), f);
    fclose(f);
  }
  if (report && report_len > 0) {
    snprintf(report, report_len, "%s", rep.c_str());
  }
  return MAXSIM_OK;
}

// --------------------------------------------------------------- top-k --

// ------------------------------------------- residual-compressed docs --

namespace {

struct ResPlan {
  ResParams P;
  size_t ws = 0;
};

// Untuned keys: ids two tiles ahead of the table gathers, which run two tiles
// ahead of the compute.
constexpr int RES_DEFAULT_PIPE = 2;

maxsim_status plan_residual(const maxsim_csr* q, const maxsim_residual_docs* d,
                            const maxsim_candidates* cand, float* scores, ResPlan& pl,
                            int force_pipe = -1) {
  if (!q || !d) return fail(MAXSIM_EINVAL, "residual: NULL descriptor");
  if (q->dtype != MAXSIM_F16) return fail(MAXSIM_EUNSUPPORTED, "residual: queries must be F16");
  if (d->dim != 64 && d->dim != 128 && d->dim != 256)
    return fail(MAXSIM_EUNSUPPORTED, "residual: dim %d must be 64, 128 or 256", d->dim);
  if (q->dim != d->dim) return fail(MAXSIM_EINVAL, "residual: query dim != document dim");
  if (d->nbits != 1 && d->nbits != 2 && d->nbits != 4)
    return fail(MAXSIM_EUNSUPPORTED, "residual: nbits must be 1, 2 or 4");
  if (q->n_sets < 0 || q->n_tokens < 0 || q->max_len < 0)
    return fail(MAXSIM_EINVAL, "residual: negative query sizes");
  if (q->max_len > 64) return fail(MAXSIM_EUNSUPPORTED, "residual: max_len exceeds 64 query tokens");
  if (!q->offsets || (q->n_tokens > 0 && !q->tokens))
    return fail(MAXSIM_EINVAL, "residual: NULL query arrays");
  if (q->tokens && !aligned(q->tokens, 16))
    return fail(MAXSIM_EINVAL, "residual: query tokens must be 16-byte aligned");
  if (d->n_centroids < 1) return fail(MAXSIM_EINVAL, "residual: n_centroids must be >= 1");
  if (!d->centroids || !d->weights || !d->offsets ||
      (d->n_tokens > 0 && (!d->centroid_ids || !d->residuals)))
    return fail(MAXSIM_EINVAL, "residual: NULL document arrays");
  if (!aligned(d->centroids, 16) || !aligned(d->weights, 2) ||
      (d->residuals && !aligned(d->residuals, 16)) ||
      (d->centroid_ids && !aligned(d->centroid_ids, 4)) || !aligned(d->offsets, 8))
    return fail(MAXSIM_EINVAL,
                "residual: centroids and residuals must be 16-byte aligned (ids 4, offsets 8)");
  if (d->n_docs < 0 || d->n_tokens < 0)
    return fail(MAXSIM_EINVAL, "residual: negative document sizes");
  int64_t n_pairs;
  if (cand) {
    if (!cand->offsets || cand->n_total < 0 || (cand->n_total > 0 && !cand->doc_ids))
      return fail(MAXSIM_EINVAL, "residual: bad candidates");
    n_pairs = cand->n_total;
  } else {
    n_pairs = q->n_sets * d->n_docs;
  }
  if (n_pairs > 0 && !scores) return fail(MAXSIM_EINVAL, "residual: scores is NULL");
  ResParams& P = pl.P;
  P.q_tok = q->tokens;
  P.q_off = q->offsets;
  P.n_q = q->n_sets;
  P.n_qtok = q->n_tokens;
  P.centroids = d->centroids;
  P.n_centroids = d->n_centroids;
  P.weights = d->weights;
  P.ids = d->centroid_ids;
  P.residuals = d->residuals;
  P.d_off = d->offsets;
  P.n_docs = d->n_docs;
  P.cand_off = cand ? cand->offsets : nullptr;
  P.cand_ids = cand ? cand->doc_ids : nullptr;
  P.scores = scores;
  P.table = nullptr;
  P.dim = d->dim;
  P.nbits = d->nbits;
  P.nqb = pow2_at_least(std::max(1, (q->max_len + 15) / 16));
  // about eight resident workgroups per CU over the launch, chunks of at
  // least 64 documents
  const int64_t per_query = cand ? (q->n_sets > 0 ? cand->n_total / q->n_sets : 0) : d->n_docs;
  const int64_t want = (int64_t)device_info().cus * 8;
  const int64_t nq = std::max<int64_t>(1, q->n_sets);
  int64_t n_chunks = std::max<int64_t>(1, (want + nq - 1) / nq);
  n_chunks = std::min<int64_t>(n_chunks, std::max<int64_t>(1, per_query / 64));
  if (n_chunks * nq > 0x7fffffffLL) return fail(MAXSIM_EUNSUPPORTED, "residual: too many work items");
  // a work item's span of documents (or candidate positions) stays in 32 bits
  const int64_t span_bound = (cand ? cand->n_total : d->n_docs) / n_chunks + 1;
  if (span_bound >= 0x7fffffffLL - 64)
    return fail(MAXSIM_EUNSUPPORTED, "residual: too many documents per work item");
  P.n_chunks = (int)n_chunks;
  P.n_cols = q->n_sets * 16 * P.nqb;
  if (d->n_centroids >= (1 << 24) || P.n_cols >= (1 << 24) ||
      (uint64_t)d->n_centroids * (uint64_t)P.n_cols >= (1ull << 32))
    return fail(MAXSIM_EUNSUPPORTED,
                "residual: n_centroids and n_queries x 16 x ceil(max_len / 16) (rounded up to a "
                "power of two) below 2^24, their product below 2^32 table entries");
  const size_t table = (size_t)d->n_centroids * (size_t)P.n_cols * 4;
  pl.ws = (table + 255) / 256 * 256;
  int pipe = force_pipe;
  if (pipe < 0) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_res_tuned.find(ResKey{d->nbits, d->dim, P.nqb, cand ? 1 : 0});
    pipe = it == g_res_tuned.end() ? RES_DEFAULT_PIPE : it->second.pipe;
  }
  P.pipe = pipe;
  return MAXSIM_OK;
}

}  // namespace

size_t maxsim_residual_score_workspace_size(const maxsim_csr* queries,
                                            const maxsim_residual_docs* docs,
                                            const maxsim_candidates* cand) {
  ResPlan pl;
  std::string saved = g_err;
  if (plan_residual(queries, docs, cand, (float*)1, pl)) {
    g_err = saved;
    return 0;
  }
  return pl.ws;
}

maxsim_status maxsim_residual_score(const maxsim_csr* queries, const maxsim_residual_docs* docs,
                                    const maxsim_candidates* cand, float* scores,
                                    void* workspace, size_t ws_bytes, maxsim_stream_t stream) {
  ResPlan pl;
  maxsim_status st = plan_residual(queries, docs, cand, scores, pl);
  if (st) return st;
  if (pl.ws > 0 && (!workspace || ws_bytes < pl.ws))
    return fail(MAXSIM_EWORKSPACE, "residual: workspace needs %zu bytes", pl.ws);
  if (pl.ws > 0 && !aligned(workspace, 16))
    return fail(MAXSIM_EINVAL, "residual: workspace must be 16-byte aligned");
  const int64_t n_pairs = cand ? cand->n_total : queries->n_sets * docs->n_docs;
  if (n_pairs == 0) return MAXSIM_OK;
  pl.P.table = (float*)workspace;
  hipError_t e = launch_residual(pl.P, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "residual launch");
  return MAXSIM_OK;
}

maxsim_status maxsim_residual_autotune(const maxsim_csr* queries,
                                       const maxsim_residual_docs* docs,
                                       const maxsim_candidates* cand, float* scores,
                                       void* workspace, size_t ws_bytes, maxsim_stream_t stream,
                                       int32_t reps, const char* cache_path, char* report,
                                       size_t report_len) {
  ResPlan probe;
  maxsim_status st = plan_residual(queries, docs, cand, scores, probe);
  if (st) return st;
  if (probe.ws > 0 && (!workspace || ws_bytes < probe.ws))
    return fail(MAXSIM_EWORKSPACE, "residual autotune: workspace needs %zu bytes", probe.ws);
  const int64_t n_pairs = cand ? cand->n_total : queries->n_sets * docs->n_docs;
  if (reps < 1) reps = 1;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(MAXSIM_EHIP, "residual autotune: event creation failed");
  const ResKey key{docs->nbits, docs->dim, probe.P.nqb, cand ? 1 : 0};
  std::string rep = "{\"residual\":1,\"nbits\":" + std::to_string(key.nbits) +
                    ",\"dim\":" + std::to_string(key.dim) + ",\"nqb\":" +
                    std::to_string(key.nqb) + ",\"cand\":" + std::to_string(key.cand) +
                    ",\"trials\":[";
  float best_ms = 1e30f;
  int best = RES_DEFAULT_PIPE;
  bool first = true;
  for (int pipe = 0; pipe < RES_PIPES && n_pairs > 0; ++pipe) {
    ResPlan pl;
    if (plan_residual(queries, docs, cand, scores, pl, pipe)) continue;
    pl.P.table = (float*)workspace;
    if (launch_residual(pl.P, s) != hipSuccess) continue;
    (void)hipEventRecord(e0, s);
    bool ok = true;
    for (int r = 0; r < reps && ok; ++r) ok = launch_residual(pl.P, s) == hipSuccess;
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess || !ok) continue;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= reps;
    char b[96];
    snprintf(b, sizeof b, "%s{\"pipe\":%d,\"ms\":%.5f}", first ? "" : ",", pipe, ms);
    rep += b;
    first = false;
    if (ms < best_ms) {
      best_ms = ms;
      best = pipe;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  char b[96];
  snprintf(b, sizeof b, "],\"best\":{\"pipe\":%d,\"ms\":%.5f}}", best, best_ms);
  rep += b;
  std::string all;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_res_tuned[key] = ResCfg{best};
    all = cfg_json_all();
  }
  if (cache_path) {
    FILE* f = fopen(cache_path, "wb");
    if (!f) return fail(MAXSIM_EINVAL, "residual autotune: cannot write %s", cache_path);
    fputs(all.c_str(), f);
    fclose(f);
  }
  if (report && report_len > 0) snprintf(report, report_len, "%s", rep.c_str());
  return MAXSIM_OK;
}

size_t maxsim_topk_workspace_size(int64_t n_segments, int32_t k) {
  if (n_segments < 0 || k < 1 || k > 1024) return 0;
  return topk_ws_bytes(n_segments, k);
}

maxsim_status maxsim_topk(const float* scores, const int64_t* seg_offsets, int64_t n_segments,
                          int64_t n_total, const int32_t* ids, int32_t k, float* out_scores,
                          int32_t* out_ids, void* workspace, size_t ws_bytes,
                          maxsim_stream_t stream) {
  if (k < 1 || k > 1024) return fail(MAXSIM_EUNSUPPORTED, "topk: k must be in [1, 1024]");
  if (n_segments < 0 || n_total < 0) return fail(MAXSIM_EINVAL, "topk: negative sizes");
  if (n_segments > 65535) return fail(MAXSIM_EUNSUPPORTED, "topk: at most 65535 segments");
  if (n_segments == 0) return MAXSIM_OK;
  if (!seg_offsets || !out_scores || !out_ids || (n_total > 0 && !scores))
    return fail(MAXSIM_EINVAL, "topk: NULL pointer");
  size_t need = topk_ws_bytes(n_segments, k);
  if (!workspace || ws_bytes < need) return fail(MAXSIM_EWORKSPACE, "topk: workspace needs %zu bytes", need);
  hipError_t e = launch_topk(scores, seg_offsets, n_segments, n_total, ids, k, out_scores, out_ids,
                             workspace, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "topk launch");
  return MAXSIM_OK;
}

// ---------------------------------------------------- device checks --

namespace {

maxsim_status validate_common(const maxsim_csr* queries, const int64_t* doc_off, int64_t n_docs,
                              int64_t n_doc_tokens, const maxsim_candidates* cand,
                              int32_t* flags, hipStream_t s) {
  hipError_t e = launch_clear_flags(flags, s);
  if (e == hipSuccess)
    e = launch_check_offsets(doc_off, n_docs, n_doc_tokens, -1, MAXSIM_CHECK_DOC_OFFSETS, 0, flags,
                             s);
  if (e == hipSuccess && queries) {
    e = launch_check_offsets(queries->offsets, queries->n_sets, queries->n_tokens,
                             queries->max_len, MAXSIM_CHECK_QUERY_OFFSETS,
                             MAXSIM_CHECK_QUERY_LENGTH, flags, s);
    if (e == hipSuccess && queries->dtype == MAXSIM_F8E4M3)
      e = launch_check_scales(queries->scales, queries->n_tokens, MAXSIM_CHECK_FP8_SCALES, flags,
                              s);
  }
  if (e == hipSuccess && cand) {
    const int64_t nq = queries ? queries->n_sets : 0;
    if (queries)
      e = launch_check_offsets(cand->offsets, nq, cand->n_total, -1, MAXSIM_CHECK_CAND_OFFSETS, 0,
                               flags, s);
    if (e == hipSuccess)
      e = launch_check_ids(cand->doc_ids, cand->n_total, n_docs, MAXSIM_CHECK_CAND_IDS, flags, s);
  }
  if (e != hipSuccess) return hip_fail(e, "validate launch");
  return MAXSIM_OK;
}

maxsim_status check_cand_desc(const maxsim_csr* queries, const maxsim_candidates* cand) {
  if (!cand) return MAXSIM_OK;
  if (!queries) return fail(MAXSIM_EINVAL, "validate: candidates need the queries descriptor");
  if (cand->n_total < 0 || !cand->offsets || (cand->n_total > 0 && !cand->doc_ids))
    return fail(MAXSIM_EINVAL, "validate: bad candidates descriptor");
  return MAXSIM_OK;
}

}  // namespace

maxsim_status maxsim_validate(const maxsim_csr* queries, const maxsim_csr* docs,
                              const maxsim_candidates* cand, int32_t* flags,
                              maxsim_stream_t stream) {
  if (!flags) return fail(MAXSIM_EINVAL, "validate: flags is NULL");
  maxsim_status st = check_csr(docs, "docs", false);
  if (st) return st;
  if (queries && (st = check_csr(queries, "queries", true))) return st;
  if ((st = check_cand_desc(queries, cand))) return st;
  hipStream_t s = (hipStream_t)stream;
  st = validate_common(queries, docs->offsets, docs->n_sets, docs->n_tokens, cand, flags, s);
  if (st) return st;
  if (docs->dtype == MAXSIM_F8E4M3) {
    hipError_t e = launch_check_scales(docs->scales, docs->n_tokens, MAXSIM_CHECK_FP8_SCALES,
                                       flags, s);
    if (e != hipSuccess) return hip_fail(e, "validate launch");
  }
  return MAXSIM_OK;
}

maxsim_status maxsim_validate_pq(const maxsim_csr* queries, const maxsim_pq_docs* docs,
                                 const maxsim_candidates* cand, int32_t* flags,
                                 maxsim_stream_t stream) {
  if (!flags) return fail(MAXSIM_EINVAL, "validate: flags is NULL");
  if (!docs || !docs->offsets || docs->n_docs < 0 || docs->n_tokens < 0 ||
      (docs->n_tokens > 0 && !docs->codes) || docs->M < 1 || docs->K < 1)
    return fail(MAXSIM_EINVAL, "validate: bad PQ descriptor");
  maxsim_status st;
  if (queries && (st = check_csr(queries, "queries", true))) return st;
  if ((st = check_cand_desc(queries, cand))) return st;
  hipStream_t s = (hipStream_t)stream;
  st = validate_common(queries, docs->offsets, docs->n_docs, docs->n_tokens, cand, flags, s);
  if (st) return st;
  hipError_t e = launch_check_codes(docs->codes, docs->n_tokens * docs->M, docs->K,
                                    MAXSIM_CHECK_PQ_CODES, flags, s);
  if (e != hipSuccess) return hip_fail(e, "validate launch");
  return MAXSIM_OK;
}

maxsim_status maxsim_validate_residual(const maxsim_csr* queries,
                                       const maxsim_residual_docs* docs,
                                       const maxsim_candidates* cand, int32_t* flags,
                                       maxsim_stream_t stream) {
  if (!flags) return fail(MAXSIM_EINVAL, "validate: flags is NULL");
  if (!docs || !docs->offsets || docs->n_docs < 0 || docs->n_tokens < 0 ||
      (docs->n_tokens > 0 && !docs->centroid_ids) || docs->n_centroids < 1)
    return fail(MAXSIM_EINVAL, "validate: bad residual descriptor");
  maxsim_status st;
  if (queries && (st = check_csr(queries, "queries", true))) return st;
  if ((st = check_cand_desc(queries, cand))) return st;
  hipStream_t s = (hipStream_t)stream;
  st = validate_common(queries, docs->offsets, docs->n_docs, docs->n_tokens, cand, flags, s);
  if (st) return st;
  hipError_t e = launch_check_ids(docs->centroid_ids, docs->n_tokens, docs->n_centroids,
                                  MAXSIM_CHECK_CENTROID_IDS, flags, s);
  if (e != hipSuccess) return hip_fail(e, "validate launch");
  return MAXSIM_OK;
}

maxsim_status maxsim_check(const int32_t* flags, maxsim_stream_t stream) {
  if (!flags) return fail(MAXSIM_EINVAL, "check: flags is NULL");
  int32_t v = 0;
  hipError_t e = hipMemcpyAsync(&v, flags, sizeof v, hipMemcpyDeviceToHost, (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "check: reading the flags");
  if (v == 0) return MAXSIM_OK;
  static const char* names[] = {"document offsets",  "query offsets", "query longer than max_len",
                                "candidate offsets", "candidate ids", "FP8 scales",
                                "PQ codes",          "centroid ids"};
  std::string msg = "device check failed:";
  for (int b = 0; b < 8; ++b)
    if (v & (1 << b)) msg += std::string(" [") + names[b] + "]";
  return fail(MAXSIM_EDEVCHECK, "%s", msg.c_str());
}

// ------------------------------------------------------- read ceiling --

maxsim_status maxsim_stream_probe(const void* buf, size_t bytes, int32_t variant, uint32_t* sink,
                                  int64_t sink_len, maxsim_stream_t stream) {
  if (!buf || !sink) return fail(MAXSIM_EINVAL, "stream_probe: NULL buffer");
  if (!aligned(buf, 16)) return fail(MAXSIM_EINVAL, "stream_probe: buffer must be 16-byte aligned");
  if (variant < 0 || variant > 5) return fail(MAXSIM_EINVAL, "stream_probe: variant must be in [0, 5]");
  if (sink_len < 4) return fail(MAXSIM_EINVAL, "stream_probe: sink needs at least 4 entries");
  int64_t grid = std::min<int64_t>(sink_len / 4, (int64_t)device_info().cus * 8);
  hipError_t e = launch_stream_probe(buf, bytes, variant, sink, (int)grid, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "stream_probe launch");
  return MAXSIM_OK;
}

maxsim_status maxsim_lds_probe(const void* buf, size_t bytes, int32_t variant,
                               int32_t table_bytes, uint32_t* sink, int64_t sink_len,
                               maxsim_stream_t stream) {
  if (!buf || !sink) return fail(MAXSIM_EINVAL, "lds_probe: NULL buffer");
  if (!aligned(buf, 16)) return fail(MAXSIM_EINVAL, "lds_probe: buffer must be 16-byte aligned");
  if (variant < 0 || variant > 2) return fail(MAXSIM_EINVAL, "lds_probe: variant must be in [0, 2]");
  if (table_bytes != 65536 && table_bytes != 131072)
    return fail(MAXSIM_EINVAL, "lds_probe: table_bytes must be 65536 or 131072");
  if ((size_t)table_bytes > device_info().max_lds)
    return fail(MAXSIM_EUNSUPPORTED, "lds_probe: table exceeds the LDS");
  if (sink_len < 16) return fail(MAXSIM_EINVAL, "lds_probe: sink needs at least 16 entries");
  const int64_t grid = std::min<int64_t>(sink_len / 16, (int64_t)device_info().cus);
  hipError_t e =
      launch_lds_probe(buf, bytes, variant, table_bytes, sink, (int)grid, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "lds_probe launch");
  return MAXSIM_OK;
}

// ------------------------------------------------------------ autotune --

maxsim_status maxsim_load_tune_cache(const char* path) {
  if (!path) return fail(MAXSIM_EINVAL, "load_tune_cache: NULL path");
  FILE* f = fopen(path, "rb");
  if (!f) return MAXSIM_OK;
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
  fclose(f);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  size_t pos = 0;
  while ((pos = txt.find("{\"dtype\"", pos)) != std::string::npos) {
    size_t end = txt.find('}', pos);
    if (end == std::string::npos) break;
    std::string obj = txt.substr(pos, end - pos + 1);
    TuneKey k{};
    FusedCfg c{};
    if (json_int(obj.c_str(), "dtype", k.dt) && json_int(obj.c_str(), "dim", k.dim) &&
        json_int(obj.c_str(), "nqb", k.nqb) && json_int(obj.c_str(), "pf", c.pf) &&
        json_int(obj.c_str(), "nw", c.nw) && json_int(obj.c_str(), "wg_per_cu", c.wg_per_cu)) {
      if (!json_int(obj.c_str(), "stage", c.stage)) c.stage = 0;  // older caches
      if (!json_int(obj.c_str(), "rows", c.rows)) c.rows = 16;
      if ((c.pf >= 2 && c.pf <= 4) && (c.nw == 4 || c.nw == 8) && (c.stage == 0 || c.stage == 1) &&
          (c.rows == 16 || c.rows == 32))
        g_tuned[k] = c;
    }
    pos = end;
  }
  pos = 0;
  while ((pos = txt.find("{\"pq\"", pos)) != std::string::npos) {
    size_t end = txt.find('}', pos);
    if (end == std::string::npos) break;
    std::string obj = txt.substr(pos, end - pos + 1);
    PqKey k{};
    PqCfg c{};
    if (json_int(obj.c_str(), "M", k.M) && json_int(obj.c_str(), "dsub", k.dsub) &&
        json_int(obj.c_str(), "bpq", k.bpq) && json_int(obj.c_str(), "cand", k.cand) &&
        json_int(obj.c_str(), "variant", c.variant) && json_int(obj.c_str(), "nqb", c.nqb)) {
      if ((c.variant == 0 || c.variant == 1) && (c.nqb >= 0 && c.nqb <= 8)) g_pq_tuned[k] = c;
    }
    pos = end;
  }
  pos = 0;
  while ((pos = txt.find("{\"residual\"", pos)) != std::string::npos) {
    size_t end = txt.find('}', pos);
    if (end == std::string::npos) break;
    std::string obj = txt.substr(pos, end - pos + 1);
    ResKey k{};
    ResCfg c{};
    if (json_int(obj.c_str(), "nbits", k.nbits) && json_int(obj.c_str(), "dim", k.dim) &&
        json_int(obj.c_str(), "nqb", k.nqb) && json_int(obj.c_str(), "cand", k.cand) &&
        json_int(obj.c_str(), "pipe", c.pipe) && c.pipe >= 0 && c.pipe < RES_PIPES)
      g_res_tuned[k] = c;
    pos = end;
  }
  return MAXSIM_OK;
}

maxsim_status maxsim_autotune(const maxsim_csr* queries, const maxsim_csr* docs,
                              const maxsim_candidates* cand, float* scores, void* workspace,
                              size_t ws_bytes, maxsim_stream_t stream, int32_t reps,
                              const char* cache_path, char* report, size_t report_len) {
  (void)workspace;
  (void)ws_bytes;
  FusedPlan pl;
  maxsim_status st = plan_fused(queries, docs, cand, scores, pl);
  if (st) return st;
  if (reps < 1) reps = 1;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(MAXSIM_EHIP, "autotune: event creation failed");
  std::vector<FusedCfg> space;
  const bool rows32 = pl.dt == MAXSIM_F8E4M3 && pl.qreg;
  for (int rows : {16, 32})
    for (int stage : {0, 1})
      for (int pf : {2, 3, 4})
        for (int nw : {4, 8})
          for (int wpc : {0, 1, 2}) {
            if (rows == 32 && (!rows32 || !stage)) continue;
            FusedCfg c;
            c.pf = pf;
            c.nw = nw;
            c.wg_per_cu = wpc;
            c.stage = stage;
            c.rows = rows;
            space.push_back(c);
          }
  std::string rep = "{\"dtype\":" + std::to_string(pl.dt) + ",\"dim\":" +
                    std::to_string(queries->dim) + ",\"nqb\":" + std::to_string(pl.nqb) +
                    ",\"trials\":[";
  float best_ms = 1e30f;
  FusedCfg best = default_cfg(pl.dt, pl.qreg ? 0 : pl.lds, pl.dch);
  bool first = true;
  for (const FusedCfg& c : space) {
    if (run_fused(pl, c, s)) continue;  // warm-up (also skips shapes that do not fit)
    (void)hipEventRecord(e0, s);
    bool ok = true;
    for (int r = 0; r < reps && ok; ++r) ok = run_fused(pl, c, s) == MAXSIM_OK;
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess || !ok) continue;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= reps;
    char b[128];
    snprintf(b, sizeof b,
             "%s{\"stage\":%d,\"rows\":%d,\"pf\":%d,\"nw\":%d,\"wg_per_cu\":%d,\"ms\":%.5f}",
             first ? "" : ",", c.stage, c.rows, c.pf, c.nw, c.wg_per_cu, ms);
    rep += b;
    first = false;
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  char b[128];
  snprintf(b, sizeof b,
           "],\"best\":{\"stage\":%d,\"rows\":%d,\"pf\":%d,\"nw\":%d,\"wg_per_cu\":%d,"
           "\"ms\":%.5f}}",
           best.stage, best.rows, best.pf, best.nw, best.wg_per_cu, best_ms);
  rep += b;
  std::string all;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[{pl.dt, queries->dim, pl.nqb}] = best;
    all = cfg_json_all();
  }
  if (cache_path) {
    FILE* f = fopen(cache_path, "wb");
    if (!f) return fail(MAXSIM_EINVAL, "autotune: cannot write %s", cache_path);
    fputs(all.c_str(), f);
    fclose(f);
  }
  if (report && report_len > 0) {
    size_t n = std::min(report_len - 1, rep.size());
    memcpy(report, rep.data(), n);
    report[n] = 0;
  }
  return MAXSIM_OK;
}
