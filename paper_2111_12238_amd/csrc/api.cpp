// C ABI of the fused sparse executor: schedule lifecycle, device upload,
// executor calls, refinement driver and autotuner.  See include/sf.h for the
// contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "kargs.h"
#include "probe.h"
#include "schedule.h"

using namespace sf;

namespace {

sf_status hip_status(hipError_t e) {
  if (e == hipSuccess) return SF_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SF_ERR_OOM;
  return SF_ERR_HIP;
}

#define SF_HIP(x)                                  \
  do {                                             \
    const hipError_t e_ = (x);                     \
    if (e_ != hipSuccess) return hip_status(e_);   \
  } while (0)

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return cus;
}

// Sub-allocator over one hipMalloc'ed block: arrays are placed at 256-byte
// aligned offsets.
struct Packer {
  struct Item {
    size_t at;
    const void* data;
    size_t bytes;
  };
  size_t off = 0;
  std::vector<Item> items;
  template <typename E>
  size_t add(const std::vector<E>* v) {
    const size_t at = off;
    const size_t bytes = v->size() * sizeof(E);
    items.push_back({at, v->data(), bytes});
    off += (bytes + 255) / 256 * 256;
    if (bytes == 0) off += 256;
    return at;
  }
};

uint64_t pattern_fingerprint(sf_schedule_s* s);  // autotuner cache key (below)

// Record that every launch of an executor call is enqueued on `stream`
// (the schedule's "done" event, created with its device arrays) and pass r
// through.
sf_status enqueued(sf_schedule_s* s, void* stream, sf_status r) {
  if (r != SF_OK || !s || !s->dev.ready || !s->dev.done) return r;
  return hip_status(hipEventRecord(static_cast<hipEvent_t>(s->dev.done), static_cast<hipStream_t>(stream)));
}

// Wait until the work of the last executor call on the schedule is done.
void wait_done(sf_schedule_s* s) {
  if (s->dev.done) hipEventSynchronize(static_cast<hipEvent_t>(s->dev.done));
}

// Release the device buffers once the last executor call's work is done.
void free_device(sf_schedule_s* s) {
  DeviceBuffers& d = s->dev;
  if (d.device >= 0) {
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(d.device);
    if (d.done) {
      hipEventSynchronize(static_cast<hipEvent_t>(d.done));
      hipEventDestroy(static_cast<hipEvent_t>(d.done));
    }
    if (d.block) hipFree(d.block);
    if (d.state) hipFree(d.state);
    if (d.xi) hipFree(d.xi);
    if (d.units) hipFree(d.units);
    for (StaticPlan* P : {&s->msp, &s->wavefront})
      if (P->dev) hipFree(P->dev);
    hipSetDevice(cur);
  }
  for (StaticPlan* P : {&s->msp, &s->wavefront}) P->dev = nullptr;
  d = DeviceBuffers();
}

// Upload the constant arrays and the work items; allocate the state block
// and one flag per row.  Called at the first executor call (and again after
// the items are re-cut by the autotuner).
sf_status upload(sf_schedule_s* s, hipStream_t st) {
  DeviceBuffers& d = s->dev;
  int cur = 0;
  SF_HIP(hipGetDevice(&cur));
  if (d.ready && d.device == cur) return SF_OK;
  if (d.ready && d.device != cur) return SF_ERR_ARG;  // a schedule lives on one device
  Packer pk;
  const size_t oLrp = pk.add(&s->L.rp), oLci = pk.add(&s->L.ci);
  const size_t oArp = pk.add(&s->A.rp), oAci = pk.add(&s->A.ci);
  const size_t oOrd = pk.add(&s->order), oIp = pk.add(&s->item_ptr), oTi = pk.add(&s->trsv_items);
  const size_t oSi = pk.add(&s->spmv_items);
  const size_t oLi = pk.add(&s->lvl_items), oLip = pk.add(&s->lvl_item_ptr);
  const size_t oLTrp = pk.add(&s->LT.rp), oLTci = pk.add(&s->LT.ci), oLTm = pk.add(&s->LT_map);
  const size_t oATrp = pk.add(&s->AT.rp), oATci = pk.add(&s->AT.ci), oATm = pk.add(&s->AT_map);
  const size_t oBo = pk.add(&s->border), oBip = pk.add(&s->bitem_ptr);
  const size_t oPp = pk.add(&s->pair_ptr), oPu = pk.add(&s->pair_u), oPq = pk.add(&s->pair_q);
  const size_t oDp = pk.add(&s->dpos), oPr = pk.add(&s->prng), oPv = pk.add(&s->piv);
  const size_t oCo = pk.add(&s->corder), oCip = pk.add(&s->citem_ptr), oCti = pk.add(&s->ctrsv_items);
  const size_t oCl = pk.add(&s->clloc), oCe = pk.add(&s->celoc);
  const size_t oQr = pk.add(&s->qrng), oCqr = pk.add(&s->cqrng);
  const size_t oBco = pk.add(&s->bcorder), oBcip = pk.add(&s->bcitem_ptr);
  const size_t oBcl = pk.add(&s->bclloc), oBce = pk.add(&s->bceloc);
  const size_t oRo = pk.add(&s->rorder), oRip = pk.add(&s->ritem_ptr), oRti = pk.add(&s->rtrsv_items);
  const size_t oRq = pk.add(&s->rqrng), oRr = pk.add(&s->rroff), oRb = pk.add(&s->rbatch);
  const size_t oRbp = pk.add(&s->rbatch_ptr), oRx = pk.add(&s->rext), oRxp = pk.add(&s->rext_ptr);
  const size_t oRc = pk.add(&s->rcode);
  const size_t oPqr = pk.add(&s->pqrng), oApre = pk.add(&s->apre);
  const size_t oBro = pk.add(&s->brorder), oBrip = pk.add(&s->britem_ptr), oBrr = pk.add(&s->brroff);
  const size_t oBrb = pk.add(&s->brbatch), oBrbp = pk.add(&s->brbatch_ptr), oBrx = pk.add(&s->brext);
  const size_t oBrxp = pk.add(&s->brext_ptr), oBrc = pk.add(&s->brcode);
  void* block = nullptr;
  SF_HIP(hipMalloc(&block, pk.off));
  char* b = static_cast<char*>(block);
  for (auto& it : pk.items)
    if (it.bytes)
      if (hipMemcpyAsync(b + it.at, it.data, it.bytes, hipMemcpyHostToDevice, st) != hipSuccess) {
        hipFree(block);
        return SF_ERR_HIP;
      }
  auto P = [&](size_t o) { return reinterpret_cast<int32_t*>(b + o); };
  d.block = block;
  d.block_bytes = pk.off;
  d.Lrp = P(oLrp); d.Lci = P(oLci); d.Arp = P(oArp); d.Aci = P(oAci);
  d.order = P(oOrd); d.item_ptr = P(oIp); d.trsv_items = P(oTi); d.spmv_items = P(oSi);
  d.lvl_items = P(oLi); d.lvl_item_ptr = P(oLip);
  d.LTrp = P(oLTrp); d.LTci = P(oLTci); d.LTmap = P(oLTm);
  d.ATrp = P(oATrp); d.ATci = P(oATci); d.ATmap = P(oATm);
  d.border = P(oBo); d.bitem_ptr = P(oBip);
  d.pair_ptr = P(oPp); d.pair_u = P(oPu); d.pair_q = P(oPq);
  d.dpos = P(oDp);
  d.prng = P(oPr);
  d.piv = P(oPv);
  d.corder = P(oCo); d.citem_ptr = P(oCip); d.ctrsv_items = P(oCti);
  d.clloc = reinterpret_cast<uint8_t*>(b + oCl);
  d.celoc = reinterpret_cast<uint8_t*>(b + oCe);
  d.qrng = P(oQr); d.cqrng = P(oCqr);
  d.bcorder = P(oBco); d.bcitem_ptr = P(oBcip);
  d.bclloc = reinterpret_cast<uint8_t*>(b + oBcl);
  d.bceloc = reinterpret_cast<uint8_t*>(b + oBce);
  d.rorder = P(oRo); d.ritem_ptr = P(oRip); d.rtrsv_items = P(oRti); d.rqrng = P(oRq); d.rroff = P(oRr);
  d.rbatch = P(oRb); d.rbatch_ptr = P(oRbp); d.rext = P(oRx); d.rext_ptr = P(oRxp);
  d.rcode = reinterpret_cast<uint16_t*>(b + oRc);
  d.pqrng = P(oPqr); d.apre = P(oApre);
  d.brorder = P(oBro); d.britem_ptr = P(oBrip); d.brroff = P(oBrr);
  d.brbatch = P(oBrb); d.brbatch_ptr = P(oBrbp); d.brext = P(oBrx); d.brext_ptr = P(oBrxp);
  d.brcode = reinterpret_cast<uint16_t*>(b + oBrc);
  if (!d.state) {
    std::vector<int32_t> init(kStateWords, 0);
    for (int p = 0; p < 2; ++p) init[info_off(p)] = kInfoNone;
    SF_HIP(hipMalloc(&d.state, kStateWords * sizeof(int32_t)));
    SF_HIP(hipMemcpy(d.state, init.data(), kStateWords * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  if (!d.done) {
    hipEvent_t ev = nullptr;
    SF_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    d.done = ev;
  }
  SF_HIP(hipStreamSynchronize(st));  // host vectors may change after a re-cut
  d.device = cur;
  d.ready = true;
  return SF_OK;
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Library-owned workspace of the multi-RHS executors, all in the
// interleaved block layout (k_layout.hip): the solution xi (its own
// readiness flags; the refinement reads it as the correction), the packed
// right-hand sides bi and the packed SpMV result yi.
struct MultiWs {
  void* xi;
  void* bi;
  void* yi;
};

sf_status multi_ws(sf_schedule_s* s, int kb, int nrhs, size_t es, hipStream_t st, MultiWs& w) {
  DeviceBuffers& d = s->dev;
  // the executors address a block's interleaved x with 32-bit offsets
  if (int64_t(s->n) * kb > int64_t(INT32_MAX)) return SF_ERR_UNSUPPORTED;
  const size_t cols = size_t((nrhs + kb - 1) / kb) * size_t(kb);
  const size_t bx = align256(std::max<size_t>(size_t(s->n) * cols * es, 1));
  const size_t by = align256(std::max<size_t>(size_t(s->m) * cols * es, 1));
  const size_t bytes = 2 * bx + by;
  if (d.xi_bytes < bytes) {
    SF_HIP(hipStreamSynchronize(st));
    wait_done(s);
    if (d.xi) SF_HIP(hipFree(d.xi));
    d.xi = nullptr;
    d.xi_bytes = 0;
    SF_HIP(hipMalloc(&d.xi, bytes));
    d.xi_bytes = bytes;
  }
  char* b = static_cast<char*>(d.xi);
  w.xi = b;
  w.bi = b + bx;
  w.yi = b + 2 * bx;
  return SF_OK;
}

// Next launch epoch.  Only its parity matters on the device (the state
// block alternates by parity); the counter restarts before it could wrap,
// keeping the parity sequence.
sf_status next_epoch(sf_schedule_s* s, hipStream_t st, LaunchState& ls) {
  DeviceBuffers& d = s->dev;
  uint32_t e = d.epoch + 1;
  if (e >= (1u << 30)) e = (e & 1u) ? 1u : 2u;
  d.epoch = e;
  ls.state = d.state;
  ls.epoch = int32_t(e);
  ls.spin_limit = int32_t(std::min<int64_t>(s->spin_limit, std::numeric_limits<int32_t>::max()));
  ls.streams = std::max(1, std::min(s->claim_streams, kStreams));
  return SF_OK;
}

int persistent_grid(sf_schedule_s* s, int occupancy_blocks_per_cu, int waves_per_cu = 0) {
  const int cus = std::max(1, device_cus());
  const int want = std::max(1, (waves_per_cu > 0 ? waves_per_cu : s->waves_per_cu) * 64 / kBlockThreads);
  const int per_cu = std::min(want, std::max(1, occupancy_blocks_per_cu));
  return std::max(cus * per_cu, kStreams);
}

struct Timer {
  sf_schedule_s* s;
  hipStream_t st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  Timer(sf_schedule_s* s_, hipStream_t st_) : s(s_), st(st_) {
    if (s->timing) {
      hipEventCreate(&e0);
      hipEventCreate(&e1);
      hipEventRecord(e0, st);
    }
  }
  void stop() {
    if (s->timing && e0) {
      hipEventRecord(e1, st);
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      s->last_kernel_ms = ms;
      hipEventDestroy(e0);
      hipEventDestroy(e1);
      e0 = e1 = nullptr;
    }
  }
  ~Timer() { stop(); }
};

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

int default_kb(int nrhs) {
  int kb = 2;
  while (kb < nrhs && kb < 64) kb *= 2;
  return kb;
}

// Right-hand sides per block of the multi-RHS solve (1 for a single one).
int solve_kb(const sf_schedule_s* s, int nrhs) {
  if (nrhs == 1) return 1;
  return s->rhs_block > 0 ? std::min(s->rhs_block, 64) : default_kb(nrhs);
}

TsArgs ts_args(sf_schedule_s* s, const void* Lv, const void* Av, const void* B, int ldb, int nrhs,
               void* X, int ldx, void* Y, int ldy) {
  const DeviceBuffers& d = s->dev;
  TsArgs a{};
  a.n = int32_t(s->n);
  a.m = int32_t(s->m);
  a.Lrp = d.Lrp; a.Lci = d.Lci; a.Lv = Lv;
  a.Arp = d.Arp; a.Aci = d.Aci; a.Av = Av;
  a.B = B; a.ldb = ldb; a.X = X; a.ldx = ldx; a.Y = Y; a.ldy = ldy;
  a.nrhs = nrhs;
  a.order = d.order;
  a.qrng = d.qrng;
  a.item_ptr = d.item_ptr;
  if (Y) {
    a.item_list = nullptr;
    a.n_work = int32_t(s->item_ptr.size() - 1);
  } else {
    a.item_list = d.trsv_items;
    a.n_work = int32_t(s->trsv_items.size());
  }
  return a;
}

// Multi-RHS plan for blocks of 64 / rpb rows: the level items split into
// units of at most rpb rows (rows of a level item are independent, so the
// units keep the claim order valid), kept on the device until the items are
// re-cut or another block width is asked for.  Per unit the range of its
// claim positions; the SpTRSV units alone (in claim order, hence by level)
// and, per level, the first of them for the level-set baseline.
sf_status ensure_units(sf_schedule_s* s, int rpb, hipStream_t st) {
  DeviceBuffers& d = s->dev;
  if (d.units && d.units_rpb == rpb) return SF_OK;
  std::vector<int32_t> all, trsv, lvl(size_t(std::max(s->depth, 0)) + 1, 0);
  for (size_t t = 0; t + 1 < s->item_ptr.size(); ++t)
    for (int32_t b = s->item_ptr[t]; b < s->item_ptr[t + 1]; b += rpb) {
      const int32_t e = std::min(b + rpb, s->item_ptr[t + 1]);
      all.push_back(b);
      all.push_back(e);
      const int32_t id = s->order[b];
      if (id < s->n) {
        trsv.push_back(b);
        trsv.push_back(e);
        ++lvl[size_t(s->level[id]) + 1];
      }
    }
  for (size_t l = 1; l < lvl.size(); ++l) lvl[l] += lvl[l - 1];
  SF_HIP(hipStreamSynchronize(st));
  wait_done(s);
  if (d.units) SF_HIP(hipFree(d.units));
  d.units = nullptr;
  const size_t b0 = std::max<size_t>(all.size(), 2) * 4, b1 = std::max<size_t>(trsv.size(), 2) * 4;
  SF_HIP(hipMalloc(&d.units, b0 + b1 + lvl.size() * 4));
  d.unit_rng = static_cast<int32_t*>(d.units);
  d.unit_trsv_rng = reinterpret_cast<int32_t*>(static_cast<char*>(d.units) + b0);
  d.lvl_unit_ptr = reinterpret_cast<int32_t*>(static_cast<char*>(d.units) + b0 + b1);
  if (!all.empty()) SF_HIP(hipMemcpy(d.unit_rng, all.data(), all.size() * 4, hipMemcpyHostToDevice));
  if (!trsv.empty()) SF_HIP(hipMemcpy(d.unit_trsv_rng, trsv.data(), trsv.size() * 4, hipMemcpyHostToDevice));
  SF_HIP(hipMemcpy(d.lvl_unit_ptr, lvl.data(), lvl.size() * 4, hipMemcpyHostToDevice));
  d.units_rpb = rpb;
  d.n_units = int32_t(all.size() / 2);
  d.n_unit_trsv = int32_t(trsv.size() / 2);
  return SF_OK;
}

// Residency target of the multi-RHS executors.  Units of one level run in
// parallel and a few levels overlap; wavefronts beyond that only poll, so
// by default the target follows the units per level (mean level width over
// the rows per unit, times the blocks).
int multi_waves(const sf_schedule_s* s, int kb, int nrhs) {
  if (s->multi_waves_per_cu > 0) return s->multi_waves_per_cu;
  const double width = double(s->n) / double(std::max(s->depth, 1));
  const double units = width / double(std::max(1, 64 / kb)) * double((nrhs + kb - 1) / kb);
  return units < 256 ? 8 : (units < 4096 ? 16 : 32);
}

// Fused multi-RHS executor on interleaved data: bi (n rows) -> xi, whose
// every value must hold the pending pattern, and yi (m rows; nullptr = no
// SpMV), nblk = ceil(nrhs / kb) blocks of kb columns.
sf_status exec_multi_core(sf_schedule_s* s, int dtype, const void* Lv, const void* Av, const void* bi, void* xi,
                          void* yi, int nrhs, int kb, hipStream_t st) {
  TsArgs a = ts_args(s, Lv, Av, bi, int32_t(s->n), nrhs, nullptr, int32_t(s->n), yi, int32_t(s->m));
  sf_status r = ensure_units(s, std::max(1, 64 / kb), st);
  if (r != SF_OK) return r;
  a.unit_rng = reinterpret_cast<const int2*>(yi ? s->dev.unit_rng : s->dev.unit_trsv_rng);
  a.item_ptr = nullptr;
  a.item_list = nullptr;
  a.n_work = yi ? s->dev.n_units : s->dev.n_unit_trsv;
  if (a.n_work == 0) return SF_OK;
  r = next_epoch(s, st, a.ls);
  if (r != SF_OK) return r;
  a.kb = kb;
  a.nblk = (nrhs + kb - 1) / kb;
  a.xi = xi;
  const int grid = persistent_grid(s, occupancy_ts_multi(dtype, kb), multi_waves(s, kb, nrhs));
  return hip_status(launch_ts_multi(a, dtype, kb, grid, st));
}

// The region poller's settings from the "region_poll" parameter: lanes
// (bits 0-7), back-off rounds (bits 8-15), lanes before the first input
// (bits 16-23, 0 = all lanes).
static void set_poll(RegionArgs& r, int32_t v) {
  r.poll_lanes = std::max(1, std::min(64, v & 0xff));
  r.poll_sleep = (v >> 8) & 0xff;
  const int gate = (v >> 16) & 0xff;
  r.poll_gate = gate == 0 ? r.poll_lanes : std::min(gate, r.poll_lanes);
}

RegionArgs region_args(const sf_schedule_s* s) {
  RegionArgs r{};
  r.batch = s->dev.rbatch;
  r.batch_ptr = s->dev.rbatch_ptr;
  r.ext = s->dev.rext;
  r.ext_ptr = s->dev.rext_ptr;
  r.roff = s->dev.rroff;
  r.code = s->dev.rcode;
  r.rows_max = std::max(1, s->region_rows_max);
  r.entries_max = std::max(1, s->region_entries_max);
  r.ext_max = std::max(1, s->region_ext_max);
  r.batches_max = std::max(1, s->region_batches_max);
  set_poll(r, s->region_poll);
  return r;
}

// The backward region plan's arguments (k_bwd_region).
RegionArgs back_region_args(const sf_schedule_s* s) {
  RegionArgs r{};
  r.batch = s->dev.brbatch;
  r.batch_ptr = s->dev.brbatch_ptr;
  r.ext = s->dev.brext;
  r.ext_ptr = s->dev.brext_ptr;
  r.roff = s->dev.brroff;
  r.code = s->dev.brcode;
  r.rows_max = std::max(1, s->back_region_rows_max);
  r.entries_max = std::max(1, s->back_region_entries_max);
  r.ext_max = std::max(1, s->back_region_ext_max);
  r.batches_max = std::max(1, s->back_region_batches_max);
  set_poll(r, s->region_poll);
  return r;
}

// 64-bit words of the trace buffer: the item records, then two words per
// iteration id (trace mode, kTraceItemWords).
size_t trace_words(const sf_schedule_s* s) {
  return s->trace_items * kTraceItemWords + 2 * size_t(s->n + s->m);
}

// Several right-hand sides as one chain of the single-RHS items per column
// (multi_path 2, or by default on a coarsened plan of a narrow DAG -- mean
// wavefront under 2048 rows -- with at most 8 right-hand sides) instead of
// interleaved blocks over the level units.
bool column_chains(const sf_schedule_s* s, int nrhs) {
  const bool narrow = s->n < 2048 * int64_t(std::max(s->depth, 1));
  return nrhs > 1 && (s->multi_path == 2 || (s->multi_path == 0 && s->chunked && nrhs <= 8 && narrow));
}

sf_status exec_ts_fused(sf_schedule_s* s, sf_dtype dt, const void* Lv, const void* Av, const void* B,
                        int ldb, int nrhs, void* X, int ldx, void* Y, int ldy, hipStream_t st) {
  const int dtype = dt == SF_F64 ? 0 : 1;
  const size_t es = dt == SF_F64 ? 8 : 4;
  TsArgs a = ts_args(s, Lv, Av, B, ldb, nrhs, X, ldx, Y, ldy);
  if (a.n_work == 0) return SF_OK;
  // x doubles as its own readiness flag: it is filled with the pending
  // pattern first (part of the timed execution).  Several right-hand sides
  // run either in interleaved blocks over the level units (below) or, with
  // column chains, as separate chains of the single-RHS items on the
  // caller's columns (multi_path).  Chains gather one value per column and
  // entry, so they pay only where the units' hop per level dominates: by
  // default on a coarsened plan of a narrow DAG (mean wavefront under 2048
  // rows) with at most 8 right-hand sides (2D 9-point 2048^2, k = 8: 9.3 ->
  // 7.8 ms; at k >= 32, or on wide DAGs, the units are faster).
  if (nrhs == 1 || column_chains(s, nrhs)) {
    if (int64_t(a.n_work) * nrhs > int64_t(INT32_MAX) / 2) return SF_ERR_UNSUPPORTED;
    sf_status r = next_epoch(s, st, a.ls);
    if (r != SF_OK) return r;
    a.kb = 1;
    a.nblk = 1;
    a.col_units = nrhs;
    a.cached = s->cached_reads;
    a.trace = nrhs == 1 ? s->trace : nullptr;
    a.rtrace = a.trace && s->trace_level == 1 ? a.trace + s->trace_items * kTraceItemWords : nullptr;
    if (s->regioned) {
      a.order = s->dev.rorder;
      a.qrng = s->dev.rqrng;
      a.item_ptr = s->dev.ritem_ptr;
      a.item_list = Y ? nullptr : s->dev.rtrsv_items;
      a.n_work = Y ? int32_t(s->ritem_ptr.size() - 1) : int32_t(s->rtrsv_items.size());
      if (int64_t(a.n_work) * nrhs > int64_t(INT32_MAX) / 2) return SF_ERR_UNSUPPORTED;
      const RegionArgs ra = region_args(s);
      // blocks of two wavefronts (a computing and a polling one)
      const int waves = nrhs == 1 ? s->waves_per_cu : (s->multi_waves_per_cu > 0 ? s->multi_waves_per_cu : 8);
      const int per_cu = std::min(std::max(1, occupancy_region(ra, dtype)), std::max(1, waves / 2));
      const int grid = std::max(std::max(1, device_cus()) * per_cu, kStreams);
      if (a.trace) SF_HIP(launch_fill_u64(a.trace, int32_t(trace_words(s)), st));
      SF_HIP(launch_fill_pending_cols(X, int32_t(s->n), ldx, nrhs, dtype, st));
      Timer tm(s, st);  // the executor's kernel alone
      return hip_status(launch_ts_region(a, ra, dtype, grid, st));
    }
    if (s->chunked) {
      a.order = s->dev.corder;
      a.qrng = s->dev.cqrng;
      a.item_ptr = s->dev.citem_ptr;
      a.item_list = Y ? nullptr : s->dev.ctrsv_items;
      a.n_work = Y ? int32_t(s->citem_ptr.size() - 1) : int32_t(s->ctrsv_items.size());
      a.lloc = s->dev.clloc;
      a.eloc = s->dev.celoc;
    }
    // prefix fusion on level items: SpMV rows' prefixes are folded by their
    // SpTRSV rows and handed over through Y (filled with the pending pattern)
    const bool prefix = !s->chunked && Y && s->spmv_prefix && !s->apre.empty();
    if (prefix) {
      a.qrng = s->dev.pqrng;
      a.apre = s->dev.apre;
    }
    const int waves = nrhs == 1 ? s->waves_per_cu
                                : (s->multi_waves_per_cu > 0 ? s->multi_waves_per_cu : (nrhs <= 8 ? 8 : 16));
    const int grid = persistent_grid(s, prefix ? occupancy_ts_fused_pre(dtype) : occupancy_ts_fused(dtype), waves);
    if (a.trace) SF_HIP(launch_fill_u64(a.trace, int32_t(trace_words(s)), st));  // counts start at 0
    SF_HIP(launch_fill_pending_cols(X, int32_t(s->n), ldx, nrhs, dtype, st));
    if (prefix) SF_HIP(launch_fill_pending_cols(Y, int32_t(s->m), ldy, nrhs, dtype, st));
    Timer tm(s, st);  // the executor's kernel alone
    return hip_status(launch_ts_fused(a, dtype, grid, st));
  }
  const int kb = solve_kb(s, nrhs);
  MultiWs w{};
  sf_status r = multi_ws(s, kb, nrhs, es, st, w);
  if (r == SF_OK) r = ensure_units(s, std::max(1, 64 / kb), st);  // before the timed region
  if (r != SF_OK) return r;
  Timer tm(s, st);
  // B -> interleaved blocks, the solution buffer filled with the pending pattern
  SF_HIP(launch_pack(B, dtype, ldb, int32_t(s->n), nrhs, w.bi, dtype, w.xi, kb, st));
  r = exec_multi_core(s, dtype, Lv, Av, w.bi, w.xi, Y ? w.yi : nullptr, nrhs, kb, st);
  if (r != SF_OK) return r;
  SF_HIP(launch_unpack(w.xi, dtype, int32_t(s->n), nrhs, X, ldx, kb, st));
  if (Y) SF_HIP(launch_unpack(w.yi, dtype, int32_t(s->m), nrhs, Y, ldy, kb, st));
  return SF_OK;
}

sf_status exec_ts_unfused(sf_schedule_s* s, sf_dtype dt, const void* Lv, const void* Av, const void* B,
                          int ldb, int nrhs, void* X, int ldx, void* Y, int ldy, hipStream_t st) {
  const int dtype = dt == SF_F64 ? 0 : 1;
  const size_t es = dt == SF_F64 ? 8 : 4;
  LevelArgs la{};
  la.ts = ts_args(s, Lv, Av, B, ldb, nrhs, X, ldx, Y, ldy);
  la.ts.item_list = s->dev.lvl_items;
  la.ts.n_work = int32_t(s->lvl_items.size());
  la.lvl_item_ptr = s->dev.lvl_item_ptr;
  la.depth = s->depth;
  // several right-hand sides: the same interleaved blocks as the fused path
  const int kb = solve_kb(s, nrhs);
  MultiWs w{};
  if (nrhs > 1) {
    // the level's SpTRSV units (as in the fused path), spread over the grid
    sf_status r = multi_ws(s, kb, nrhs, es, st, w);
    if (r == SF_OK) r = ensure_units(s, std::max(1, 64 / kb), st);
    if (r != SF_OK) return r;
    la.ts.B = w.bi;
    la.ts.X = nullptr;
    la.ts.xi = w.xi;
    la.ts.unit_rng = reinterpret_cast<const int2*>(s->dev.unit_trsv_rng);
    la.lvl_item_ptr = s->dev.lvl_unit_ptr;
  }
  la.ts.kb = kb;
  la.ts.nblk = (nrhs + kb - 1) / kb;
  sf_status r = next_epoch(s, st, la.ts.ls);
  if (r != SF_OK) return r;
  Timer tm(s, st);
  if (nrhs > 1) SF_HIP(launch_pack(B, dtype, ldb, int32_t(s->n), nrhs, w.bi, dtype, nullptr, kb, st));
  if (s->n > 0 && s->depth > 0) {
    const int cus = std::max(1, device_cus());
    const int occ = occupancy_trsv_levelset(dtype, kb);
    int grid = cus * std::min(occ, std::max(1, s->levelset_waves_per_cu * 64 / kBlockThreads));
    SF_HIP(launch_trsv_levelset(la, dtype, grid, st));
  }
  if (Y && s->m > 0 && nrhs == 1) {
    TsArgs sa = ts_args(s, Lv, Av, B, ldb, nrhs, X, ldx, Y, ldy);
    sa.item_list = s->dev.spmv_items;
    sa.n_work = int32_t(s->spmv_items.size());
    SF_HIP(launch_spmv_items(sa, dtype, st));
  } else if (Y && s->m > 0) {
    SpmvArgs sa{};
    sa.m = int32_t(s->m);
    sa.n = int32_t(s->n);
    sa.kb = kb;
    sa.nblk = la.ts.nblk;
    sa.Arp = s->dev.Arp;
    sa.Aci = s->dev.Aci;
    sa.Av = Av;
    sa.X = w.xi;
    sa.Y = w.yi;
    SF_HIP(launch_spmv(sa, dtype, st));
  }
  if (nrhs > 1) {
    SF_HIP(launch_unpack(w.xi, dtype, int32_t(s->n), nrhs, X, ldx, kb, st));
    if (Y) SF_HIP(launch_unpack(w.yi, dtype, int32_t(s->m), nrhs, Y, ldy, kb, st));
  }
  return SF_OK;
}

sf_status check_ts_args(sf_schedule_s* s, sf_dtype dt, const void* Lv, const void* Av, const void* B,
                        int ldb, int nrhs, void* X, int ldx, void* Y, int ldy) {
  if (!s) return SF_ERR_ARG;
  if (s->kind != SF_TRSV_SPMV) return SF_ERR_ARG;
  if (dt != SF_F64 && dt != SF_F32) return SF_ERR_ARG;
  if (nrhs < 1 || nrhs > 64) return SF_ERR_ARG;
  // size limits of the multi-RHS executors, checked before anything else
  // touches the buffers: interleaved blocks are addressed with 32-bit
  // offsets (n * block width), column chains index work as item * columns
  if (nrhs > 1 && !s->no_fusion && column_chains(s, nrhs)) {
    const size_t items = s->chunked ? s->citem_ptr.size() : s->item_ptr.size();
    if (int64_t(items) * nrhs > int64_t(INT32_MAX) / 2) return SF_ERR_UNSUPPORTED;
  } else if (nrhs > 1 && int64_t(s->n) * solve_kb(s, nrhs) > int64_t(INT32_MAX)) {
    return SF_ERR_UNSUPPORTED;
  }
  if (s->n > 0 && (!Lv || !B || !X)) return SF_ERR_ARG;
  if (Y && s->A.nnz() > 0 && !Av) return SF_ERR_ARG;
  if (ldb < s->n || ldx < s->n || (Y && ldy < s->m)) return SF_ERR_SHAPE;
  if (B == X && s->n > 0) return SF_ERR_ARG;
  return SF_OK;
}

// No unknowns: x is empty and y = A x is zero in every row of A.
sf_status empty_solve(sf_schedule_s* s, sf_dtype dt, void* Y, int32_t ldy, int32_t nrhs, void* stream) {
  if (!Y || s->m == 0) return SF_OK;
  return hip_status(launch_zero_cols(Y, int32_t(s->m), ldy, nrhs, dt == SF_F64 ? 0 : 1,
                                     static_cast<hipStream_t>(stream)));
}

// Kernel combinations 1 and 2 of Table 2 (see k_pair).  mode 2: B = x,
// Y = y (may be null), Z = z; mode 1: B = b, Y = x, Z = z.
sf_status exec_pair(sf_schedule_s* s, sf_dtype dt, int mode, const void* Lv, const void* Av, const void* B,
                    void* Y, void* Z, bool fused, hipStream_t st) {
  const int dtype = dt == SF_F64 ? 0 : 1;
  const DeviceBuffers& d = s->dev;
  if (!fused) {
    // unfused baseline: the first kernel in full, then the level-set solve
    void* mid = Y;  // y (combination 2) or x (combination 1): the second kernel's input
    if (mode == 2) {
      // the SpMV items of the level plan, entry-streamed, x read through the caches
      TsArgs sa = ts_args(s, Lv, Av, nullptr, int32_t(s->n), 1, const_cast<void*>(B), int32_t(s->n), mid,
                          int32_t(s->m));
      sa.item_list = d.spmv_items;
      sa.n_work = int32_t(s->spmv_items.size());
      if (sa.n_work > 0) SF_HIP(launch_spmv_items(sa, dtype, st));
    } else {
      sf_status r = exec_ts_unfused(s, dt, Lv, nullptr, B, int32_t(s->n), 1, mid, int32_t(s->n), nullptr, 0, st);
      if (r != SF_OK) return r;
    }
    return exec_ts_unfused(s, dt, Lv, nullptr, mid, int32_t(s->n), 1, Z, int32_t(s->n), nullptr, 0, st);
  }
  // k_pair: mode 2 writes z into X and y into Y; mode 1 writes x into X and z into Y
  TsArgs a = ts_args(s, Lv, Av, B, int32_t(s->n), 1, mode == 2 ? Z : Y, int32_t(s->n), nullptr, 0);
  // the region plan's SpTRSV regions (k_pair_region) on request (coarsen 3)
  // or without a coarsened plan: the pair's second sweep (y_i staged per
  // row, or the z regions after the x regions) measured slower on regions
  // than on coarsened items (3D 7-point 128^3: 0.465 / 0.493 ms against
  // 0.440 / 0.468 ms for combinations 2 / 1)
  if (s->regioned && !s->rtrsv_items.empty() && (s->coarsen == 3 || !s->chunked)) {
    a.order = d.rorder;
    a.qrng = d.rqrng;
    a.item_ptr = d.ritem_ptr;
    a.item_list = d.rtrsv_items;
    a.n_work = int32_t(s->rtrsv_items.size());
    a.Y = mode == 2 ? Y : Z;
    sf_status r = next_epoch(s, st, a.ls);
    if (r != SF_OK) return r;
    const RegionArgs ra = region_args(s);
    const int per_cu = std::min(std::max(1, occupancy_region(ra, dtype)), std::max(1, s->waves_per_cu / 2));
    const int grid = std::max(std::max(1, device_cus()) * per_cu, kStreams);
    Timer tm(s, st);
    SF_HIP(launch_fill_pending(Z, size_t(s->n), dtype, st));
    if (mode == 1) SF_HIP(launch_fill_pending(Y, size_t(s->n), dtype, st));
    return hip_status(launch_pair_region(a, ra, dtype, mode, grid, st));
  }
  if (s->chunked) {
    a.order = d.corder;
    a.qrng = d.cqrng;
    a.item_ptr = d.citem_ptr;
    a.item_list = d.ctrsv_items;
    a.n_work = int32_t(s->ctrsv_items.size());
    a.lloc = d.clloc;
    a.eloc = d.celoc;
  } else {
    a.item_list = d.trsv_items;
    a.n_work = int32_t(s->trsv_items.size());
  }
  a.Y = mode == 2 ? Y : Z;
  a.kb = 1;
  a.nblk = 1;
  sf_status r = next_epoch(s, st, a.ls);
  if (r != SF_OK) return r;
  const int grid = persistent_grid(s, occupancy_pair(dtype, mode));
  Timer tm(s, st);
  SF_HIP(launch_fill_pending(Z, size_t(s->n), dtype, st));
  if (mode == 1) SF_HIP(launch_fill_pending(Y, size_t(s->n), dtype, st));
  return hip_status(launch_pair(a, dtype, mode, grid, st));
}

sf_status check_pair_args(sf_schedule_s* s, sf_dtype dt, int mode, const void* Lv, const void* Av, const void* B,
                          const void* Y, const void* Z, bool fused) {
  if (!s || s->kind != SF_TRSV_SPMV) return SF_ERR_ARG;
  if (dt != SF_F64 && dt != SF_F32) return SF_ERR_ARG;
  if (s->n == 0) return SF_OK;
  if (!Lv || !B || !Z) return SF_ERR_ARG;
  if (mode == 2) {
    if (s->m != s->n) return SF_ERR_SHAPE;  // row r of A x feeds row r of the solve
    if (!Av) return SF_ERR_ARG;
    if (!fused && !Y) return SF_ERR_ARG;  // the unfused baseline stores y between its kernels
  } else if (!Y) {
    return SF_ERR_ARG;
  }
  if (B == Z || (Y && (Y == Z || Y == B))) return SF_ERR_ARG;
  return SF_OK;
}

sf_status pair_entry(sf_schedule s, sf_dtype dtype, int mode, const void* L_val, const void* A_val, const void* B,
                     void* Y, void* Z, bool fused, void* stream) {
  sf_status r = check_pair_args(s, dtype, mode, L_val, A_val, B, Y, Z, fused);
  if (r != SF_OK || s->n == 0) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  r = upload(s, st);
  if (r != SF_OK) return r;
  return exec_pair(s, dtype, mode, L_val, A_val, B, Y, Z, fused && !s->no_fusion, st);
}

// Preconditioner apply z = L^{-T} L^{-1} r.  Fused: forward and backward
// items in one launch -- on both region plans when the schedule has them
// (k_precond_region), else level or coarsened items (k_precond); unfused:
// the forward solve as its own launch, then a backward-only launch.
sf_status exec_precond(sf_schedule_s* s, sf_dtype dt, const void* Lv, const void* R, void* W, void* Z, bool fused,
                       hipStream_t st) {
  const int dtype = dt == SF_F64 ? 0 : 1;
  const DeviceBuffers& d = s->dev;
  PrecondArgs a{};
  a.n = int32_t(s->n);
  a.Lci = d.Lci;
  a.LTrp = d.LTrp;
  a.LTci = d.LTci;
  a.LTmap = d.LTmap;
  a.Lv = Lv;
  a.R = R;
  a.W = W;
  a.Z = Z;
  if (s->bchunked) {
    a.border = d.bcorder;
    a.bitem_ptr = d.bcitem_ptr;
    a.n_bwd = int32_t(s->bcitem_ptr.size() - 1);
    a.blloc = d.bclloc;
    a.beloc = d.bceloc;
  } else {
    a.border = d.border;
    a.bitem_ptr = d.bitem_ptr;
    a.n_bwd = int32_t(s->bitem_ptr.size() - 1);
  }
  if (fused && s->regioned && s->bregioned && !s->rtrsv_items.empty() && s->precond_regions) {
    // both solves on their region plans, in one launch
    a.forder = d.rorder;
    a.fqrng = d.rqrng;
    a.fitem_ptr = d.ritem_ptr;
    a.fitems = d.rtrsv_items;
    a.n_fwd = int32_t(s->rtrsv_items.size());
    a.border = d.brorder;
    a.bitem_ptr = d.britem_ptr;
    a.n_bwd = int32_t(s->britem_ptr.size() - 1);
    sf_status r = next_epoch(s, st, a.ls);
    if (r != SF_OK) return r;
    const RegionArgs rf = region_args(s), rb = back_region_args(s);
    const int per_cu =
        std::min(std::max(1, occupancy_precond_region(rf, rb, dtype)), std::max(1, s->waves_per_cu / 2));
    const int grid = std::max(std::max(1, device_cus()) * per_cu, kStreams);
    Timer tm(s, st);
    SF_HIP(launch_fill_pending(W, size_t(s->n), dtype, st));
    SF_HIP(launch_fill_pending(Z, size_t(s->n), dtype, st));
    return hip_status(launch_precond_region(a, rf, rb, dtype, grid, st));
  }
  if (fused) {
    if (s->chunked) {
      a.forder = d.corder;
      a.fqrng = d.cqrng;
      a.fitem_ptr = d.citem_ptr;
      a.fitems = d.ctrsv_items;
      a.n_fwd = int32_t(s->ctrsv_items.size());
      a.flloc = d.clloc;
      a.feloc = d.celoc;
    } else {
      a.forder = d.order;
      a.fqrng = d.qrng;
      a.fitem_ptr = d.item_ptr;
      a.fitems = d.trsv_items;
      a.n_fwd = int32_t(s->trsv_items.size());
    }
  } else {
    sf_status r = exec_ts_fused(s, dt, Lv, nullptr, R, int32_t(s->n), 1, W, int32_t(s->n), nullptr, 0, st);
    if (r != SF_OK) return r;
  }
  sf_status r = next_epoch(s, st, a.ls);
  if (r != SF_OK) return r;
  const int grid = persistent_grid(s, occupancy_precond(dtype));
  Timer tm(s, st);
  if (fused) SF_HIP(launch_fill_pending(W, size_t(s->n), dtype, st));
  SF_HIP(launch_fill_pending(Z, size_t(s->n), dtype, st));
  return hip_status(launch_precond(a, dtype, grid, st));
}

sf_status precond_entry(sf_schedule s, sf_dtype dtype, const void* L_val, const void* R, void* W, void* Z,
                        bool fused, void* stream) {
  if (!s || s->kind != SF_TRSV_SPMV || !s->has_back) return SF_ERR_ARG;
  if (dtype != SF_F64 && dtype != SF_F32) return SF_ERR_ARG;
  if (s->n == 0) return SF_OK;
  if (!L_val || !R || !W || !Z || R == W || R == Z || W == Z) return SF_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  sf_status r = upload(s, st);
  if (r != SF_OK) return r;
  return exec_precond(s, dtype, L_val, R, W, Z, fused && !s->no_fusion, st);
}

}  // namespace

extern "C" {

sf_status sf_exec_ic_apply(sf_schedule s, sf_dtype dtype, const void* L_val, const void* R, void* W, void* Z,
                           void* stream) {
  return enqueued(s, stream, precond_entry(s, dtype, L_val, R, W, Z, true, stream));
}

sf_status sf_exec_unfused_ic_apply(sf_schedule s, sf_dtype dtype, const void* L_val, const void* R, void* W,
                                   void* Z, void* stream) {
  return enqueued(s, stream, precond_entry(s, dtype, L_val, R, W, Z, false, stream));
}

sf_status sf_exec_spmv_trsv(sf_schedule s, sf_dtype dtype, const void* A_val, const void* L_val, const void* X,
                            void* Y, void* Z, void* stream) {
  return enqueued(s, stream, pair_entry(s, dtype, 2, L_val, A_val, X, Y, Z, true, stream));
}

sf_status sf_exec_unfused_spmv_trsv(sf_schedule s, sf_dtype dtype, const void* A_val, const void* L_val,
                                    const void* X, void* Y, void* Z, void* stream) {
  return enqueued(s, stream, pair_entry(s, dtype, 2, L_val, A_val, X, Y, Z, false, stream));
}

sf_status sf_exec_trsv_trsv(sf_schedule s, sf_dtype dtype, const void* L_val, const void* B, void* X, void* Z,
                            void* stream) {
  return enqueued(s, stream, pair_entry(s, dtype, 1, L_val, nullptr, B, X, Z, true, stream));
}

sf_status sf_exec_unfused_trsv_trsv(sf_schedule s, sf_dtype dtype, const void* L_val, const void* B, void* X,
                                    void* Z, void* stream) {
  return enqueued(s, stream, pair_entry(s, dtype, 1, L_val, nullptr, B, X, Z, false, stream));
}

sf_status sf_device_probe(int32_t what, sf_probe_result* out, void* stream) {
  if (!out) return SF_ERR_ARG;
  const int32_t all = SF_PROBE_COPY | SF_PROBE_HOP | SF_PROBE_GATHER;
  if (what == 0) what = all;
  if (what & ~all) return SF_ERR_ARG;
  *out = sf_probe_result{-1.0, -1.0, -1.0, -1.0};
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int cus = std::max(1, device_cus());
  if (what & SF_PROBE_COPY) SF_HIP(probe_copy(cus, st, &out->copy_GBps));
  if (what & SF_PROBE_HOP) SF_HIP(probe_hop(st, &out->hop_us_same_xcd, &out->hop_us_cross_xcd));
  if (what & SF_PROBE_GATHER) SF_HIP(probe_gather(cus, st, &out->gathers_per_s));
  return SF_OK;
}

const char* sf_version(void) { return "sparsefusion-mi355x 0.1 (gfx950)"; }

const char* sf_status_str(sf_status st) {
  switch (st) {
    case SF_OK: return "ok";
    case SF_ERR_ARG: return "invalid argument";
    case SF_ERR_CSR: return "malformed CSR (row pointers, column range, order or duplicates)";
    case SF_ERR_NOT_LOWER: return "L has an entry above the diagonal";
    case SF_ERR_ZERO_DIAG: return "a row of L has no stored diagonal";
    case SF_ERR_SHAPE: return "dimension mismatch";
    case SF_ERR_NOT_SPD: return "incomplete Cholesky breakdown (non-positive pivot)";
    case SF_ERR_HIP: return "HIP runtime or launch error";
    case SF_ERR_OOM: return "out of memory";
    case SF_ERR_TIMEOUT: return "executor watchdog: a dependence never became ready";
    case SF_ERR_UNSUPPORTED: return "unsupported in this build";
  }
  return "unknown status";
}

// Default residency of the factorisation executors (SpIC0 / SpILU0 ->
// SpTRSV): the smallest power of two from 4 to 32 waves per CU that holds
// the mean work items of one wavefront of the DAG per CU at once.  Their
// items are single batches whose cost is one dependency chain, so waves
// beyond a level's items only poll; fewer leave a level's items queued.
// Taken for the 256 CUs of an MI355X (no device query at inspection).
int32_t factor_waves(const sf_schedule_s* s) {
  constexpr double kCus = 256.0;
  const double items = double(s->item_ptr.empty() ? 0 : s->item_ptr.size() - 1);
  const double per_cu = items / double(std::max(1, s->depth)) / kCus;
  int32_t w = 4;
  while (w < 32 && double(w) < per_cu) w *= 2;
  return w;
}

sf_status sf_inspect(const sf_csr_pattern* L, const sf_csr_pattern* A, const sf_inspect_opts* opts,
                     sf_schedule* out) {
  if (!out) return SF_ERR_ARG;
  *out = nullptr;
  sf_inspect_opts o{};
  if (opts) o = *opts;
  if (o.kind != SF_TRSV_SPMV && o.kind != SF_IC0_TRSV && o.kind != SF_ILU0_TRSV) return SF_ERR_ARG;
  if (o.lanes_per_row != 0 && !pow2_in(o.lanes_per_row, 2, 64)) return SF_ERR_ARG;
  if (o.rows_per_item < 0 || o.max_item_nnz < 0) return SF_ERR_ARG;
  if (o.rhs_block != 0 && !pow2_in(o.rhs_block, 2, 64)) return SF_ERR_ARG;
  if (o.coarsen < 0 || o.coarsen > 3) return SF_ERR_ARG;
  if (o.kind == SF_TRSV_SPMV && !A) return SF_ERR_ARG;
  const auto t0 = std::chrono::steady_clock::now();
  sf_status st = o.kind == SF_ILU0_TRSV ? sf::check_square_diag(L) : sf::check_lower(L);
  if (st != SF_OK) return st;
  if (o.kind == SF_TRSV_SPMV) {
    st = sf::check_general(A, L->nrows);
    if (st != SF_OK) return st;
  }
  sf_schedule_s* s = new (std::nothrow) sf_schedule_s();
  if (!s) return SF_ERR_OOM;
  try {
    st = sf::build_schedule(s, L, A, o);
  } catch (const std::bad_alloc&) {
    st = SF_ERR_OOM;
  }
  if (st == SF_OK && o.validate && sf::validate_forward(s) != 0) st = SF_ERR_ARG;
  if (st != SF_OK) {
    delete s;
    return st;
  }
  s->claim_streams = kStreams;
  if (o.kind != SF_TRSV_SPMV) s->waves_per_cu = factor_waves(s);
  s->inspect_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = s;
  return SF_OK;
}

sf_status sf_schedule_free(sf_schedule s) {
  if (!s) return SF_OK;
  if (s->trace) {
    wait_done(s);
    hipFree(s->trace);
  }
  free_device(s);
  delete s;
  return SF_OK;
}

sf_status sf_schedule_info(sf_schedule s, sf_schedule_stats* st) {
  if (!s || !st) return SF_ERR_ARG;
  st->n = s->n;
  st->m = s->m;
  st->nnz_l = s->L.nnz();
  st->nnz_a = s->A.nnz();
  st->depth = s->depth;
  st->joint_depth = s->joint_depth;
  st->back_depth = s->back_depth;
  st->n_items = int32_t(s->regioned ? s->ritem_ptr.size() : s->chunked ? s->citem_ptr.size() : s->item_ptr.size()) - 1;
  st->n_back_items = s->has_back
                        ? int32_t((s->bregioned ? s->britem_ptr : s->bchunked ? s->bcitem_ptr : s->bitem_ptr).size()) - 1
                        : 0;
  st->max_level_width = s->max_level_width;
  st->lanes_per_row = s->lanes_trsv;
  st->lanes_per_spmv = s->lanes_spmv;
  st->reuse_ratio = s->reuse;
  st->inspect_seconds = s->inspect_seconds;
  st->coarsened = s->chunked ? 1 : 0;
  st->chunk_items = int32_t(s->ctrsv_items.size());
  st->chunk_chain = s->chunk_chain;
  st->max_local_depth = s->max_local_depth;
  st->est_level_us = s->est_level_us;
  st->est_chunk_us = s->est_chunk_us;
  st->back_coarsened = s->bchunked ? 1 : 0;
  st->back_chunk_chain = s->back_chunk_chain;
  st->est_back_level_us = s->est_back_level_us;
  st->est_back_chunk_us = s->est_back_chunk_us;
  return SF_OK;
}

sf_status sf_schedule_export(sf_schedule s, int32_t* level, int32_t* order, int32_t* item_ptr) {
  if (!s) return SF_ERR_ARG;
  if (level) std::copy(s->level.begin(), s->level.end(), level);
  if (order) {
    if (s->kind == SF_TRSV_SPMV) {
      const std::vector<int32_t>& o = s->regioned ? s->rorder : s->chunked ? s->corder : s->order;
      std::copy(o.begin(), o.end(), order);
    } else {
      // each row contributes its SpIC0 iteration (id i) then its SpTRSV one (id n + i)
      for (size_t q = 0; q < s->order.size(); ++q) {
        order[2 * q] = s->order[q];
        order[2 * q + 1] = int32_t(s->n) + s->order[q];
      }
    }
  }
  if (item_ptr) {
    const int mult = s->kind == SF_TRSV_SPMV ? 1 : 2;
    const std::vector<int32_t>& ip = s->regioned ? s->ritem_ptr : s->chunked ? s->citem_ptr : s->item_ptr;
    for (size_t t = 0; t < ip.size(); ++t) item_ptr[t] = mult * ip[t];
  }
  return SF_OK;
}

sf_status sf_schedule_export_local(sf_schedule s, uint8_t* local_level, uint8_t* entry_slot) {
  if (!s) return SF_ERR_ARG;
  const size_t npos = s->kind == SF_TRSV_SPMV ? size_t(s->n + s->m) : size_t(2 * s->n);
  if (local_level) {
    if (s->regioned) std::copy(s->rlloc.begin(), s->rlloc.end(), local_level);
    else if (s->chunked) std::copy(s->clloc.begin(), s->clloc.end(), local_level);
    else std::fill(local_level, local_level + npos, uint8_t(0));
  }
  if (entry_slot) {  // regions address their columns with 16-bit codes: reported as 0xFF
    if (s->chunked && !s->regioned) std::copy(s->celoc.begin(), s->celoc.end(), entry_slot);
    else std::fill(entry_slot, entry_slot + size_t(s->L.nnz()), uint8_t(0xFF));
  }
  return SF_OK;
}

sf_status sf_schedule_export_backward(sf_schedule s, int32_t* rlevel, int32_t* order, int32_t* item_ptr) {
  if (!s || !s->has_back) return SF_ERR_ARG;
  const std::vector<int32_t>& o = s->bregioned ? s->brorder : s->bchunked ? s->bcorder : s->border;
  const std::vector<int32_t>& ip = s->bregioned ? s->britem_ptr : s->bchunked ? s->bcitem_ptr : s->bitem_ptr;
  if (rlevel) std::copy(s->rlevel.begin(), s->rlevel.end(), rlevel);
  if (order) std::copy(o.begin(), o.end(), order);
  if (item_ptr) std::copy(ip.begin(), ip.end(), item_ptr);
  return SF_OK;
}

sf_status sf_schedule_export_backward_local(sf_schedule s, uint8_t* local_level, uint8_t* entry_slot) {
  if (!s || !s->has_back) return SF_ERR_ARG;
  if (local_level) {
    if (s->bregioned) std::copy(s->brlloc.begin(), s->brlloc.end(), local_level);
    else if (s->bchunked) std::copy(s->bclloc.begin(), s->bclloc.end(), local_level);
    else std::fill(local_level, local_level + size_t(s->n), uint8_t(0));
  }
  if (entry_slot) {
    if (s->bchunked && !s->bregioned) std::copy(s->bceloc.begin(), s->bceloc.end(), entry_slot);
    else std::fill(entry_slot, entry_slot + size_t(s->LT.nnz()), uint8_t(0xFF));
  }
  return SF_OK;
}

sf_status sf_exec_trsv_spmv(sf_schedule s, sf_dtype dtype, const void* L_val, const void* A_val,
                            const void* B, int32_t ldb, int32_t nrhs, void* X, int32_t ldx, void* Y,
                            int32_t ldy, void* stream) {
  sf_status r = check_ts_args(s, dtype, L_val, A_val, B, ldb, nrhs, X, ldx, Y, ldy);
  if (r != SF_OK) return r;
  if (s->n == 0) return empty_solve(s, dtype, Y, ldy, nrhs, stream);
  hipStream_t st = static_cast<hipStream_t>(stream);
  r = upload(s, st);
  if (r != SF_OK) return r;
  if (s->no_fusion) return enqueued(s, stream, exec_ts_unfused(s, dtype, L_val, A_val, B, ldb, nrhs, X, ldx, Y, ldy, st));
  return enqueued(s, stream, exec_ts_fused(s, dtype, L_val, A_val, B, ldb, nrhs, X, ldx, Y, ldy, st));
}

// ---- static plans: the paper's fused partitioning (MSP) and the fused
// wavefront baseline, run by one cooperative launch with a grid barrier
// between s-partitions (static_plan.cpp, k_static)

sf_status static_dev(sf_schedule_s* s, StaticPlan& P, hipStream_t st) {
  if (P.dev) return SF_OK;
  const size_t N = P.order.size();
  const size_t parts[5] = {N, 2 * N, P.s_ptr.size(), P.w_batch.size(), P.batch_ptr.size()};
  size_t total = 0;
  for (size_t c : parts) total += align256(std::max<size_t>(c, 1) * 4);
  SF_HIP(hipStreamSynchronize(st));
  SF_HIP(hipMalloc(&P.dev, total));
  char* b = static_cast<char*>(P.dev);
  int32_t** dst[5] = {&P.d_order, &P.d_qrng, &P.d_s_ptr, &P.d_w_batch, &P.d_batch_ptr};
  const std::vector<int32_t>* src[5] = {&P.order, &P.qrng, &P.s_ptr, &P.w_batch, &P.batch_ptr};
  for (int k = 0; k < 5; ++k) {
    *dst[k] = reinterpret_cast<int32_t*>(b);
    if (!src[k]->empty()) SF_HIP(hipMemcpy(b, src[k]->data(), src[k]->size() * 4, hipMemcpyHostToDevice));
    b += align256(std::max<size_t>(parts[k], 1) * 4);
  }
  (void)s;
  return SF_OK;
}

sf_status sf_schedule_static_info(sf_schedule s, int32_t plan, int32_t* n_spart, int32_t* n_wpart,
                                  int32_t* n_batches, int32_t* merged, int32_t* slack_moved) {
  if (!s || s->kind != SF_TRSV_SPMV || (plan != SF_STATIC_MSP && plan != SF_STATIC_WAVEFRONT)) return SF_ERR_ARG;
  sf_status r = build_static(s, plan);
  if (r != SF_OK) return r;
  const StaticPlan& P = static_plan(s, plan);
  if (n_spart) *n_spart = int32_t(P.s_ptr.size()) - 1;
  if (n_wpart) *n_wpart = int32_t(P.w_ptr.size()) - 1;
  if (n_batches) *n_batches = int32_t(P.batch_ptr.size()) - 1;
  if (merged) *merged = P.merged;
  if (slack_moved) *slack_moved = P.slack_moved;
  return SF_OK;
}

sf_status sf_schedule_export_static(sf_schedule s, int32_t plan, int32_t* s_ptr, int32_t* w_ptr, int32_t* order) {
  if (!s || s->kind != SF_TRSV_SPMV || (plan != SF_STATIC_MSP && plan != SF_STATIC_WAVEFRONT)) return SF_ERR_ARG;
  sf_status r = build_static(s, plan);
  if (r != SF_OK) return r;
  const StaticPlan& P = static_plan(s, plan);
  if (s_ptr) std::copy(P.s_ptr.begin(), P.s_ptr.end(), s_ptr);
  if (w_ptr) std::copy(P.w_ptr.begin(), P.w_ptr.end(), w_ptr);
  if (order) std::copy(P.order.begin(), P.order.end(), order);
  return SF_OK;
}

sf_status sf_exec_static_trsv_spmv(sf_schedule s, int32_t plan, sf_dtype dtype, const void* L_val,
                                   const void* A_val, const void* B, void* X, void* Y, void* stream) {
  if (!s || s->kind != SF_TRSV_SPMV || (plan != SF_STATIC_MSP && plan != SF_STATIC_WAVEFRONT)) return SF_ERR_ARG;
  if (dtype != SF_F64 && dtype != SF_F32) return SF_ERR_ARG;
  if (s->m > 0 && (!Y || (s->A.nnz() > 0 && !A_val))) return SF_ERR_ARG;
  if (s->n == 0) return empty_solve(s, dtype, Y, int32_t(s->m), 1, stream);
  if (!L_val || !B || !X || B == X) return SF_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  sf_status r = upload(s, st);
  if (r == SF_OK) r = build_static(s, plan);
  StaticPlan& P = static_plan(s, plan);
  if (r == SF_OK) r = static_dev(s, P, st);
  if (r != SF_OK) return r;
  const int dt = dtype == SF_F64 ? 0 : 1;
  StaticArgs a{};
  a.ts = ts_args(s, L_val, A_val, B, int32_t(s->n), 1, X, int32_t(s->n), Y, int32_t(std::max<int64_t>(s->m, 1)));
  a.ts.order = P.d_order;
  a.ts.qrng = P.d_qrng;
  a.ts.item_ptr = nullptr;
  a.ts.item_list = nullptr;
  a.ts.kb = 1;
  a.ts.nblk = 1;
  a.s_ptr = P.d_s_ptr;
  a.w_batch = P.d_w_batch;
  a.batch_ptr = P.d_batch_ptr;
  a.nb = int32_t(P.s_ptr.size()) - 1;
  r = next_epoch(s, st, a.ts.ls);
  if (r != SF_OK) return r;
  const int cus = std::max(1, device_cus());
  const int grid = cus * std::min(occupancy_static(dt), std::max(1, s->levelset_waves_per_cu * 64 / kBlockThreads));
  Timer tm(s, st);
  return enqueued(s, stream, hip_status(launch_static(a, dt, grid, st)));
}

sf_status sf_exec_unfused_trsv_spmv(sf_schedule s, sf_dtype dtype, const void* L_val, const void* A_val,
                                    const void* B, int32_t ldb, int32_t nrhs, void* X, int32_t ldx,
                                    void* Y, int32_t ldy, void* stream) {
  sf_status r = check_ts_args(s, dtype, L_val, A_val, B, ldb, nrhs, X, ldx, Y, ldy);
  if (r != SF_OK) return r;
  if (s->n == 0) return empty_solve(s, dtype, Y, ldy, nrhs, stream);
  hipStream_t st = static_cast<hipStream_t>(stream);
  r = upload(s, st);
  if (r != SF_OK) return r;
  return enqueued(s, stream, exec_ts_unfused(s, dtype, L_val, A_val, B, ldb, nrhs, X, ldx, Y, ldy, st));
}

static sf_status ic0_common(sf_schedule s, sf_dtype dtype, const void* A_lower_val, void* L_val,
                            const void* B, int32_t ldb, int32_t nrhs, void* X, int32_t ldx,
                            int32_t* d_info, bool fused, void* stream) {
  if (!s || s->kind != SF_IC0_TRSV) return SF_ERR_ARG;
  if (dtype != SF_F64) return SF_ERR_UNSUPPORTED;
  if (nrhs != 1) return SF_ERR_UNSUPPORTED;
  if (s->n > 0 && (!A_lower_val || !L_val)) return SF_ERR_ARG;
  if (ldb < s->n || ldx < s->n) return SF_ERR_SHAPE;
  const bool solve = B != nullptr;
  if (solve && !X) return SF_ERR_ARG;
  if (s->n == 0) return SF_OK;
  if (s->max_offdiag > s->lanes_trsv) return SF_ERR_UNSUPPORTED;  // one lane per entry of a row
  hipStream_t st = static_cast<hipStream_t>(stream);
  sf_status r = upload(s, st);
  if (r != SF_OK) return r;
  const DeviceBuffers& d = s->dev;
  Ic0Args a{};
  a.n = int32_t(s->n);
  a.Lrp = d.Lrp;
  a.Lci = d.Lci;
  a.Aval = static_cast<const double*>(A_lower_val);
  a.Lval = static_cast<double*>(L_val);
  a.B = static_cast<const double*>(B);
  a.X = static_cast<double*>(X);
  a.pair_ptr = d.pair_ptr;
  a.pair_u = d.pair_u;
  a.pair_q = d.pair_q;
  a.qrng = d.qrng;
  a.prng = d.prng;
  a.piv = d.piv;
  a.order = d.order;
  a.item_ptr = d.item_ptr;
  a.d_info = d_info;
  a.factor = 1;
  const int cus = std::max(1, device_cus());
  Timer tm(s, st);
  if (fused) {
    r = next_epoch(s, st, a.ls);
    if (r != SF_OK) return r;
    a.item_list = nullptr;
    a.n_work = int32_t(s->item_ptr.size() - 1);
    a.solve = solve ? 1 : 0;
    const int grid = persistent_grid(s, occupancy_ic0(s->lanes_trsv, 0));
    a.trace = s->trace;
    a.rtrace = a.trace && s->trace_level == 1 ? a.trace + s->trace_items * kTraceItemWords : nullptr;
    a.cached = s->ic0_cached;
    if (a.trace) SF_HIP(launch_fill_u64(a.trace, int32_t(trace_words(s)), st));  // counts start at 0
    // every factor value and x_i is its own readiness flag
    SF_HIP(launch_fill_pending(L_val, size_t(s->L.nnz()), 0, st));
    if (solve) SF_HIP(launch_fill_pending(X, size_t(s->n), 0, st));
    return hip_status(launch_ic0_fused(a, s->lanes_trsv, grid, st));
  }
  // unfused: level-set factorisation, then a level-set solve
  r = next_epoch(s, st, a.ls);
  if (r != SF_OK) return r;
  a.item_list = d.lvl_items;
  a.n_work = int32_t(s->lvl_items.size());
  a.lvl_item_ptr = d.lvl_item_ptr;
  a.depth = s->depth;
  a.solve = 0;
  int grid = cus * std::min(occupancy_ic0(s->lanes_trsv, 1), std::max(1, s->levelset_waves_per_cu * 64 / kBlockThreads));
  SF_HIP(launch_ic0_levelset(a, s->lanes_trsv, grid, st));
  if (!solve) return SF_OK;
  LevelArgs la{};
  la.ts.n = int32_t(s->n);
  la.ts.Lrp = d.Lrp;
  la.ts.Lci = d.Lci;
  la.ts.Lv = L_val;
  la.ts.B = B;
  la.ts.ldb = ldb;
  la.ts.X = X;
  la.ts.ldx = ldx;
  la.ts.nrhs = 1;
  la.ts.kb = 1;
  la.ts.nblk = 1;
  la.ts.order = d.order;
  la.ts.qrng = d.qrng;
  la.ts.item_ptr = d.item_ptr;
  la.ts.item_list = d.lvl_items;
  la.ts.n_work = a.n_work;
  la.lvl_item_ptr = d.lvl_item_ptr;
  la.depth = s->depth;
  r = next_epoch(s, st, la.ts.ls);
  if (r != SF_OK) return r;
  grid = cus * std::min(occupancy_trsv_levelset(0, 1), std::max(1, s->levelset_waves_per_cu * 64 / kBlockThreads));
  return hip_status(launch_trsv_levelset(la, 0, grid, st));
}

// Fused SpILU0 -> unit-lower SpTRSV (k_ilu.hip); unfused: level-set
// factorisation, then a level-set solve reading the factor.
static sf_status ilu0_common(sf_schedule s, sf_dtype dtype, const void* A_val, void* LU_val, const void* X,
                             void* Y, int32_t* d_info, bool fused, void* stream) {
  if (!s || s->kind != SF_ILU0_TRSV) return SF_ERR_ARG;
  if (dtype != SF_F64) return SF_ERR_UNSUPPORTED;
  const bool solve = X != nullptr;
  if (s->n > 0 && (!A_val || !LU_val)) return SF_ERR_ARG;
  if (solve && (!Y || X == Y)) return SF_ERR_ARG;
  if (s->n == 0) return SF_OK;
  if (s->max_offdiag + 1 > s->lanes_trsv) return SF_ERR_UNSUPPORTED;  // one lane per stored entry
  hipStream_t st = static_cast<hipStream_t>(stream);
  sf_status r = upload(s, st);
  if (r != SF_OK) return r;
  const DeviceBuffers& d = s->dev;
  Ic0Args a{};
  a.n = int32_t(s->n);
  a.Lrp = d.Lrp;
  a.Lci = d.Lci;
  a.Aval = static_cast<const double*>(A_val);
  a.Lval = static_cast<double*>(LU_val);
  a.B = static_cast<const double*>(X);
  a.X = static_cast<double*>(Y);
  a.pair_ptr = d.pair_ptr;
  a.pair_u = d.pair_u;
  a.pair_q = d.pair_q;
  a.dpos = d.dpos;
  a.order = d.order;
  a.item_ptr = d.item_ptr;
  a.d_info = d_info;
  a.factor = 1;
  const int cus = std::max(1, device_cus());
  Timer tm(s, st);
  if (fused) {
    r = next_epoch(s, st, a.ls);
    if (r != SF_OK) return r;
    a.item_list = nullptr;
    a.n_work = int32_t(s->item_ptr.size() - 1);
    a.solve = solve ? 1 : 0;
    const int grid = persistent_grid(s, occupancy_ilu0(s->lanes_trsv, 0));
    // every factor value and y_i is its own readiness flag
    SF_HIP(launch_fill_pending(LU_val, size_t(s->L.nnz()), 0, st));
    if (solve) SF_HIP(launch_fill_pending(Y, size_t(s->n), 0, st));
    return hip_status(launch_ilu0_fused(a, s->lanes_trsv, grid, st));
  }
  a.item_list = d.lvl_items;
  a.n_work = int32_t(s->lvl_items.size());
  a.lvl_item_ptr = d.lvl_item_ptr;
  a.depth = s->depth;
  const int grid =
      cus * std::min(occupancy_ilu0(s->lanes_trsv, 1), std::max(1, s->levelset_waves_per_cu * 64 / kBlockThreads));
  r = next_epoch(s, st, a.ls);
  if (r != SF_OK) return r;
  a.solve = 0;
  SF_HIP(launch_ilu0_levelset(a, s->lanes_trsv, grid, st));
  if (!solve) return SF_OK;
  r = next_epoch(s, st, a.ls);
  if (r != SF_OK) return r;
  a.factor = 0;
  a.solve = 1;
  a.d_info = nullptr;
  return hip_status(launch_ilu0_levelset(a, s->lanes_trsv, grid, st));
}

sf_status sf_exec_ic0_trsv(sf_schedule s, sf_dtype dtype, const void* A_lower_val, void* L_val,
                           const void* B, int32_t ldb, int32_t nrhs, void* X, int32_t ldx,
                           int32_t* d_info, void* stream) {
  const bool fused = !(s && s->no_fusion);
  return enqueued(s, stream, ic0_common(s, dtype, A_lower_val, L_val, B, ldb, nrhs, X, ldx, d_info, fused, stream));
}

sf_status sf_exec_unfused_ic0_trsv(sf_schedule s, sf_dtype dtype, const void* A_lower_val, void* L_val,
                                   const void* B, int32_t ldb, int32_t nrhs, void* X, int32_t ldx,
                                   int32_t* d_info, void* stream) {
  return enqueued(s, stream, ic0_common(s, dtype, A_lower_val, L_val, B, ldb, nrhs, X, ldx, d_info, false, stream));
}

sf_status sf_exec_ilu0_trsv(sf_schedule s, sf_dtype dtype, const void* A_val, void* LU_val, const void* X,
                            void* Y, int32_t* d_info, void* stream) {
  return enqueued(s, stream, ilu0_common(s, dtype, A_val, LU_val, X, Y, d_info, !(s && s->no_fusion), stream));
}

sf_status sf_exec_unfused_ilu0_trsv(sf_schedule s, sf_dtype dtype, const void* A_val, void* LU_val,
                                    const void* X, void* Y, int32_t* d_info, void* stream) {
  return enqueued(s, stream, ilu0_common(s, dtype, A_val, LU_val, X, Y, d_info, false, stream));
}

size_t sf_backward_workspace_bytes(sf_schedule s, sf_dtype dtype, int32_t nrhs) {
  if (!s) return 0;
  const size_t es = dtype == SF_F64 ? 8 : 4;
  return size_t(std::max<int64_t>(s->n, 1)) * size_t(std::max(nrhs, 1)) * es;
}

}  // extern "C"

namespace {

// The adjoint's launches (sf_backward): x recomputed into `workspace` when
// X is NULL (by the fused forward executor), then the backward executor.
// Makes no allocation once the schedule is resident on the device.
sf_status backward_core(sf_schedule_s* s, sf_dtype dtype, const void* L_val, const void* A_val, const void* X,
                        const void* B, const void* G, void* grad_B, void* grad_L_val, void* workspace,
                        hipStream_t st) {
  const int dt = dtype == SF_F64 ? 0 : 1;
  const void* x = X;
  if (!x) {
    sf_status r = exec_ts_fused(s, dtype, L_val, nullptr, B, int32_t(s->n), 1, workspace, int32_t(s->n), nullptr, 0, st);
    if (r != SF_OK) return r;
    x = workspace;
  }
  const DeviceBuffers& d = s->dev;
  BwdArgs a{};
  a.n = int32_t(s->n);
  a.LTrp = d.LTrp; a.LTci = d.LTci; a.LTmap = d.LTmap;
  a.ATrp = d.ATrp; a.ATci = d.ATci; a.ATmap = d.ATmap;
  a.Lrp = d.Lrp; a.Lci = d.Lci;
  a.Lv = L_val; a.Av = A_val; a.X = x; a.G = G;
  a.lam = grad_B; a.gradL = grad_L_val;
  if (s->bregioned) {
    a.order = d.brorder;
    a.item_ptr = d.britem_ptr;
    a.n_work = int32_t(s->britem_ptr.size() - 1);
    sf_status r = next_epoch(s, st, a.ls);
    if (r != SF_OK) return r;
    const RegionArgs ra = back_region_args(s);
    // blocks of two wavefronts (a computing and a polling one)
    const int per_cu = std::min(std::max(1, occupancy_bwd_region(ra, dt)), std::max(1, s->waves_per_cu / 2));
    const int grid = std::max(std::max(1, device_cus()) * per_cu, kStreams);
    Timer tm(s, st);
    SF_HIP(launch_fill_pending(grad_B, size_t(s->n), dt, st));
    return hip_status(launch_bwd_region(a, ra, dt, grid, st));
  }
  if (s->bchunked) {
    a.order = d.bcorder;
    a.item_ptr = d.bcitem_ptr;
    a.n_work = int32_t(s->bcitem_ptr.size() - 1);
    a.lloc = d.bclloc;
    a.eloc = d.bceloc;
  } else {
    a.order = d.border;
    a.item_ptr = d.bitem_ptr;
    a.n_work = int32_t(s->bitem_ptr.size() - 1);
  }
  sf_status r = next_epoch(s, st, a.ls);
  if (r != SF_OK) return r;
  const int grid = persistent_grid(s, occupancy_bwd(dt, s->lanes_trsv));
  Timer tm(s, st);
  // grad_B is the lambda buffer and its own readiness flag
  SF_HIP(launch_fill_pending(grad_B, size_t(s->n), dt, st));
  return hip_status(launch_bwd(a, dt, std::min(s->lanes_trsv, 32), grid, st));
}

sf_status check_backward_args(sf_schedule_s* s, sf_dtype dtype, const void* L_val, const void* A_val,
                              const void* X, const void* B, const void* G, void* grad_B, void* grad_L_val) {
  if (!s || s->kind != SF_TRSV_SPMV) return SF_ERR_ARG;
  if (!s->has_back) return SF_ERR_ARG;
  if (dtype != SF_F64 && dtype != SF_F32) return SF_ERR_ARG;
  if (s->n == 0) return SF_OK;
  if (!L_val || !G || !grad_B || !grad_L_val || (s->m > 0 && !A_val)) return SF_ERR_ARG;
  if (!X && !B) return SF_ERR_ARG;
  return SF_OK;
}

}  // namespace

extern "C" {

sf_status sf_backward(sf_schedule s, sf_dtype dtype, const void* L_val, const void* A_val, const void* X,
                      const void* B, const void* G, void* grad_B, void* grad_L_val, void* workspace,
                      size_t ws_bytes, void* stream) {
  sf_status r = check_backward_args(s, dtype, L_val, A_val, X, B, G, grad_B, grad_L_val);
  if (r != SF_OK || s->n == 0) return r;
  if (!X && (!workspace || ws_bytes < sf_backward_workspace_bytes(s, dtype, 1))) return SF_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  r = upload(s, st);
  if (r != SF_OK) return r;
  return enqueued(s, stream, backward_core(s, dtype, L_val, A_val, X, B, G, grad_B, grad_L_val, workspace, st));
}

sf_status sf_backward_noalloc(sf_schedule s, sf_dtype dtype, const void* L_val, const void* A_val, const void* X,
                              const void* B, const void* G, void* grad_B, void* grad_L_val, void* stream) {
  sf_status r = check_backward_args(s, dtype, L_val, A_val, X, B, G, grad_B, grad_L_val);
  if (r != SF_OK) return r;
  // the recomputed x must fit the fixed scratch
  if (!X && size_t(s->n) * (dtype == SF_F64 ? 8 : 4) > scratch_bytes()) return SF_ERR_UNSUPPORTED;
  if (s->n == 0) return SF_OK;
  // no allocation here: the schedule's device arrays (and its event) must
  // already be resident on the current device, made by an earlier executor
  // call with this schedule (e.g. the forward pass)
  int cur = -1;
  SF_HIP(hipGetDevice(&cur));
  if (!s->dev.ready || s->dev.device != cur || !s->dev.done) return SF_ERR_ARG;
  void* x = nullptr;
  if (!X) SF_HIP(scratch_device_ptr(&x));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int saved_timing = s->timing;  // timing events would be created per call
  s->timing = 0;
  r = backward_core(s, dtype, L_val, A_val, X, B, G, grad_B, grad_L_val, x, st);
  s->timing = saved_timing;
  return enqueued(s, stream, r);
}

// Refinement workspace, in the interleaved block layout of the solve (a
// plain vector per array for a single right-hand side):
//   r32 | d32 | x ping | x pong | b64 | y64 | max-abs accumulators
// r32 is the FP32 right-hand side of each solve, d32 the single-RHS
// correction (several right-hand sides keep it in the solve's workspace),
// b64 the packed FP64 right-hand sides and y64 the packed product
// (the last two only with several right-hand sides).
struct RefineWs {
  float *r32, *d32;
  double *xa, *xb, *b64, *y64;
  unsigned long long* mx;
  size_t bytes;
};

RefineWs refine_layout(const sf_schedule_s* s, int nrhs, void* base) {
  const int kb = solve_kb(s, nrhs);
  const size_t cols = size_t((nrhs + kb - 1) / kb) * size_t(kb);
  const size_t n = size_t(std::max<int64_t>(s->n, 1)), m = size_t(std::max<int64_t>(s->m, 1));
  const bool multi = kb > 1;
  const size_t sizes[7] = {align256(n * cols * 4), align256(multi ? 256 : n * 4), align256(n * cols * 8),
                           align256(n * cols * 8), align256(multi ? n * cols * 8 : 256),
                           align256(multi ? m * cols * 8 : 256), 2 * 64 * 8};
  char* p = static_cast<char*>(base);
  void* at[7];
  size_t off = 0;
  for (int k = 0; k < 7; ++k) {
    at[k] = p ? p + off : nullptr;
    off += sizes[k];
  }
  RefineWs w{static_cast<float*>(at[0]),  static_cast<float*>(at[1]),  static_cast<double*>(at[2]),
             static_cast<double*>(at[3]), static_cast<double*>(at[4]), static_cast<double*>(at[5]),
             static_cast<unsigned long long*>(at[6]), off};
  return w;
}

// Workspace of the fused refinement (k_rfused.hip): the stage tuples
// (4 floats per row and column at most), then with several right-hand
// sides the packed FP64 right-hand sides, the interleaved x (its own
// readiness flags) and the packed product, all in the block layout of the
// solve; then the max-abs accumulators.
struct FusedRefineWs {
  float* tup;
  double *b64, *xf, *y64;
  unsigned long long* mx;
  size_t bytes;
};

// Block width of the fused refinement: the solve's.
int fused_refine_kb(const sf_schedule_s* s, int nrhs) { return solve_kb(s, nrhs); }

FusedRefineWs fused_refine_layout(const sf_schedule_s* s, int nrhs, void* base) {
  const int kb = fused_refine_kb(s, nrhs);
  const size_t cols = size_t((nrhs + kb - 1) / kb) * size_t(kb);
  const size_t n = size_t(std::max<int64_t>(s->n, 1)), m = size_t(std::max<int64_t>(s->m, 1));
  const bool multi = kb > 1;
  const size_t sizes[5] = {align256(n * cols * 16), align256(multi ? n * cols * 8 : 256),
                           align256(multi ? n * cols * 8 : 256), align256(multi ? m * cols * 8 : 256), 2 * 64 * 8};
  char* p = static_cast<char*>(base);
  void* at[5];
  size_t off = 0;
  for (int k = 0; k < 5; ++k) {
    at[k] = p ? p + off : nullptr;
    off += sizes[k];
  }
  return FusedRefineWs{static_cast<float*>(at[0]), static_cast<double*>(at[1]), static_cast<double*>(at[2]),
                       static_cast<double*>(at[3]), static_cast<unsigned long long*>(at[4]), off};
}

size_t sf_refine_workspace_bytes(sf_schedule s, int32_t nrhs) {
  if (!s || nrhs < 1 || nrhs > 64) return 0;
  return std::max(refine_layout(s, nrhs, nullptr).bytes, fused_refine_layout(s, nrhs, nullptr).bytes);
}

}  // extern "C"

namespace {

// Per-column relative residuals from the max-abs accumulators (host copy).
sf_status read_relres(const unsigned long long* mx, int nrhs, double* out, hipStream_t st) {
  if (!out) return SF_OK;
  std::vector<unsigned long long> h(size_t(2 * nrhs));
  SF_HIP(hipMemcpyAsync(h.data(), mx, h.size() * 8, hipMemcpyDeviceToHost, st));
  SF_HIP(hipStreamSynchronize(st));
  for (int c = 0; c < nrhs; ++c) {
    double rm, bm;
    std::memcpy(&rm, &h[2 * c], 8);
    std::memcpy(&bm, &h[2 * c + 1], 8);
    out[c] = bm > 0 ? rm / bm : rm;
  }
  return SF_OK;
}

// The fused refinement: every stage of every right-hand side in one launch
// over the joint SpTRSV -> SpMV schedule (level items, or the multi-RHS
// units), packing and unpacking around it for several right-hand sides.
sf_status refine_fused(sf_schedule_s* s, const float* L32, const double* L64, const double* A64, const double* B,
                       int32_t ldb, int32_t nrhs, double* X, int32_t ldx, double* Y, int32_t ldy, int32_t nc,
                       double* out_relres, void* workspace, hipStream_t st) {
  const int kb = fused_refine_kb(s, nrhs);
  const bool multi = kb > 1;
  const FusedRefineWs ws = fused_refine_layout(s, nrhs, workspace);
  const int n = int32_t(s->n);
  const int nblk = (nrhs + kb - 1) / kb;
  const size_t cols = size_t(nblk) * size_t(kb);
  const int S4 = rf_tuple_floats(nc);
  RfArgs a{};
  a.ts = ts_args(s, L64, A64, nullptr, n, nrhs, multi ? nullptr : X, n, multi ? nullptr : Y, int32_t(s->m));
  a.L32 = L32;
  a.tup = reinterpret_cast<unsigned long long*>(ws.tup);
  a.maxabs = ws.mx;
  a.nrhs = nrhs;
  if (multi) {
    sf_status r = ensure_units(s, std::max(1, 64 / kb), st);
    if (r != SF_OK) return r;
    a.ts.unit_rng = reinterpret_cast<const int2*>(Y ? s->dev.unit_rng : s->dev.unit_trsv_rng);
    a.ts.item_ptr = nullptr;
    a.ts.item_list = nullptr;
    a.ts.n_work = Y ? s->dev.n_units : s->dev.n_unit_trsv;
    a.ts.kb = kb;
    a.ts.nblk = nblk;
    a.ts.xi = ws.xf;
    a.ts.Y = Y ? ws.y64 : nullptr;
    a.B = ws.b64;
  } else {
    a.B = B;  // one right-hand side: b, x and y are plain vectors (x doubles as the SpMV rows' flags)
  }
  sf_status r = next_epoch(s, st, a.ts.ls);
  if (r != SF_OK) return r;
  const int waves = multi ? multi_waves(s, kb, nrhs) : s->waves_per_cu;
  const int grid = persistent_grid(s, occupancy_rfused(nc, kb), waves);
  Timer tm(s, st);
  SF_HIP(launch_fill_pending(ws.tup, size_t(n) * cols * size_t(S4), 1, st));
  SF_HIP(launch_fill_u64(ws.mx, 2 * nrhs, st));
  if (multi) {
    // B -> interleaved FP64 blocks; x (interleaved) filled with the pending pattern
    SF_HIP(launch_pack(B, 0, ldb, n, nrhs, ws.b64, 0, ws.xf, kb, st));
  } else {
    SF_HIP(launch_fill_pending(X, size_t(n), 0, st));
  }
  if (a.ts.n_work > 0) SF_HIP(launch_rfused(a, nc, kb, grid, st));
  if (multi) {
    SF_HIP(launch_unpack(ws.xf, 0, n, nrhs, X, ldx, kb, st));
    if (Y) SF_HIP(launch_unpack(ws.y64, 0, int32_t(s->m), nrhs, Y, ldy, kb, st));
  }
  tm.stop();
  r = enqueued(s, st, SF_OK);
  if (r != SF_OK) return r;
  return read_relres(ws.mx, nrhs, out_relres, st);
}

}  // namespace

extern "C" {

sf_status sf_refine_trsv_spmv(sf_schedule s, const float* L32, const double* L64, const double* A64,
                              const double* B, int32_t ldb, int32_t nrhs, double* X, int32_t ldx,
                              double* Y, int32_t ldy, int32_t n_corrections, double* out_relres,
                              void* workspace, size_t ws_bytes, void* stream) {
  if (!s || s->kind != SF_TRSV_SPMV) return SF_ERR_ARG;
  if (nrhs < 1 || nrhs > 64 || n_corrections < 0 || n_corrections > 8) return SF_ERR_ARG;
  if (ldb < s->n || ldx < s->n || (Y && ldy < s->m)) return SF_ERR_SHAPE;
  if (s->n == 0) return SF_OK;
  if (!L32 || !L64 || !B || !X || (Y && !A64)) return SF_ERR_ARG;
  if (!workspace || ws_bytes < sf_refine_workspace_bytes(s, nrhs)) return SF_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // fused by default; a single right-hand side on a coarsened plan (deep,
  // narrow DAGs) runs the staged passes, whose FP32 solves use that plan
  // while the fused refinement walks level items
  const bool fused = s->refine_path == 0 && n_corrections <= 3 && !(nrhs == 1 && s->chunked);
  if (fused) {
    if (int64_t(s->n) * fused_refine_kb(s, nrhs) > int64_t(INT32_MAX)) return SF_ERR_UNSUPPORTED;
    sf_status r = upload(s, st);
    if (r != SF_OK) return r;
    return refine_fused(s, L32, L64, A64, B, ldb, nrhs, X, ldx, Y, ldy, n_corrections, out_relres, workspace, st);
  }
  // staged: one launch per pass (FP32 solves, FP64 residual passes, final pass)
  sf_status r = upload(s, st);
  if (r != SF_OK) return r;
  const int kb = solve_kb(s, nrhs);
  const bool multi = kb > 1;
  const RefineWs ws = refine_layout(s, nrhs, workspace);
  const int n = int32_t(s->n);
  MultiWs mw{};
  if (multi) {
    r = multi_ws(s, kb, nrhs, 4, st, mw);
    if (r == SF_OK) r = ensure_units(s, std::max(1, 64 / kb), st);
    if (r != SF_OK) return r;
  }
  // One FP32 solve L32 d = r32: several right-hand sides stay interleaved
  // (d in the solve's workspace, which the passes read as the correction).
  auto solve32 = [&]() -> sf_status {
    if (!multi) return exec_ts_fused(s, SF_F32, L32, nullptr, ws.r32, n, 1, ws.d32, n, nullptr, 0, st);
    return exec_multi_core(s, 1, L32, nullptr, ws.r32, mw.xi, nullptr, nrhs, kb, st);
  };
  const float* corr = multi ? static_cast<const float*>(mw.xi) : ws.d32;
  const double* b64 = multi ? ws.b64 : B;  // one right-hand side: B is its own layout
  // 1. x0 = L32^{-1} b in FP32 (b rounded to FP32)
  if (multi) {
    SF_HIP(launch_pack(B, 0, ldb, n, nrhs, ws.b64, 0, nullptr, kb, st));
    SF_HIP(launch_pack(B, 0, ldb, n, nrhs, ws.r32, 1, mw.xi, kb, st));
  } else {
    SF_HIP(launch_convert_f64_f32(B, ws.r32, n, st));
  }
  r = solve32();
  if (r != SF_OK) return r;
  // 2. corrections: x <- x + d, r = b - L64 x, d = L32^{-1} r
  const double* xin = nullptr;
  double* xout = ws.xa;
  for (int t = 0; t < n_corrections; ++t) {
    ResArgs ra{};
    ra.n = n;
    ra.m = int32_t(s->m);
    ra.nrhs = nrhs;
    ra.kb = kb;
    ra.Lrp = s->dev.Lrp;
    ra.Lci = s->dev.Lci;
    ra.L64 = L64;
    ra.B = b64;
    ra.xin = xin;
    ra.d = corr;
    ra.xout = xout;
    ra.r32 = ws.r32;
    SF_HIP(launch_residual(ra, st));
    if (multi) SF_HIP(launch_fill_pending(mw.xi, size_t(n) * size_t((nrhs + kb - 1) / kb) * size_t(kb), 1, st));
    r = solve32();
    if (r != SF_OK) return r;
    xin = xout;
    xout = (xout == ws.xa) ? ws.xb : ws.xa;
  }
  // 3. x_final = x + d; y = A64 x_final; r = b - L64 x_final (FP64)
  SF_HIP(launch_fill_u64(ws.mx, 2 * nrhs, st));
  ResArgs fa{};
  fa.n = n;
  fa.m = Y ? int32_t(s->m) : 0;
  fa.nrhs = nrhs;
  fa.kb = kb;
  fa.Lrp = s->dev.Lrp;
  fa.Lci = s->dev.Lci;
  fa.L64 = L64;
  fa.Arp = s->dev.Arp;
  fa.Aci = s->dev.Aci;
  fa.A64 = A64;
  fa.B = b64;
  fa.xin = xin;
  fa.d = corr;
  fa.xout = multi ? xout : X;
  fa.r32 = nullptr;
  fa.Y = Y ? (multi ? ws.y64 : Y) : nullptr;
  fa.maxabs = ws.mx;
  SF_HIP(launch_final(fa, st));
  if (multi) {
    SF_HIP(launch_unpack(xout, 0, n, nrhs, X, ldx, kb, st));
    if (Y) SF_HIP(launch_unpack(ws.y64, 0, int32_t(s->m), nrhs, Y, ldy, kb, st));
  }
  r = enqueued(s, stream, SF_OK);
  if (r != SF_OK) return r;
  return read_relres(ws.mx, nrhs, out_relres, st);
}

// Re-cut the work items after a parameter they depend on changed; the
// device copy is rebuilt at the next executor call.
sf_status recut(sf_schedule_s* s) {
  try {
    sf::cut_items(s);
  } catch (const std::bad_alloc&) {
    return SF_ERR_OOM;
  }
  if (s->trace) {  // sized for the old items
    wait_done(s);
    hipFree(s->trace);
    s->trace = nullptr;
  }
  if (s->dev.ready) {
    // the item arrays changed size: rebuild the constant block
    wait_done(s);
    if (s->dev.block) hipFree(s->dev.block);
    s->dev.block = nullptr;
    s->dev.ready = false;
  }
  if (s->dev.units) {
    wait_done(s);
    hipFree(s->dev.units);
    s->dev.units = nullptr;
    s->dev.units_rpb = 0;
  }
  return SF_OK;
}

sf_status sf_set_param(sf_schedule s, const char* key, int64_t v) {
  if (!s || !key) return SF_ERR_ARG;
  const std::string k(key);
  if (k == "lanes_trsv") {
    const bool factor_kind = s->kind == SF_IC0_TRSV || s->kind == SF_ILU0_TRSV;
    if (!pow2_in(int(v), factor_kind ? 4 : 2, factor_kind ? 64 : 32)) return SF_ERR_ARG;
    s->lanes_trsv = int32_t(v);
    if (factor_kind) return recut(s);  // factorisation items hold one batch of 64 / lanes rows
  } else if (k == "lanes_spmv") {
    if (!pow2_in(int(v), 4, 32)) return SF_ERR_ARG;
    s->lanes_spmv = int32_t(v);
  } else if (k == "rhs_block") {
    if (v != 0 && !pow2_in(int(v), 2, 64)) return SF_ERR_ARG;
    s->rhs_block = int32_t(v);
  } else if (k == "waves_per_cu") {
    if (v < 4 || v > 32) return SF_ERR_ARG;
    s->waves_per_cu = int32_t(v);
  } else if (k == "levelset_waves_per_cu") {
    if (v < 4 || v > 32) return SF_ERR_ARG;
    s->levelset_waves_per_cu = int32_t(v);
  } else if (k == "multi_waves_per_cu") {
    if (v != 0 && (v < 4 || v > 32)) return SF_ERR_ARG;
    s->multi_waves_per_cu = int32_t(v);
  } else if (k == "multi_path") {
    if (v < 0 || v > 2) return SF_ERR_ARG;
    s->multi_path = int32_t(v);
  } else if (k == "msp_parts") {
    if (v < 1 || v > (int64_t(1) << 20)) return SF_ERR_ARG;
    if (s->msp_parts != int32_t(v)) {
      s->msp_parts = int32_t(v);
      if (s->msp.dev) {
        wait_done(s);
        hipFree(s->msp.dev);
      }
      s->msp = StaticPlan();
    }
  } else if (k == "spin_limit") {
    if (v < 1) return SF_ERR_ARG;
    s->spin_limit = v;
  } else if (k == "claim_streams") {
    if (v < 1 || v > kStreams) return SF_ERR_ARG;
    s->claim_streams = int32_t(v);
  } else if (k == "rows_per_item" || k == "max_item_nnz" || k == "spmv_delay" || k == "coarsen") {
    if (k == "coarsen" ? (v < 0 || v > 3 || s->kind != SF_TRSV_SPMV)
        : k == "spmv_delay" ? (v < -1 || v > (int64_t(1) << 30)) : (v < 1 || v > (int64_t(1) << 30)))
      return SF_ERR_ARG;
    if (k == "rows_per_item" && v > 64) return SF_ERR_ARG;  // one lane finishes each row
    if (k == "rows_per_item") s->rows_per_item = int32_t(v);
    else if (k == "max_item_nnz") s->max_item_nnz = int32_t(v);
    else if (k == "coarsen") s->coarsen = int32_t(v);
    else s->spmv_delay = int32_t(v);
    const sf_status rc = recut(s);
    if (rc != SF_OK) return rc;
  } else if (k == "region_rows") {
    if (v < 64 || v > 16384 || s->kind != SF_TRSV_SPMV) return SF_ERR_ARG;
    s->region_rows = int32_t(v);
    const sf_status rc = recut(s);
    if (rc != SF_OK) return rc;
  } else if (k == "region_poll") {
    if ((v & 0xff) < 1 || (v & 0xff) > 64 || ((v >> 16) & 0xff) > 64 || v < 0 || v > 0xffffff) return SF_ERR_ARG;
    s->region_poll = int32_t(v);
  } else if (k == "cached_reads") {
    if (v < 0 || v > 3) return SF_ERR_ARG;
    s->cached_reads = int32_t(v);
  } else if (k == "refine_path") {
    if (v < 0 || v > 1) return SF_ERR_ARG;
    s->refine_path = int32_t(v);
  } else if (k == "autotune_cache") {
    s->autotune_cache = v ? 1 : 0;
  } else if (k == "no_fusion") {
    s->no_fusion = v ? 1 : 0;
  } else if (k == "timing") {
    s->timing = v ? 1 : 0;
  } else if (k == "ic0_cached") {
    if (v < 0 || v > 1) return SF_ERR_ARG;
    s->ic0_cached = int32_t(v);
  } else if (k == "spmv_prefix") {
    if (v < 0 || v > 1) return SF_ERR_ARG;
    s->spmv_prefix = int32_t(v);
  } else if (k == "spmv_item_scale") {
    if (v < 1 || v > 8 || s->kind != SF_TRSV_SPMV) return SF_ERR_ARG;
    s->spmv_item_scale = int32_t(v);
    const sf_status rc = recut(s);
    if (rc != SF_OK) return rc;
  } else if (k == "precond_regions") {
    if (v < 0 || v > 1) return SF_ERR_ARG;
    s->precond_regions = int32_t(v);
  } else if (k == "trace") {
    // trace mode: the fused single-RHS executor stamps every item (debug
    // aid); 2: items only, no per-iteration publication stamps
    if (v < 0 || v > 2) return SF_ERR_ARG;
    s->trace_level = int32_t(v);
    if (s->trace) {
      wait_done(s);
      hipFree(s->trace);
      s->trace = nullptr;
    }
    if (v) {
      s->trace_items = std::max(std::max(s->item_ptr.size(), s->citem_ptr.size()), s->ritem_ptr.size()) + 1;
      const size_t bytes = trace_words(s) * sizeof(unsigned long long);
      if (trace_words(s) > size_t(INT32_MAX)) return SF_ERR_UNSUPPORTED;
      if (hipMalloc(&s->trace, bytes) != hipSuccess) return SF_ERR_OOM;
      if (hipMemset(s->trace, 0, bytes) != hipSuccess) return SF_ERR_HIP;
    }
  } else {
    return SF_ERR_ARG;
  }
  return SF_OK;
}

sf_status sf_get_param(sf_schedule s, const char* key, int64_t* v) {
  if (!s || !key || !v) return SF_ERR_ARG;
  const std::string k(key);
  if (k == "lanes_trsv") *v = s->lanes_trsv;
  else if (k == "lanes_spmv") *v = s->lanes_spmv;
  else if (k == "rhs_block") *v = s->rhs_block;
  else if (k == "waves_per_cu") *v = s->waves_per_cu;
  else if (k == "levelset_waves_per_cu") *v = s->levelset_waves_per_cu;
  else if (k == "multi_waves_per_cu") *v = s->multi_waves_per_cu;
  else if (k == "spin_limit") *v = s->spin_limit;
  else if (k == "msp_parts") *v = s->msp_parts;
  else if (k == "multi_path") *v = s->multi_path;
  else if (k == "claim_streams") *v = s->claim_streams;
  else if (k == "rows_per_item") *v = s->rows_per_item;
  else if (k == "max_item_nnz") *v = s->max_item_nnz;
  else if (k == "spmv_delay") *v = s->spmv_delay;
  else if (k == "coarsen") *v = s->coarsen;
  else if (k == "coarsened") *v = s->chunked ? 1 : 0;
  else if (k == "pairs") *v = s->pair_ptr.empty() ? 0 : int64_t(s->pair_ptr.back());  // SpIC0 / SpILU0 intersection pairs (read only)
  else if (k == "back_coarsened") *v = s->bchunked ? 1 : 0;
  else if (k == "back_regioned") *v = s->bregioned ? 1 : 0;  // read only: the backward region plan is in effect
  else if (k == "back_region_chain") *v = s->back_region_chain;
  else if (k == "no_fusion") *v = s->no_fusion;
  else if (k == "autotune_cache") *v = s->autotune_cache;
  else if (k == "refine_path") *v = s->refine_path;
  else if (k == "cached_reads") *v = s->cached_reads;
  else if (k == "region_rows") *v = s->region_rows;
  else if (k == "region_poll") *v = s->region_poll;
  else if (k == "regioned") *v = s->regioned ? 1 : 0;  // read only: the region plan is in effect
  else if (k == "region_chain") *v = s->region_chain;
  else if (k == "tuned_from_cache") *v = s->tuned_from_cache;  // read only: last sf_autotune reused a result
  else if (k == "fingerprint") *v = int64_t(pattern_fingerprint(s) & 0x7fffffffffffffffull);
  else if (k == "timing") *v = s->timing;
  else if (k == "trace") *v = s->trace ? s->trace_level : 0;
  else if (k == "spmv_prefix") *v = s->spmv_prefix;
  else if (k == "precond_regions") *v = s->precond_regions;
  else if (k == "spmv_item_scale") *v = s->spmv_item_scale;
  else if (k == "ic0_cached") *v = s->ic0_cached;
  else if (k == "prefix_rows") *v = s->prefix_rows;  // read only: SpMV rows with a fusable prefix
  else if (k == "prefix_entries") *v = s->prefix_entries;  // read only: A entries in those prefixes
  else return SF_ERR_ARG;
  return SF_OK;
}

}  // extern "C"

namespace {

// ---- autotuner results, shared by every schedule of the process ----
// Keyed by the pattern's fingerprint (sizes, depth and a 64-bit FNV-1a hash
// of both CSR patterns), the value type, the right-hand-side count and
// whether y is computed: a schedule inspected again from the same matrix
// takes the tuned parameters without timing anything.
const char* const kTuneKeys[] = {"coarsen",       "multi_path",   "rhs_block",    "spmv_delay",
                                 "rows_per_item", "max_item_nnz", "waves_per_cu", "multi_waves_per_cu",
                                 "cached_reads",  "spmv_prefix", "spmv_item_scale"};
constexpr int kNTune = int(sizeof(kTuneKeys) / sizeof(kTuneKeys[0]));
struct Tuned {
  int64_t v[kNTune];
  double best_ms;
};
using TuneKey = std::tuple<uint64_t, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, Tuned>& tune_cache() {
  static std::map<TuneKey, Tuned> m;
  return m;
}

uint64_t fnv1a(uint64_t h, const void* p, size_t bytes) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < bytes; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

uint64_t pattern_fingerprint(sf_schedule_s* s) {
  if (s->fingerprint) return s->fingerprint;
  uint64_t h = 14695981039346656037ull;
  const int64_t head[6] = {s->n, s->m, s->L.nnz(), s->A.nnz(), s->depth, s->kind};
  h = fnv1a(h, head, sizeof(head));
  for (const sf::Pattern* P : {&s->L, &s->A}) {
    h = fnv1a(h, P->rp.data(), P->rp.size() * 4);
    h = fnv1a(h, P->ci.data(), P->ci.size() * 4);
  }
  s->fingerprint = h ? h : 1;
  return s->fingerprint;
}

}  // namespace

extern "C" {

sf_status sf_autotune(sf_schedule s, sf_dtype dtype, const void* L_val, const void* A_val, const void* B,
                      int32_t ldb, int32_t nrhs, void* X, int32_t ldx, void* Y, int32_t ldy, void* stream,
                      double* out_best_ms) {
  sf_status r = check_ts_args(s, dtype, L_val, A_val, B, ldb, nrhs, X, ldx, Y, ldy);
  if (r != SF_OK) return r;
  if (s->n == 0) return SF_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  s->tuned_from_cache = 0;
  const TuneKey key{pattern_fingerprint(s), int(dtype), int(nrhs), Y ? 1 : 0};
  if (s->autotune_cache) {
    Tuned hit{};
    bool found = false;
    {
      std::lock_guard<std::mutex> g(g_tune_mu);
      auto it = tune_cache().find(key);
      if (it != tune_cache().end()) {
        hit = it->second;
        found = true;
      }
    }
    if (found) {
      for (int k = 0; k < kNTune; ++k) {
        int64_t cur = 0;
        sf_get_param(s, kTuneKeys[k], &cur);
        if (cur != hit.v[k]) {
          r = sf_set_param(s, kTuneKeys[k], hit.v[k]);
          if (r != SF_OK) return r;
        }
      }
      s->tuned_from_cache = 1;
      if (out_best_ms) *out_best_ms = hit.best_ms;
      return SF_OK;
    }
  }
  hipEvent_t e0, e1;
  SF_HIP(hipEventCreate(&e0));
  SF_HIP(hipEventCreate(&e1));
  const int saved_timing = s->timing;
  s->timing = 0;
  auto time_once = [&](double& best) -> sf_status {
    sf_status rr = upload(s, st);
    if (rr != SF_OK) return rr;
    best = 1e30;
    for (int rep = 0; rep < 4; ++rep) {
      hipEventRecord(e0, st);
      rr = exec_ts_fused(s, dtype, L_val, A_val, B, ldb, nrhs, X, ldx, Y, ldy, st);
      if (rr != SF_OK) return rr;
      hipEventRecord(e1, st);
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) best = std::min(best, double(ms));  // first run warms up
    }
    return SF_OK;
  };
  double best = 1e30;
  r = time_once(best);
  // coordinate search: plan, RHS block, SpMV delay, item size and budget, residency
  auto try_param = [&](const char* key, const std::vector<int64_t>& cands) -> sf_status {
    int64_t keep = 0;
    sf_get_param(s, key, &keep);
    for (int64_t c : cands) {
      if (c == keep) continue;
      if (sf_set_param(s, key, c) != SF_OK) continue;
      double t = 0;
      sf_status rr = time_once(t);
      if (rr != SF_OK) return rr;
      if (t < best * 0.98) {
        best = t;
        keep = c;
      }
    }
    return sf_set_param(s, key, keep);
  };
  // one right-hand side: level items vs coarsened items first (the entry
  // stream makes lanes per row irrelevant there)
  if (r == SF_OK && nrhs == 1) r = try_param("coarsen", {1, 2, 3});
  if (r == SF_OK && nrhs > 1) r = try_param("multi_path", {1, 2});
  if (r == SF_OK && nrhs > 1) r = try_param("rhs_block", {8, 16, 32, 64});
  if (r == SF_OK && Y) r = try_param("spmv_delay", {1, 2, 4, 8, 16, 32, 1 << 20});
  if (r == SF_OK) r = try_param("rows_per_item", {8, 16, 32, 64});
  if (r == SF_OK && nrhs == 1) r = try_param("max_item_nnz", {128, 256, 512, 1024, 2048});
  if (r == SF_OK && nrhs == 1) r = try_param("waves_per_cu", {4, 8, 16});
  if (r == SF_OK && nrhs == 1 && Y && !s->chunked && !s->regioned) r = try_param("spmv_item_scale", {1, 2, 4});
  if (r == SF_OK && Y && s->prefix_rows > 0) r = try_param("spmv_prefix", {0, 1});
  if (r == SF_OK && nrhs > 1) r = try_param("multi_waves_per_cu", {8, 16, 32});
  if (r == SF_OK) r = upload(s, st);
  r = enqueued(s, stream, r);
  s->timing = saved_timing;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (out_best_ms) *out_best_ms = best;
  if (r == SF_OK && s->autotune_cache) {
    Tuned t{};
    for (int k = 0; k < kNTune; ++k) sf_get_param(s, kTuneKeys[k], &t.v[k]);
    t.best_ms = best;
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_cache()[key] = t;
  }
  return r;
}

sf_status sf_sync_status(sf_schedule s, void* stream) {
  if (!s) return SF_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  SF_HIP(hipStreamSynchronize(st));
  if (!s->dev.state) return SF_OK;
  int32_t v = 0;
  SF_HIP(hipMemcpy(&v, s->dev.state + kStatusOff, sizeof(v), hipMemcpyDeviceToHost));
  if (v != 0) {
    const int32_t z = 0;
    SF_HIP(hipMemcpy(s->dev.state + kStatusOff, &z, sizeof(z), hipMemcpyHostToDevice));
    return SF_ERR_TIMEOUT;
  }
  return SF_OK;
}

sf_status sf_trace_export(sf_schedule s, unsigned long long* out, int64_t count) {
  if (!s || !out || !s->trace) return SF_ERR_ARG;
  const size_t items = (s->regioned ? s->ritem_ptr.size() : s->chunked ? s->citem_ptr.size() : s->item_ptr.size()) - 1;
  const size_t rows = 2 * size_t(s->n + s->m);
  if (count < int64_t(items * kTraceItemWords + rows)) return SF_ERR_SHAPE;
  wait_done(s);
  const size_t at = s->trace_items * kTraceItemWords;
  if (hipMemcpy(out, s->trace, items * kTraceItemWords * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return SF_ERR_HIP;
  if (hipMemcpy(out + items * kTraceItemWords, s->trace + at, rows * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return SF_ERR_HIP;
  return SF_OK;
}

sf_status sf_last_kernel_ms(sf_schedule s, double* ms) {
  if (!s || !ms) return SF_ERR_ARG;
  *ms = s->last_kernel_ms;
  return SF_OK;
}

}  // extern "C"
