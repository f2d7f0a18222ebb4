// Internal definitions shared by the host inspector, the C ABI and the
// kernel launchers.  Not part of the public interface (include/sf.h).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sf.h"

namespace sf {

// A CSR pattern owned by the schedule (host copy).
struct Pattern {
  int32_t nrows = 0, ncols = 0;
  std::vector<int32_t> rp, ci;
  int64_t nnz() const { return rp.empty() ? 0 : rp.back(); }
};

// Layout of the small per-schedule device state block (int32 words).  Each
// field sits on its own 256-byte line.  Fields indexed by parity p = epoch & 1
// belong to the launch with that epoch parity; every launch clears the fields
// of the other parity for the launch that follows it on the stream.
constexpr int kLine = 64;                 // int32 words per 256-byte line
constexpr int kStreams = 32;              // claim counters per parity
inline constexpr int ctr_off(int p, int s) { return (p * kStreams + s) * kLine; }
inline constexpr int done_off(int p) { return (2 * kStreams + p) * kLine; }
inline constexpr int info_off(int p) { return (2 * kStreams + 2 + p) * kLine; }
inline constexpr int bar_off(int p) { return (2 * kStreams + 4 + p) * kLine; }
// The watchdog status of the launch with parity p (it makes that launch's
// waves drain; cleared for the next launch like the other per-parity
// fields) and a sticky report that only sf_sync_status reads and clears, so
// a timeout is reported but never shortens the waits of a later launch.
inline constexpr int status_off(int p) { return (2 * kStreams + 6 + p) * kLine; }
constexpr int kStatusOff = (2 * kStreams + 8) * kLine;
constexpr int kStateWords = (2 * kStreams + 10) * kLine;
constexpr int kChunkEntries = 512;        // off-diagonals of one coarsened item (one stream pass)
constexpr int kInfoNone = 0x7f7f7f7f;     // "no failing row" (byte-fill value of the block)
constexpr int kStatusTimeout = 1;
// Trace mode: per work item kTraceItemWords 64-bit words -- real-time-counter
// stamps at the start, once its indices and values are loaded, once every
// input is ready and at the end, then how many times the item ran -- and,
// after the items, two words per iteration id (stamp taken just before the
// value was published, publication count).
constexpr int kTraceItemWords = 8;
// LDS of a region (k_region.hip): per row a head record -- the first
// kRegionAhead entries' values and input slots, the right-hand side, the
// diagonal, the iteration id and the row's share of the overflow table --
// then the x slots (the region's rows, its external inputs and a slot
// holding 0), the overflow entries (values and slots of entries past the
// first kRegionAhead), the external columns and the batch table; at most
// kRegionLdsMax bytes (else the region plan is not used).  `ovf` counts the
// region's overflow entries.
constexpr size_t kRegionLdsMax = 64 * 1024;
constexpr int kRegionAhead = 4;
inline size_t region_head_bytes(int vb) { return vb == 8 ? 64 : 48; }
inline size_t region_lds_bytes(int rows, int ovf, int ext, int batches, int vb) {
  const size_t a = size_t(rows) * region_head_bytes(vb) + size_t(rows + ext + 1) * size_t(vb) +
                   size_t(ovf) * size_t(vb + 2) + size_t(ext) * 4 + size_t(batches + 1) * 4;
  return (a + 255) / 256 * 256 + 256;
}

struct DeviceBuffers {
  int device = -1;
  bool ready = false;
  void* block = nullptr;    // single allocation holding every array below
  size_t block_bytes = 0;
  // patterns
  int32_t *Lrp = nullptr, *Lci = nullptr, *Arp = nullptr, *Aci = nullptr;
  // forward schedule
  int32_t *order = nullptr, *item_ptr = nullptr, *trsv_items = nullptr, *spmv_items = nullptr;
  int32_t *lvl_items = nullptr;     // item list of the level-set baseline
  int32_t *lvl_item_ptr = nullptr;  // per level, into lvl_items
  // coarsened plan of the one-right-hand-side fused executor
  int32_t *corder = nullptr, *citem_ptr = nullptr, *ctrsv_items = nullptr;
  int32_t *qrng = nullptr, *cqrng = nullptr;
  uint8_t *clloc = nullptr;         // local wavefront of each claim position
  uint8_t *celoc = nullptr;         // per stored L entry: slot of its column in the row's item, or 0xFF
  // backward
  int32_t *LTrp = nullptr, *LTci = nullptr, *LTmap = nullptr;
  int32_t *ATrp = nullptr, *ATci = nullptr, *ATmap = nullptr;
  int32_t *border = nullptr, *bitem_ptr = nullptr;
  int32_t *bcorder = nullptr, *bcitem_ptr = nullptr;
  uint8_t *bclloc = nullptr, *bceloc = nullptr;
  // backward region plan
  int32_t *brorder = nullptr, *britem_ptr = nullptr, *brroff = nullptr;
  int32_t *brbatch = nullptr, *brbatch_ptr = nullptr, *brext = nullptr, *brext_ptr = nullptr;
  uint16_t* brcode = nullptr;
  // prefix fusion (level plan)
  int32_t *pqrng = nullptr, *apre = nullptr;
  // region plan
  int32_t *rorder = nullptr, *ritem_ptr = nullptr, *rtrsv_items = nullptr, *rqrng = nullptr, *rroff = nullptr;
  int32_t *rbatch = nullptr, *rbatch_ptr = nullptr, *rext = nullptr, *rext_ptr = nullptr;
  uint16_t* rcode = nullptr;
  // SpIC0 intersection lists
  int32_t *pair_ptr = nullptr, *pair_u = nullptr, *pair_q = nullptr;
  int32_t *prng = nullptr, *piv = nullptr;
  int32_t* dpos = nullptr;          // SpILU0: diagonal position of each row
  // mutable state
  int32_t* state = nullptr;
  void* xi = nullptr;           // interleaved right-hand-side workspace
  size_t xi_bytes = 0;
  // multi-RHS plan: the level items split into units of at most units_rpb
  // rows; per unit its range of claim positions (all units in claim order,
  // and the SpTRSV units alone, which are sorted by level), and per level
  // the first SpTRSV unit (level-set baseline)
  void* units = nullptr;
  int32_t *unit_rng = nullptr, *unit_trsv_rng = nullptr;  // (first, end) pairs
  int32_t* lvl_unit_ptr = nullptr;
  int32_t units_rpb = 0, n_units = 0, n_unit_trsv = 0;
  uint32_t epoch = 0;
  // recorded on the caller's stream after each executor call's launches:
  // freeing the schedule waits for it instead of for the whole device
  void* done = nullptr;  // hipEvent_t
};

// Static two-level plan of the SpTRSV -> SpMV pair (static_plan.cpp): the
// paper's fused partitioning (Sec. 3) or the fused-wavefront baseline.  The
// s-partitions run in sequence with a grid barrier between them; the
// w-partitions of one s-partition are independent; the rows of one
// w-partition run in order, cut into batches of up to 64 rows of one kind
// and one wavefront for the executor.
struct StaticPlan {
  bool built = false;
  int32_t parts = 0;                // requested w-partitions per s-partition (MSP's r)
  std::vector<int32_t> s_ptr;       // nb + 1: w-partitions of each s-partition
  std::vector<int32_t> w_ptr;       // nw + 1: positions of each w-partition
  std::vector<int32_t> order;       // n + m iteration ids (as the joint order)
  std::vector<int32_t> w_batch;     // nw + 1: batches of each w-partition
  std::vector<int32_t> batch_ptr;   // nbatch + 1: positions of each batch
  std::vector<int32_t> qrng;        // 2 (n + m): CSR range per position (as qrng)
  int32_t merged = 0;               // pair partitions merged (MSP)
  int32_t slack_moved = 0;          // slack rows placed by balancing (MSP)
  void* dev = nullptr;              // device copy: order | qrng | s_ptr | w_batch | batch_ptr
  int32_t *d_order = nullptr, *d_qrng = nullptr, *d_s_ptr = nullptr, *d_w_batch = nullptr,
          *d_batch_ptr = nullptr;
};

}  // namespace sf

struct sf_schedule_s {
  int kind = SF_TRSV_SPMV;
  sf::Pattern L, A;
  int64_t n = 0, m = 0;

  // Forward analysis.
  std::vector<int32_t> level;        // n: wavefront of each SpTRSV row
  std::vector<int32_t> ready;        // m: joint wavefront of each SpMV row
  int32_t depth = 0, joint_depth = 0, max_level_width = 0;
  int32_t max_offdiag = 0;           // longest row of L, diagonal excluded

  // Fused forward schedule: iteration ids in claim order cut into items.
  // SF_TRSV_SPMV: id i < n is SpTRSV row i, id n + r is SpMV row r.
  // SF_IC0_TRSV: ids are rows; row i's item runs SpIC0 row i then SpTRSV row i.
  std::vector<int32_t> order, item_ptr;
  std::vector<int32_t> trsv_items;   // items holding SpTRSV rows, in claim order
  std::vector<int32_t> spmv_items;   // items holding SpMV rows, in claim order
  // Per claim position q, the CSR range the row's dot product runs over:
  // [qrng[2q], qrng[2q+1]) -- the off-diagonals of an SpTRSV row (its
  // diagonal sits at qrng[2q+1]), the whole row of an SpMV row -- so an
  // item's loads do not wait for the row pointers.  SF_IC0_TRSV: the
  // ranges of the SpTRSV rows (used by the unfused baseline's solve).
  std::vector<int32_t> qrng, cqrng;  // level plan, coarsened plan
  // Level-set baseline: items of SpTRSV rows grouped by level.
  std::vector<int32_t> lvl_items, lvl_item_ptr;

  // Coarsened plan (SF_TRSV_SPMV, one right-hand side).  The SpTRSV rows
  // are cut into items of up to 64 rows that may depend on each other
  // inside the item (several wavefronts per item, the paper's w-partitions);
  // an item's rows are sorted by their local wavefront (clloc).  The items
  // are contiguous runs of one topological order, so the item graph is
  // acyclic and claiming items in that order cannot deadlock.  SpMV rows
  // follow the item that finishes their last input.
  int32_t coarsen = 0;               // requested: 0 auto, 1 level items, 2 coarsened
  bool chunked = false;              // the coarsened plan is in effect
  std::vector<int32_t> corder, citem_ptr, ctrsv_items;
  std::vector<uint8_t> clloc, celoc;
  int32_t chunk_chain = 0, max_local_depth = 0;
  double est_level_us = 0.0, est_chunk_us = 0.0;

  double est_chunk_pipe_us = 0.0;    // the coarsened plan under the pipelined-item model (region_estimate)

  // Region plan (SF_TRSV_SPMV, one right-hand side; coarsen = 3, or chosen
  // by the model): regions of up to region_rows rows, each run by one
  // wavefront level by level with its x in LDS, every row waiting only for
  // its own inputs (inspect.cpp, build_regions; k_region.hip).
  // Prefix fusion on the level plan: SpMV row r's entries up to its
  // diagonal, when their columns are exactly SpTRSV row r's (L = lower(A)),
  // are folded by SpTRSV row r's item from the x values it gathers anyway;
  // the SpMV row continues the fold past them.  apre: per claim position of
  // `order`, A's first position of the SpTRSV row's prefix or -1; pqrng:
  // qrng with each such SpMV row's range starting past its prefix, encoded
  // -(start + 1).
  int32_t spmv_prefix = 1;              // 0: off
  int32_t precond_regions = 1;          // fused preconditioner apply on the region plans when both exist
  int32_t spmv_item_scale = 4;          // level items: SpMV items take this many times the rows and budget
  int32_t ic0_cached = 0;               // fused SpIC0 reads its values through the caches first (Ic0Args::cached)
  int64_t prefix_rows = 0;              // SpMV rows with a fused prefix
  int64_t prefix_entries = 0;           // A entries in those prefixes (diagonals included)
  std::vector<int32_t> pqrng, apre;
  int32_t region_rows = 512;
  int32_t region_poll = 64 | (2 << 16);  // poller lanes (bits 0-7), back-off rounds (bits 8-15),
                                         // lanes before the first input (bits 16-23)
  bool regioned = false;             // the region plan is in effect for the fused executor
  std::vector<int32_t> rorder, ritem_ptr, rtrsv_items, rqrng, rroff;
  std::vector<uint8_t> rlloc;
  std::vector<int32_t> rbatch, rbatch_ptr;   // (first position, first external index) per batch; batches per item
  std::vector<int32_t> rext, rext_ptr;       // external inputs (columns) per item
  std::vector<uint16_t> rcode;               // per stored L entry: in-region position, or 0x8000 | external index
  int32_t region_rows_max = 0, region_entries_max = 0, region_ext_max = 0, region_batches_max = 0;
  int32_t region_chain = 0;
  double est_region_us = 0.0;

  // Backward (transposed solve) schedule.
  bool has_back = false;
  sf::Pattern LT, AT;                // CSR of L^T and A^T
  std::vector<int32_t> LT_map, AT_map;  // entry of the transpose -> entry of the source
  std::vector<int32_t> rlevel, border, bitem_ptr;
  int32_t back_depth = 0;
  // coarsened backward plan (as the forward one, over L^T)
  bool bchunked = false;
  std::vector<int32_t> bcorder, bcitem_ptr;
  std::vector<uint8_t> bclloc, bceloc;  // per claim position; per stored L^T entry
  int32_t back_chunk_chain = 0;
  // Backward region plan (the transposed solve's regions, as the forward
  // region plan over L^T; brcode indexed by L^T position).
  bool bregioned = false;
  std::vector<int32_t> brorder, britem_ptr, brroff, brbatch, brbatch_ptr, brext, brext_ptr;
  std::vector<uint8_t> brlloc;
  std::vector<uint16_t> brcode;
  int32_t back_region_rows_max = 0, back_region_entries_max = 0, back_region_ext_max = 0,
          back_region_batches_max = 0, back_region_chain = 0;
  double est_back_region_us = 0.0, est_back_chunk_pipe_us = 0.0;
  double est_back_level_us = 0.0, est_back_chunk_us = 0.0;

  // SpIC0 intersection lists, one list per stored L entry (i, j), j < i:
  // pairs (t << 16 | u, q): t = index inside row i of the entry (i, j), u =
  // index inside row i of a column k in both rows with k < j, q = position
  // of L_jk.  The lists of a row's entries are contiguous, in entry order.
  std::vector<int32_t> pair_ptr, pair_u, pair_q;
  // SF_IC0_TRSV: per claim position the range of the row's pairs (as qrng
  // gives its entries), and per stored entry (i, j), j < i, the position of
  // the pivot L_jj, so a batch's loads need no row-pointer round trips.
  std::vector<int32_t> prng, piv;
  // SF_ILU0_TRSV: the pattern of A is held in L; dpos[i] is the position of
  // row i's diagonal.  Pairs then follow build_pairs_ilu (inspect.cpp).
  std::vector<int32_t> dpos;

  // Executor parameters.
  int32_t lanes_trsv = 4, lanes_spmv = 8, rhs_block = 0, waves_per_cu = 8;
  int32_t multi_waves_per_cu = 0;  // residency target of the multi-RHS executors (0: by level width)
  int32_t levelset_waves_per_cu = 4;  // residency of the barrier-synchronised executors (level sets, static plans)
  int32_t multi_path = 0;          // several RHS: 0 auto, 1 interleaved units, 2 one item chain per column
  int32_t rows_per_item = 64, max_item_nnz = 4096;
  // wavefronts (level items) or item-chain steps (coarsened items) an SpMV
  // row is placed after its inputs are final; -1: 0 for level items, after
  // every SpTRSV item for coarsened ones
  int32_t spmv_delay = -1;
  int64_t spin_limit = int64_t(1) << 22;
  int32_t claim_streams = 1;
  int32_t no_fusion = 0;
  int32_t timing = 0;
  int32_t autotune_cache = 1;           // sf_autotune reuses results for an equal pattern
  int32_t refine_path = 0;              // sf_refine_trsv_spmv: 0 fused (one launch), 1 staged passes
  int32_t cached_reads = 0;             // fused executor: x read through the caches first (TsArgs::cached)
  int32_t tuned_from_cache = 0;         // the last sf_autotune call did
  uint64_t fingerprint = 0;             // of the patterns (computed on first use; 0: not yet)
  unsigned long long* trace = nullptr;  // device trace buffer (trace mode, layout at kTraceItemWords)
  int32_t trace_level = 0;              // 1: items and iterations, 2: items only
  size_t trace_items = 0;               // item records in it (rows follow them)
  double last_kernel_ms = -1.0;
  double reuse = 0.0, inspect_seconds = 0.0;

  // static plans (SF_TRSV_SPMV): the paper's MSP partitioning and the fused
  // wavefront baseline, built on first use
  sf::StaticPlan msp, wavefront;
  int32_t msp_parts = 1024;

  sf::DeviceBuffers dev;
};

namespace sf {

// Host inspector entry points (inspect.cpp).
sf_status check_lower(const sf_csr_pattern* L);
sf_status check_general(const sf_csr_pattern* A, int32_t ncols);
sf_status check_square_diag(const sf_csr_pattern* A);
sf_status build_schedule(sf_schedule_s* s, const sf_csr_pattern* L, const sf_csr_pattern* A,
                         const sf_inspect_opts& o);
// Re-cut the work items after a change of rows_per_item / max_item_nnz.
void cut_items(sf_schedule_s* s);
// Check every DAG edge of the built forward schedule (0 = valid).
int validate_forward(const sf_schedule_s* s);
// Static plans (static_plan.cpp); host only.  plan 0: MSP, 1: fused wavefront.
sf_status build_static(sf_schedule_s* s, int plan);
StaticPlan& static_plan(sf_schedule_s* s, int plan);

}  // namespace sf
