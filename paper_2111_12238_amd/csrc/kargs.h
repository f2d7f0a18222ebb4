// Kernel argument blocks and launcher declarations shared by the C ABI
// (api.cpp) and the kernel translation units (*.hip).  Plain structs of
// device pointers and sizes; every pointer is a device address.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sf {

// Per-launch bookkeeping shared by every persistent kernel.
struct LaunchState {
  int32_t* state;     // device state block (schedule.h layout)
  int32_t epoch;      // launch counter; its parity selects the state fields
  int32_t spin_limit; // polls before the watchdog fires
  int32_t streams;    // claim counters in use (1..kStreams)
};

// Fused SpTRSV -> SpMV (also SpTRSV alone when A == nullptr / Y == nullptr).
struct TsArgs {
  int32_t n, m;
  const int32_t *Lrp, *Lci;
  const void* Lv;
  const int32_t *Arp, *Aci;
  const void* Av;
  // One right-hand side: plain vectors (B, X of length n, Y of length m).
  // Several: B, xi and Y are in the interleaved block layout of k_layout.hip
  // (nblk blocks of kb columns; B and xi of n rows, Y of m rows), X is unused
  // and the ld fields are ignored.
  const void* B;
  int32_t ldb;
  void* X;
  int32_t ldx;
  void* Y;
  int32_t ldy;
  int32_t nrhs, kb, nblk;  // right-hand sides, block width, number of blocks
  void* xi;                // interleaved solution, also its readiness flags (nrhs > 1)
  int32_t col_units;       // > 1: that many right-hand sides, each its own chain of the items, on
                           // column-major B, X, Y (k_ts_fused; work index = item * col_units + column)
  const int32_t *order, *item_ptr, *item_list;
  const int2* unit_rng;    // multi-RHS: claim-position range of each unit (replaces item_ptr / item_list)
  const int32_t* qrng;     // per claim position: CSR range of the row's dot product (pairs)
  int32_t n_work;          // items to run (entries of item_list, or all items)
  const uint8_t* lloc;     // coarsened plan: local wavefront per claim position (else nullptr)
  const uint8_t* eloc;     // coarsened plan: per L entry, slot of its column in the item or 0xFF
  const int32_t* apre;     // prefix fusion (level items, k_ts_fused<T, true>): per claim position of an
                           // SpTRSV row i, A's first position of SpMV row i's prefix (its entries up to
                           // the diagonal, columns those of L's row i), or -1; SpMV rows with a prefix
                           // have qrng.x = -(first position past the prefix + 1) and start from Y
  int32_t cached;           // fused executor: bit 0 = SpMV rows, bit 1 = SpTRSV level items read x
                            // through the caches first (stream.h, VEC = 3)
  unsigned long long* trace;  // optional: kTraceItemWords words per item (see k_ts.hip)
  unsigned long long* rtrace; // with trace: per iteration id (SpTRSV row i, SpMV row n + r) its
                              // publication time and how many times it was published
  LaunchState ls;
};

// Region plan of the fused executor (k_region.hip, inspect.cpp build_regions).
struct RegionArgs {
  const int32_t* batch;      // per batch: (first claim position, first external input of the region)
  const int32_t* batch_ptr;  // per item: its batches (none for SpMV items)
  const int32_t* ext;        // external inputs (columns) of every region
  const int32_t* ext_ptr;    // per item: its external inputs
  const int32_t* roff;       // per claim position: offset of the row's overflow entries in its region
  const uint16_t* code;      // per stored L entry: in-region position, or 0x8000 | external index
  int32_t rows_max, entries_max, ext_max, batches_max;  // LDS sizing (largest region)
  int32_t poll_lanes, poll_sleep;  // poller: lanes watching inputs, back-off (x 128 cycles) after an idle round
  int32_t poll_gate;               // poller lanes reading until the region's first input is stored
};
size_t region_kernel_lds(const RegionArgs& r, int dtype);
int occupancy_region(const RegionArgs& r, int dtype);
hipError_t launch_bwd_region(const struct BwdArgs& a, const RegionArgs& r, int dtype, int grid, hipStream_t st);
hipError_t launch_pair_region(const struct TsArgs& a, const RegionArgs& r, int dtype, int mode, int grid,
                              hipStream_t st);
int occupancy_bwd_region(const RegionArgs& r, int dtype);

// Level-set (unfused) SpTRSV: items grouped by level, one grid barrier each.
struct LevelArgs {
  TsArgs ts;               // patterns, values, vectors (item_list = level items)
  const int32_t* lvl_item_ptr;
  int32_t depth;
};

// Static two-level plan (static_plan.cpp): the s-partitions run in sequence
// with a grid barrier between them, the w-partitions of one s-partition are
// spread over the grid, and a w-partition's batches (runs of up to 64 rows
// of one kind and one wavefront; ts.order / ts.qrng are the plan's) run in
// order.
struct StaticArgs {
  TsArgs ts;
  const int32_t *s_ptr, *w_batch, *batch_ptr;
  int32_t nb;
};

// Standalone CSR SpMV over interleaved blocks (multi-RHS baseline):
// Y = A X, X of n rows and Y of m rows, nblk blocks of kb columns each.
struct SpmvArgs {
  int32_t m, n, kb, nblk;
  const int32_t *Arp, *Aci;
  const void* Av;
  const void* X;
  void* Y;
};

// Fused SpIC0 -> SpTRSV (FP64).
struct Ic0Args {
  int32_t n;
  const int32_t *Lrp, *Lci;
  const double* Aval;      // lower(A) values in the pattern of L
  double* Lval;            // output factor
  const double* B;
  double* X;
  const int32_t *pair_ptr, *pair_u, *pair_q;
  const int32_t* dpos;     // SpILU0: diagonal position of each row (nullptr for SpIC0)
  const int32_t *order, *item_ptr, *item_list;
  const int32_t* qrng;     // SpIC0: per claim position, the row's off-diagonal range (diagonal at its end)
  const int32_t* prng;     // SpIC0: per claim position, the row's range of intersection pairs
  const int32_t* piv;      // SpIC0: per stored entry (i, j), the position of L_jj
  int32_t n_work;
  const int32_t* lvl_item_ptr;  // level-set variant
  int32_t depth;
  int32_t solve;           // 1: also solve L x = b in the same item
  int32_t factor;          // 1: compute the factor (0: solve with a given factor)
  int32_t* d_info;         // written by the last wave (may be nullptr)
  int32_t cached;          // fused SpIC0: 1 = pair values, pivots and x read through the caches first
                           // (re-read device-coherently while pending, as stream.h's VEC = 3)
  unsigned long long* trace;   // optional (fused SpIC0): kTraceItemWords words per item
  unsigned long long* rtrace;  // with trace: per row its publication stamp and count
  LaunchState ls;
};

// Backward: upper solve with L^T fused with c = A^T g and grad_L.
struct BwdArgs {
  int32_t n;
  const int32_t *LTrp, *LTci, *LTmap;
  const int32_t *ATrp, *ATci, *ATmap;
  const int32_t *Lrp, *Lci;
  const void *Lv, *Av, *X, *G;
  void *lam, *gradL;
  const int32_t *order, *item_ptr;
  int32_t n_work;
  const uint8_t* lloc;     // coarsened plan: local wavefront per claim position (else nullptr)
  const uint8_t* eloc;     // coarsened plan: per L^T entry, slot of its column in the item or 0xFF
  LaunchState ls;
};

// Preconditioner apply z = L^{-T} (L^{-1} r): forward items of the SpTRSV
// plan, then backward items of the transposed plan, in one claim sequence.
struct PrecondArgs {
  int32_t n;
  const int32_t *Lci, *LTrp, *LTci, *LTmap;
  const void* Lv;
  const void* R;
  void *W, *Z;             // w = L^{-1} r and z = L^{-T} w (both pending-filled)
  // forward plan (level or coarsened SpTRSV items)
  const int32_t *forder, *fqrng, *fitem_ptr, *fitems;
  int32_t n_fwd;
  const uint8_t *flloc, *feloc;
  // backward plan over L^T
  const int32_t *border, *bitem_ptr;
  int32_t n_bwd;
  const uint8_t *blloc, *beloc;
  LaunchState ls;
};

// Refinement passes (FP64 residual, final product).
// Interleaved blocks: element (j, c) of an n x (nblk * kb) array lives at
// ((c / kb) * n + j) * kb + c % kb, so the kb columns of a block are
// contiguous for each row (the multi-RHS solve keeps its solution so).
struct ResArgs {
  int32_t n, m, nrhs;
  int32_t kb;          // block width of the interleaved arrays = lanes per row
  const int32_t *Lrp, *Lci;
  const double* L64;
  const int32_t *Arp, *Aci;
  const double* A64;
  // Every vector below is in the interleaved block layout of k_layout.hip
  // (a plain vector when kb == 1): n rows, except Y with m rows.
  const double* B;     // right-hand sides
  const double* xin;   // current iterate, nullptr = 0
  const float* d;      // correction to add, nullptr = none
  double* xout;        // new iterate (x + d)
  float* r32;          // residual rounded to FP32 (residual pass); nullptr = not needed
  double* Y;           // final product, nullptr = none
  unsigned long long* maxabs;  // 2 * nrhs: max |r| and max |b| bit patterns
};

// Fused mixed-precision refinement (k_rfused.hip): FP32 substitution, nc
// corrections (FP64 residual, FP32 substitution), final residual norm and
// y = A64 x in one launch over the SpTRSV -> SpMV schedule.
struct RfArgs {
  TsArgs ts;            // schedule, patterns, ts.Lv = L64 values, ts.Av = A64 values, Y;
                        // one RHS: ts.X = x (FP64 output and the SpMV rows' readiness flags),
                        // level items; several: ts.xi = interleaved x, units (ts.unit_rng)
  const float* L32;     // L's values rounded to FP32
  const double* B;      // right-hand sides (one: the vector; several: interleaved blocks)
  unsigned long long* tup;  // stage tuples, rf_tuple_floats(nc) floats per (row, column) in 64-bit
                            // halves (k_rfused.hip), pending-filled
  unsigned long long* maxabs;  // 2 * nrhs: max |b - L64 x| and max |b| bit patterns (zeroed)
  int32_t nrhs;
};
int rf_tuple_floats(int nc);
int occupancy_rfused(int nc, int kb);
hipError_t launch_rfused(const RfArgs& a, int nc, int kb, int grid, hipStream_t st);

// Launchers (return the HIP error of the launch).
hipError_t launch_ts_fused(const TsArgs& a, int dtype, int grid, hipStream_t st);
int occupancy_ts_fused_pre(int dtype);
hipError_t launch_ts_region(const TsArgs& a, const RegionArgs& r, int dtype, int grid, hipStream_t st);
hipError_t launch_ts_multi(const TsArgs& a, int dtype, int kb, int grid, hipStream_t st);
hipError_t launch_pair(const TsArgs& a, int dtype, int mode, int grid, hipStream_t st);
int occupancy_pair(int dtype, int mode);
hipError_t launch_trsv_levelset(const LevelArgs& a, int dtype, int grid, hipStream_t st);  // kb = a.ts.kb
hipError_t launch_spmv(const SpmvArgs& a, int dtype, hipStream_t st);
hipError_t launch_static(const StaticArgs& a, int dtype, int grid, hipStream_t st);
int occupancy_static(int dtype);
// SpMV items of a schedule (a.item_list / a.n_work), all inputs final.
hipError_t launch_spmv_items(const TsArgs& a, int dtype, hipStream_t st);
hipError_t launch_ic0_fused(const Ic0Args& a, int g, int grid, hipStream_t st);
hipError_t launch_ic0_levelset(const Ic0Args& a, int g, int grid, hipStream_t st);
hipError_t launch_bwd(const BwdArgs& a, int dtype, int g, int grid, hipStream_t st);
hipError_t launch_ilu0_fused(const Ic0Args& a, int g, int grid, hipStream_t st);
hipError_t launch_ilu0_levelset(const Ic0Args& a, int g, int grid, hipStream_t st);
int occupancy_ilu0(int g, int levelset);
hipError_t launch_precond(const PrecondArgs& a, int dtype, int grid, hipStream_t st);
int occupancy_precond(int dtype);
// the apply on the forward and the transposed region plans (k_precond_region)
hipError_t launch_precond_region(const PrecondArgs& a, const RegionArgs& rf, const RegionArgs& rb, int dtype,
                                 int grid, hipStream_t st);
int occupancy_precond_region(const RegionArgs& rf, const RegionArgs& rb, int dtype);
hipError_t launch_residual(const ResArgs& a, hipStream_t st);
hipError_t launch_final(const ResArgs& a, hipStream_t st);
// Column-major <-> interleaved block layout (k_layout.hip).  dtype 0 = f64,
// 1 = f32; pack converts f64 -> f32 when asked and fills pend (optional,
// same layout as dst) with the pending pattern.
hipError_t launch_pack(const void* src, int src_dtype, int32_t lds, int32_t rows, int32_t ncols, void* dst,
                       int dst_dtype, void* pend, int kb, hipStream_t st);
hipError_t launch_unpack(const void* src, int dtype, int32_t rows, int32_t ncols, void* dst, int32_t ldd, int kb,
                         hipStream_t st);
// Zero ncols columns of rows entries at p + c * ld (dtype 0 = f64, 1 = f32).
hipError_t launch_zero_cols(void* p, int32_t rows, int32_t ld, int32_t ncols, int dtype, hipStream_t st);
hipError_t launch_convert_f64_f32(const double* src, float* dst, int32_t n, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, int32_t count, hipStream_t st);
// Fill a solution buffer with the pending (not yet published) pattern.
hipError_t launch_fill_pending(void* p, size_t count, int dtype, hipStream_t st);
// The same for the first rows of each of ncols columns of leading dimension ld.
hipError_t launch_fill_pending_cols(void* p, int32_t rows, int32_t ld, int32_t ncols, int dtype, hipStream_t st);


// Fixed device scratch of the allocation-free entry point (scratch.hip):
// its size, and its address on the current device (looked up once per
// device; no allocation).
size_t scratch_bytes();
hipError_t scratch_device_ptr(void** out);

// Occupancy queries per kernel family (blocks per CU).
int occupancy_ts_fused(int dtype);
int occupancy_ts_multi(int dtype, int kb);
int occupancy_trsv_levelset(int dtype, int kb);
int occupancy_ic0(int g, int levelset);
int occupancy_bwd(int dtype, int g);

constexpr int kBlockThreads = 256;  // 4 wavefronts of 64 lanes

}  // namespace sf
