// Fused SpTRSV -> SpMV executor on the region plan (gfx950).
//
// A region is a set of up to a few hundred SpTRSV rows grown around a seed
// (inspect.cpp, build_regions), run by one wavefront: the region's row data
// (right-hand sides, diagonals, the values and in-region codes of the
// off-diagonals) are staged into LDS when it is claimed, then its local
// wavefronts run in order in batches of up to 64 rows, one row per lane.  A
// row's in-region inputs are read from the region's x in LDS; its inputs
// from other regions through the readiness protocol, waited for by that row
// only, so a region starts as soon as its first rows' inputs exist and runs
// alongside the regions it depends on (a pipeline along the DAG) instead of
// waiting for all its inputs first.  The inputs from other regions are
// fetched ahead: each batch issues the loads of the inputs first used kAhead
// batches later, so a value published some time before it is needed costs
// no round trip; a value still pending when needed is polled.  Each row
// folds its terms in ascending column order and divides by its diagonal --
// the sequential definition's arithmetic, so results are bit-identical to
// forward substitution.  SpMV rows run as the fused executor's items
// (entry stream, x read through the caches first).
// No multiply-add contraction in this file.
#pragma clang fp contract(off)

#include "ts_items.h"

namespace sf {
namespace {

using dev::is_pending;
using dev::ld_co;
using dev::publishable;
using dev::st_co;

constexpr int kAhead = 4;  // batches between issuing an input's load and its first use

// The region's LDS, carved from the dynamic allocation (sizes: the largest
// region's rows R, entries E and external inputs X; region_lds_bytes).
template <typename T>
struct RegionLds {
  T *x, *b, *dii, *ev, *xv;
  int32_t *ids, *eoff, *xc, *bt;
  uint16_t* ec;
};

// Layout (region_lds_bytes): x, b, dii [R]; entry values [E]; external
// values [X]; ids [R]; entry offsets [R + 1]; external columns [X]; batch
// table [2 (NB + 1)]; entry codes [E].
template <typename T>
__device__ __forceinline__ RegionLds<T> carve(char* base, int R, int E, int X, int NB) {
  RegionLds<T> L;
  T* tp = reinterpret_cast<T*>(base);
  L.x = tp;
  L.b = tp + R;
  L.dii = tp + 2 * R;
  L.ev = tp + 3 * R;
  L.xv = tp + 3 * R + E;
  int32_t* ip = reinterpret_cast<int32_t*>(tp + 3 * R + E + X);
  L.ids = ip;
  L.eoff = ip + R;
  L.xc = ip + 2 * R + 1;
  L.bt = ip + 2 * R + 1 + X;
  L.ec = reinterpret_cast<uint16_t*>(ip + 2 * R + 1 + X + 2 * (NB + 1));
  return L;
}

template <typename T>
__device__ __forceinline__ T pending_value() {
  return __builtin_bit_cast(T, dev::Pending<T>::bits);
}

// One region (item `item`, claim positions [q0, q1), batches [b0, b1)).
template <typename T>
__device__ void region_rows(const TsArgs& a, const RegionArgs& r, int item, int q0, int q1, int b0, int b1,
                            int lane, char* lds, unsigned long long* tr) {
  const RegionLds<T> L = carve<T>(lds, r.rows_max, r.entries_max, r.ext_max, r.batches_max);
  const T* __restrict__ Lv = static_cast<const T*>(a.Lv);
  const T* __restrict__ B = static_cast<const T*>(a.B);
  T* X = static_cast<T*>(a.X);
  const int nr = q1 - q0;
  const int x0 = r.ext_ptr[item];
  const int nx = r.ext_ptr[item + 1] - x0;
  // stage the region's rows and entries (independent loads, one round trip)
  for (int k = lane; k < nr; k += 64) {
    const int id = a.order[q0 + k];
    const int2 rg = reinterpret_cast<const int2*>(a.qrng)[q0 + k];
    const int eo = r.roff[q0 + k];
    L.ids[k] = id;
    L.b[k] = B[id];
    L.dii[k] = dev::ld_stream(Lv + rg.y);
    L.eoff[k] = eo;
    for (int p = rg.x; p < rg.y; ++p) {
      L.ev[eo + p - rg.x] = dev::ld_stream(Lv + p);
      L.ec[eo + p - rg.x] = r.code[p];
    }
    if (k == nr - 1) L.eoff[nr] = eo + (rg.y - rg.x);
  }
  for (int k = lane; k < nx; k += 64) {
    L.xc[k] = r.ext[x0 + k];
    L.xv[k] = pending_value<T>();
  }
  // batch table, relative to the region: first position, first external input
  for (int k = lane; k < b1 - b0; k += 64) {
    L.bt[2 * k] = r.batch[2 * (b0 + k)] - q0;
    L.bt[2 * k + 1] = r.batch[2 * (b0 + k) + 1];
  }
  if (lane == 0) {
    L.bt[2 * (b1 - b0)] = nr;
    L.bt[2 * (b1 - b0) + 1] = nx;
  }
  // LDS accesses of one wavefront complete in order: once the barrier keeps
  // the compiler from moving reads above these writes, every lane sees them
  __builtin_amdgcn_wave_barrier();
  // first-use ranges of the external inputs: batch b uses [xs(b), xs(b + 1))
  auto xs = [&](int b) { return L.bt[2 * (b < b1 ? b - b0 : b1 - b0) + 1]; };
  // loads ahead: slot u holds the inputs of batch bb + u
  int ridx[kAhead];
  T rval[kAhead];
#pragma unroll
  for (int u = 0; u < kAhead; ++u) {
    const int b = b0 + u;
    ridx[u] = -1;
    rval[u] = T(0);
    if (b < b1) {
      const int k = xs(b) + lane;
      if (k < xs(b + 1)) {
        ridx[u] = k;
        rval[u] = ld_co(X + L.xc[k]);
      }
    }
  }
  for (int bb = b0; bb < b1; bb += kAhead) {
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
      const int b = bb + u;
      if (b >= b1) break;
      // this batch's prefetched inputs into LDS (pending ones are polled below)
      if (ridx[u] >= 0) L.xv[ridx[u]] = rval[u];
      // inputs of batch b + kAhead
      ridx[u] = -1;
      if (b + kAhead < b1) {
        const int k = xs(b + kAhead) + lane;
        if (k < xs(b + kAhead + 1)) {
          ridx[u] = k;
          rval[u] = ld_co(X + L.xc[k]);
        }
      }
      __builtin_amdgcn_wave_barrier();
      const int pb = L.bt[2 * (b - b0)];
      const int pe = L.bt[2 * (b - b0 + 1)];
      const int k = pb + lane;
      const bool mine = lane < pe - pb;
      const int t0 = mine ? L.eoff[k] : 0, t1 = mine ? L.eoff[k + 1] : 0;
      // wait for this row's inputs from other regions
      int32_t spins = 0;
      for (;;) {
        bool pend = false;
        for (int t = t0; t < t1; ++t) {
          const int code = L.ec[t];
          if (code & 0x8000) {
            const int xi = code & 0x7fff;
            if (is_pending(L.xv[xi])) {
              const T v = ld_co(X + L.xc[xi]);
              if (is_pending(v)) pend = true;
              else L.xv[xi] = v;
            }
          }
        }
        if (__ballot(pend) == 0) break;
        if (!dev::all_poll_round(spins, a.ls)) break;
      }
      if (tr && lane == 0) tr[2] = __builtin_amdgcn_s_memrealtime();
      __builtin_amdgcn_wave_barrier();
      if (mine) {
        T acc = L.b[k];
        for (int t = t0; t < t1; ++t) {
          const int code = L.ec[t];
          const T xj = (code & 0x8000) ? L.xv[code & 0x7fff] : L.x[code];
          acc = acc - L.ev[t] * xj;
        }
        const T xk = publishable(acc / L.dii[k]);
        L.x[k] = xk;
        if (a.rtrace) dev::stamp_publish(a.rtrace, true, L.ids[k]);
        st_co(X + L.ids[k], xk);
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// Claim loop, one wavefront per block: regions in topological order, SpMV
// items after them.  With col_units > 1, ticket t is column t % col_units
// of item t / col_units (one chain of the items per right-hand side).
template <typename T>
__global__ __launch_bounds__(64) void k_ts_region(TsArgs a, RegionArgs r) {
  extern __shared__ __align__(16) char lds[];
  const int lane = threadIdx.x;
  dev::reset_next_launch(a.ls);
  const int nc = a.col_units > 1 ? a.col_units : 1;
  const int total = a.n_work * nc;
  int t = dev::claim(a.ls, lane);
  while (t < total) {
    const int tn = dev::claim(a.ls, lane);
    const int u = t / nc, c = t - u * nc;
    const int item = a.item_list ? a.item_list[u] : u;
    TsArgs ac = a;
    if (nc > 1) {
      ac.B = static_cast<const T*>(a.B) + size_t(c) * size_t(a.ldb);
      ac.X = static_cast<T*>(a.X) + size_t(c) * size_t(a.ldx);
      if (a.Y) ac.Y = static_cast<T*>(a.Y) + size_t(c) * size_t(a.ldy);
    }
    const int q0 = a.item_ptr[item], q1 = a.item_ptr[item + 1];
    const int bt0 = r.batch_ptr[item], bt1 = r.batch_ptr[item + 1];
    unsigned long long* tr = (a.trace && item >= 0) ? a.trace + size_t(item) * kTraceItemWords : nullptr;
    if (tr && lane == 0) {
      const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
      tr[0] = t0;
      tr[1] = t0;
      tr[2] = t0;
      atomicAdd(tr + 4, 1ull);
    }
    if (bt1 > bt0) {
      region_rows<T>(ac, r, item, q0, q1, bt0, bt1, lane, lds, tr);
      if (tr && lane == 0) tr[3] = __builtin_amdgcn_s_memrealtime();
    } else {
      const bool mine = lane < q1 - q0;
      const int id = mine ? a.order[q0 + lane] : 0;
      const int2 rg = mine ? reinterpret_cast<const int2*>(a.qrng)[q0 + lane] : make_int2(0, 0);
      item_stream_rows<T, false, 3>(ac, q0, q1, lane, *reinterpret_cast<dev::WaveLds<T>*>(lds), tr, id, rg);
    }
    t = tn;
  }
}

template <typename K>
int occ64(K kernel, size_t lds) {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void*>(kernel), 64, lds) != hipSuccess)
    return 1;
  return b < 1 ? 1 : b;
}

}  // namespace

size_t region_kernel_lds(const RegionArgs& r, int dtype) {
  const int vb = dtype == 0 ? 8 : 4;
  const size_t reg = region_lds_bytes(r.rows_max, r.entries_max, r.ext_max, r.batches_max, vb);
  const size_t sp = dtype == 0 ? sizeof(dev::WaveLds<double>) : sizeof(dev::WaveLds<float>);
  return reg > sp ? reg : sp;
}

int occupancy_region(const RegionArgs& r, int dtype) {
  const size_t lds = region_kernel_lds(r, dtype);
  return dtype == 0 ? occ64(k_ts_region<double>, lds) : occ64(k_ts_region<float>, lds);
}

hipError_t launch_ts_region(const TsArgs& a, const RegionArgs& r, int dtype, int grid, hipStream_t st) {
  if (!a.order || !a.qrng || !a.item_ptr || !r.batch || !r.batch_ptr || !r.ext_ptr || !r.roff || !r.code)
    return hipErrorInvalidValue;
  const size_t lds = region_kernel_lds(r, dtype);
  if (dtype == 0) hipLaunchKernelGGL(k_ts_region<double>, dim3(grid), dim3(64), lds, st, a, r);
  else hipLaunchKernelGGL(k_ts_region<float>, dim3(grid), dim3(64), lds, st, a, r);
  return hipGetLastError();
}

}  // namespace sf
