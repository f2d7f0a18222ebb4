// Fused SpIC0 -> SpTRSV executor (FP64) and its level-set baseline.
//
// Row i of the zero fill-in incomplete Cholesky factor (Table 2, comb. 5),
// by the up-looking row recurrence, with P_i the stored columns of row i:
//     L_ij = (A_ij - sum_{k<j, k in P_i and P_j} L_ik L_jk) / L_jj,  j in P_i, j < i
//     L_ii = sqrt(A_ii - sum_{k<i} L_ik^2)
// and, in the same work item (the paper's interleaved packing: F = I, the
// solve of row i needs only factor rows it already reads),
//     x_i = (b_i - sum_{j<i} L_ij x_j) / L_ii.
//
// G lanes per row, lane t owns the t-th off-diagonal entry (rows with more
// than G off-diagonals are rejected by the caller).  The k-intersections
// come from inspector-built lists (u, q): u indexes row i, q is the position
// of L_jk.  Lane t gathers its list into a private LDS row M[t][u] =
// L_{j_t,k_u}; the entries of row i are then resolved in ascending u: the
// lane owning u divides by its pivot L_jj, the value is broadcast inside the
// group, every lane t > u with a pair at u subtracts M[t][u] * L_iu, and the
// row's first lane subtracts L_iu^2 from the pivot and L_iu x_{j_u} from
// b_i -- every term of the recurrences above, rounded once, in their order.
// FP64 results therefore equal the sequential definition's bit for bit.
//
// Readiness (fused launch): the factor values and x are filled with the
// pending pattern before the launch and every value is its own flag; a
// batch of rows issues all its loads (kPairRegs pairs per lane at a time,
// plus the pivots and x values), then waits for the pending ones together
// (dev::wait_ptrs, stream.h).  The level-set baseline reads them after a
// grid barrier instead.
#pragma clang fp contract(off)

#include "stream.h"

namespace sf {
namespace {

using dev::is_pending;
using dev::ld_co;
using dev::poll_value;
using dev::publishable;
using dev::st_co;

// Marker of an absent (u, t) pair in the LDS rows: a signalling NaN with a
// payload no stored factor value can carry (stored values come out of
// arithmetic, which returns NaNs quiet).
constexpr unsigned long long kAbsentBits = 0xFFF4000000000001ull;
constexpr double kAbsent = __builtin_bit_cast(double, kAbsentBits);
__device__ __forceinline__ bool is_absent(double v) {
  return __builtin_bit_cast(unsigned long long, v) == kAbsentBits;
}

// Pairs gathered per lane and round: kPairRegs per lane, G lanes per row.
constexpr int kPairRegs = 8;

// The row, its entry range and its pair range come with the claim position
// and each entry's pivot position with the entry (qrng, prng, piv), so a
// batch issues its index loads in two dependent rounds.  next / next_rg:
// the fused executor's next item, whose range is loaded here once its
// ticket has arrived (it returns before the loads above) and used after
// this item.
// LDS: the rows of one batch row's G lanes form a triangle -- lane t keeps
// M[t][u] for u < t only (a pair's matching entry precedes its own entry) --
// of G (G - 1) / 2 doubles, at group_lds.
template <int G>
constexpr int tri_size() { return G * (G - 1) / 2; }
// A group's LDS: the triangle, then the row's entries L_iu and products
// L_iu x_{j_u} by entry (G each), folded into the pivot and the right-hand
// side after the sweep.
template <int G>
constexpr int grp_size() { return tri_size<G>() + 2 * G; }
constexpr size_t grp_bytes(int g) { return size_t(g * (g - 1) / 2 + 2 * g) * sizeof(double); }
__device__ __forceinline__ int tri_row(int t) { return t * (t - 1) / 2; }

// Lane u of every 16-lane row to the whole row: DPP row_newbcast (a VALU
// move, no LDS round trip), one 32-bit half at a time.
template <int U>
__device__ __forceinline__ double row_bcast16(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(unsigned(b)), 0x150 + U, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(unsigned(b >> 32)), 0x150 + U, 0xf, 0xf, false);
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(unsigned(hi)) << 32) | unsigned(lo));
}

// Lane u (< 32) of every 32-lane group to the whole group: row_newbcast
// of lane u mod 16 inside each 16-lane row, then v_permlane16_swap, which
// exchanges the rows of each pair -- the even row's value for u < 16, the
// odd row's for u >= 16.
template <int U>
__device__ __forceinline__ double row_bcast32(double v) {
  const unsigned long long bits = __builtin_bit_cast(unsigned long long, v);
  int h[2] = {int(unsigned(bits)), int(unsigned(bits >> 32))};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int b = __builtin_amdgcn_update_dpp(0, h[k], 0x150 + (U & 15), 0xf, 0xf, false);
    const auto sw = __builtin_amdgcn_permlane16_swap(b, b, false, false);
    h[k] = int(U < 16 ? sw[0] : sw[1]);
  }
  return __builtin_bit_cast(double, (static_cast<unsigned long long>(unsigned(h[1])) << 32) | unsigned(h[0]));
}

// The value of lane u of the lane's G-lane group (u < G, a constant after
// unrolling).
template <int G>
__device__ __forceinline__ double group_bcast(double v, int u) {
  if constexpr (G == 32) {
    switch (u) {
#define SF_B(U) \
  case U:       \
    return row_bcast32<U>(v);
      SF_B(0) SF_B(1) SF_B(2) SF_B(3) SF_B(4) SF_B(5) SF_B(6) SF_B(7)
      SF_B(8) SF_B(9) SF_B(10) SF_B(11) SF_B(12) SF_B(13) SF_B(14) SF_B(15)
      SF_B(16) SF_B(17) SF_B(18) SF_B(19) SF_B(20) SF_B(21) SF_B(22) SF_B(23)
      SF_B(24) SF_B(25) SF_B(26) SF_B(27) SF_B(28) SF_B(29) SF_B(30) SF_B(31)
#undef SF_B
      default:
        return v;
    }
  } else if constexpr (G == 16) {
    switch (u) {
#define SF_B(U) \
  case U:       \
    return row_bcast16<U>(v);
      SF_B(0) SF_B(1) SF_B(2) SF_B(3) SF_B(4) SF_B(5) SF_B(6) SF_B(7)
      SF_B(8) SF_B(9) SF_B(10) SF_B(11) SF_B(12) SF_B(13) SF_B(14) SF_B(15)
#undef SF_B
      default:
        return v;
    }
  } else {
    return __shfl(v, u, G);
  }
}

// Trace mode (fused launch, tr = the item's record): tr[1] once the
// batch's index loads have returned, tr[2] once its last round of values
// is final, tr[5] after the sweep, tr[6] after the pivot fold, tr[3] after
// its stores (the last batch's stamps stay); per row, the stamp taken just
// before its first store and its publication count.
// The fused executor's hand-over between consecutive items of a wavefront:
// the next ticket's claim atomic (raw, issued before the item runs), then
// the next ticket t and its claim-position range rg, and the next item's
// first row indices of this lane (row id, off-diagonal range, pair range),
// each loaded while the current item waits for something else anyway.
struct Ic0Next {
  int32_t raw;
  int t;
  int2 rg;
  bool have;  // i, qr, pr hold the current item's row indices
  int i;
  int2 qr, pr;
};

template <int G, bool FUSED>
__device__ __forceinline__ void ic0_rows(const Ic0Args& a, int q0, int q1, int lane, double* group_lds,
                                         unsigned long long* tr = nullptr, Ic0Next* nx = nullptr) {
  constexpr int RPB = 64 / G;
  const int sub = lane & (G - 1);
  double* lds_row = group_lds + tri_row(sub);
  const int32_t par = a.ls.epoch & 1;
  for (int base = q0; base < q1; base += RPB) {
    const int q = base + lane / G;
    const bool act = q < q1;
    const bool pre = nx && nx->have && base == q0;
    const int i = pre ? nx->i : act ? a.order[q] : 0;
    const int2 rg = pre ? nx->qr : act ? reinterpret_cast<const int2*>(a.qrng)[q] : make_int2(0, 0);
    // the pairs of row i are contiguous: every entry's list, in entry order
    const int2 pr = pre ? nx->pr : act ? reinterpret_cast<const int2*>(a.prng)[q] : make_int2(0, 0);
    const int r0 = rg.x, rd = rg.y;              // off-diagonals [r0, rd); the diagonal at rd
    const int len = rd - r0;                     // off-diagonal entries (<= G)
    const bool mine = act && sub < len;
    const int p = r0 + sub;
    const int j = mine ? a.Lci[p] : 0;
    const int pjj = mine ? a.piv[p] : 0;
    const int e0 = pr.x, e1 = pr.y;
    double acc = mine ? a.Aval[p] : 0.0;
    // pivot and right-hand side of the row, on its first lane (loaded with
    // the indices: they wait for nothing)
    double d = (act && sub == 0) ? a.Aval[rd] : 1.0;
    double s = (act && sub == 0 && a.solve) ? a.B[i] : 0.0;
    if (nx && base == q0) {
      // the next ticket (its atomic has been in flight since before this
      // item) and its range: waited for while this item's loads are out
      nx->t = dev::claim_ticket(a.ls, nx->raw);
      nx->rg = nx->t < a.n_work ? make_int2(a.item_ptr[nx->t], a.item_ptr[nx->t + 1]) : make_int2(0, 0);
    }
    // M[t][u] = L_{j_t, k_u} where row j_t meets row i below column j_t, else absent
    for (int u = 0; u < G; ++u)
      if (u < sub) lds_row[u] = kAbsent;
    __builtin_amdgcn_wave_barrier();
    // Rounds of kPairRegs pairs per lane; the pivot L_jj and x_j of the
    // lane's entry ride along in the first round.  Every load of a round is
    // issued before any is waited on.
    // (further rounds while any row of the batch has pairs left: a ballot)
    double djj = 1.0, xj = 0.0;
    for (int rnd = 0; rnd == 0 || __ballot(e0 + rnd * G * kPairRegs < e1) != 0; ++rnd) {
      constexpr int R = kPairRegs + 2;
      const double* ptr[R];
      double v[R];
      int tu[kPairRegs], tq[kPairRegs];
      // the round's index loads all go out, unconditionally (a list's end
      // position is valid: the lists end with a sentinel), before any
      // address is formed
#pragma unroll
      for (int k = 0; k < kPairRegs; ++k) {
        const int e = e0 + rnd * G * kPairRegs + sub + G * k;
        const int ec = e < e1 ? e : e1;
        tu[k] = a.pair_u[ec];
        tq[k] = a.pair_q[ec];
      }
#pragma unroll
      for (int k = 0; k < kPairRegs; ++k) {
        const int e = e0 + rnd * G * kPairRegs + sub + G * k;
        if (e >= e1) tu[k] = -1;
        ptr[k] = e < e1 ? a.Lval + tq[k] : nullptr;
      }
      ptr[kPairRegs] = (rnd == 0 && mine) ? a.Lval + pjj : nullptr;
      ptr[kPairRegs + 1] = (rnd == 0 && mine && a.solve) ? a.X + j : nullptr;
      if (FUSED && tr && rnd == 0) {
        // the index loads have returned once their values are in registers
        __asm__ volatile("" ::"v"(tu[0]), "v"(pjj), "v"(j));
        if (lane == 0) tr[1] = __builtin_amdgcn_s_memrealtime();
      }
      // (cached first: a cached read returns the value or the pending
      // pattern -- a value changes once per launch and every launch starts
      // with the caches invalidated -- and wait_ptrs re-reads pending ones
      // device-coherently)
      if (FUSED && a.cached) {
#pragma unroll
        for (int e = 0; e < R; ++e) v[e] = ptr[e] ? *ptr[e] : 0.0;
      } else {
#pragma unroll
        for (int e = 0; e < R; ++e) v[e] = ptr[e] ? ld_co(ptr[e]) : 0.0;
      }
      if (nx && base == q0 && rnd == 0) {
        // the next item's row indices, in flight with this item's values
        const int qn = nx->rg.x + lane / G;
        const bool an = qn < nx->rg.y;
        nx->i = an ? a.order[qn] : 0;
        nx->qr = an ? reinterpret_cast<const int2*>(a.qrng)[qn] : make_int2(0, 0);
        nx->pr = an ? reinterpret_cast<const int2*>(a.prng)[qn] : make_int2(0, 0);
      }
      if constexpr (FUSED) dev::wait_ptrs<double, R, 64>(ptr, v, lane, a.ls);
      if (FUSED && tr && lane == 0) tr[2] = __builtin_amdgcn_s_memrealtime();
#pragma unroll
      for (int k = 0; k < kPairRegs; ++k)
        if (tu[k] >= 0) group_lds[tri_row(tu[k] >> 16) + (tu[k] & 0xffff)] = v[k];
      if (rnd == 0 && mine) {
        djj = v[kPairRegs];
        if (a.solve) xj = v[kPairRegs + 1];
      }
    }
    __builtin_amdgcn_wave_barrier();
    // the lane's row of M into registers first (one round of LDS reads;
    // entries u >= sub are not its own and stay unused -- the last lane's
    // row ends where the group's entry array starts, so every read is in
    // the group's LDS)
    double mrow[G];
#pragma unroll
    for (int u = 0; u < G; ++u) mrow[u] = lds_row[u];
    double l = 0.0;
#pragma unroll
    for (int u = 0; u < G; ++u) {
      if (__ballot(act && u < len) == 0) break;  // past the batch's longest row
      if (sub == u && mine) l = acc / djj;  // entry u is final: every k < j_u has been subtracted
      const double lu = group_bcast<G>(l, u);
      if (mine && sub > u && !is_absent(mrow[u])) acc = acc - mrow[u] * lu;
    }
    if (FUSED && tr && lane == 0) tr[5] = __builtin_amdgcn_s_memrealtime();
    // the pivot and the right-hand side fold the row's entries in order, on
    // its first lane, off the sweep's chain
    double* lv = group_lds + tri_size<G>();
    double* pv = lv + G;
    if (mine) {
      lv[sub] = l;
      pv[sub] = l * xj;
    }
    __builtin_amdgcn_wave_barrier();
    if (act && sub == 0) {
      // every slot read at once (slots past the row's end hold stale values:
      // they enter as 0, and d - 0 * 0 and s - 0 leave d and s unchanged)
      double lu[G], pu[G];
#pragma unroll
      for (int u = 0; u < G; ++u) {
        lu[u] = lv[u];
        pu[u] = pv[u];
      }
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const double x = u < len ? lu[u] : 0.0;
        d = d - x * x;
        s = s - (u < len ? pu[u] : 0.0);
      }
    }
    if (FUSED && tr && lane == 0) tr[6] = __builtin_amdgcn_s_memrealtime();
    if (FUSED && a.rtrace) dev::stamp_publish(a.rtrace, act && sub == 0, i);
    if (mine) st_co(a.Lval + p, publishable(l));
    if (act && sub == 0) {
      const double lii = sqrt(d);
      if (!(d > 0.0))
        __hip_atomic_fetch_min(a.ls.state + info_off(par), i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      st_co(a.Lval + rd, publishable(lii));
      if (a.solve) st_co(a.X + i, publishable(s / lii));
    }
    if (FUSED && tr && lane == 0) tr[3] = __builtin_amdgcn_s_memrealtime();
  }
}

__device__ __forceinline__ void write_info(const Ic0Args& a, int lane) {
  if (!a.d_info) return;
  if (dev::last_wave_done(a.ls, lane) && lane == 0) {
    const int32_t v = __hip_atomic_load(a.ls.state + info_off(a.ls.epoch & 1), __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
    *a.d_info = (v >= a.n) ? -1 : v;
  }
}

template <int G>
__global__ __launch_bounds__(kBlockThreads) void k_ic0_fused(Ic0Args a) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63;
  double* group_lds = lds + size_t(threadIdx.x / G) * grp_size<G>();
  dev::reset_next_launch(a.ls);
  // every item, in claim order (no item list): the next ticket's atomic
  // goes out before an item runs; the ticket, its range and its rows'
  // indices are loaded inside the item (ic0_rows, Ic0Next)
  int t = dev::claim(a.ls, lane);
  int2 rg = t < a.n_work ? make_int2(a.item_ptr[t], a.item_ptr[t + 1]) : make_int2(0, 0);
  Ic0Next nx{};
  nx.have = false;
  while (t < a.n_work) {
    unsigned long long* tr = a.trace ? a.trace + size_t(t) * kTraceItemWords : nullptr;
    if (tr && lane == 0) {
      const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
      tr[0] = t0;
      tr[1] = t0;
      tr[2] = t0;
      atomicAdd(tr + 4, 1ull);
    }
    nx.raw = dev::claim_issue(a.ls, lane);
    ic0_rows<G, true>(a, rg.x, rg.y, lane, group_lds, tr, &nx);
    nx.have = true;
    t = nx.t;
    rg = nx.rg;
  }
  write_info(a, lane);
}

template <int G>
__global__ __launch_bounds__(kBlockThreads) void k_ic0_levelset(Ic0Args a) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63;
  double* group_lds = lds + size_t(threadIdx.x / G) * grp_size<G>();
  dev::reset_next_launch(a.ls);
  const int wave = int(blockIdx.x) * (kBlockThreads / 64) + int(threadIdx.x >> 6);
  const int nwaves = int(gridDim.x) * (kBlockThreads / 64);
  int32_t gen = 0;
  for (int lv = 0; lv < a.depth; ++lv) {
    for (int t = a.lvl_item_ptr[lv] + wave; t < a.lvl_item_ptr[lv + 1]; t += nwaves) {
      const int it = a.item_list[t];
      ic0_rows<G, false>(a, a.item_ptr[it], a.item_ptr[it + 1], lane, group_lds);
    }
    if (lv + 1 < a.depth) dev::grid_barrier(a.ls, gen);
  }
  write_info(a, lane);
}

template <typename K>
int occ(K kernel, size_t lds) {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void*>(kernel),
                                                   kBlockThreads, lds) != hipSuccess)
    return 1;
  return b < 1 ? 1 : b;
}

}  // namespace

hipError_t launch_ic0_fused(const Ic0Args& a, int g, int grid, hipStream_t st) {
  if (!a.order || !a.item_ptr || a.item_list || !a.qrng || !a.prng || !a.piv || !a.pair_u || !a.pair_q)
    return hipErrorInvalidValue;
  const size_t lds = size_t(kBlockThreads / g) * grp_bytes(g);
#define SF_IC(G)                                                                    \
  if (g == G) {                                                                     \
    hipLaunchKernelGGL((k_ic0_fused<G>), dim3(grid), dim3(kBlockThreads), lds, st, a); \
    return hipGetLastError();                                                       \
  }
  SF_IC(4) SF_IC(8) SF_IC(16) SF_IC(32) SF_IC(64)
#undef SF_IC
  return hipErrorInvalidValue;
}

hipError_t launch_ic0_levelset(const Ic0Args& a, int g, int grid, hipStream_t st) {
  if (!a.order || !a.item_ptr || !a.item_list || !a.lvl_item_ptr || !a.qrng || !a.prng || !a.piv)
    return hipErrorInvalidValue;
  const size_t lds = size_t(kBlockThreads / g) * grp_bytes(g);
  void* args[] = {const_cast<Ic0Args*>(&a)};
#define SF_IL(G)                                                                               \
  if (g == G)                                                                                  \
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_ic0_levelset<G>), dim3(grid), \
                                      dim3(kBlockThreads), args, lds, st);
  SF_IL(4) SF_IL(8) SF_IL(16) SF_IL(32) SF_IL(64)
#undef SF_IL
  return hipErrorInvalidValue;
}

int occupancy_ic0(int g, int levelset) {
  const size_t lds = size_t(kBlockThreads / g) * grp_bytes(g);
  switch (g) {
    case 4: return levelset ? occ(k_ic0_levelset<4>, lds) : occ(k_ic0_fused<4>, lds);
    case 8: return levelset ? occ(k_ic0_levelset<8>, lds) : occ(k_ic0_fused<8>, lds);
    case 16: return levelset ? occ(k_ic0_levelset<16>, lds) : occ(k_ic0_fused<16>, lds);
    case 32: return levelset ? occ(k_ic0_levelset<32>, lds) : occ(k_ic0_fused<32>, lds);
    default: return levelset ? occ(k_ic0_levelset<64>, lds) : occ(k_ic0_fused<64>, lds);
  }
}

}  // namespace sf
