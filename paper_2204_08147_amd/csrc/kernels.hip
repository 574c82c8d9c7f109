// gfx950 kernels of the typicality RDM solver.
//
// Data layout ("panels"): a block of C columns over dim rows is stored as
// P = cpad / W panels of W = 16 / sizeof(T) columns; panel p is a dim x W
// row-major array, so one row of a panel is 16 bytes and a wave64 reading 64
// consecutive rows of one panel reads 1 KiB contiguous.  A gathered partner
// row idx ^ f of 64 consecutive rows is again an aligned 64-row block, so
// every gather of the spin-Hamiltonian apply is a fully coalesced 1 KiB read.
//
// Every kernel takes a table of segments (independent Lanczos problems) and
// a table of tiles, so a single launch advances any mix of instances of
// different sizes and at different steps (batched solves, serving).
#include "internal.h"

namespace rdm {

template <typename T> struct PanelT;
template <> struct PanelT<float> {
  typedef float V __attribute__((ext_vector_type(4)));
  static constexpr int W = 4;
};
template <> struct PanelT<double> {
  typedef double V __attribute__((ext_vector_type(2)));
  static constexpr int W = 2;
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// SplitMix64 output from state x (Steele, Lea & Flood 2014).
__device__ __forceinline__ uint64_t sm64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Rademacher sign bit of bath vector j at bath index b.
__device__ __forceinline__ uint32_t bath_bit(uint64_t seed, uint32_t j, uint64_t b) {
  const uint64_t key = sm64(seed ^ sm64((uint64_t)j));
  const uint64_t word = sm64(key ^ (b >> 6));
  return (uint32_t)((word >> (b & 63)) & 1ull);
}

template <typename T> __device__ __forceinline__ T amp_of(int nb);
template <> __device__ __forceinline__ double amp_of<double>(int nb) { return sqrt(ldexp(1.0, -nb)); }
template <> __device__ __forceinline__ float amp_of<float>(int nb) { return sqrtf(ldexpf(1.0f, -nb)); }

// The system factor of product start vector j follows the bath-vector rule
// with this seed offset, over the n_s system bits.
constexpr uint64_t kSysSeedXor = 0x9E3779B97F4A7C15ull;

// Start-block entry (row, column c): |m> (x) |v_j> with c = j*d_s + m
// (START_SYSBATH), the product |v_s^(c)> (x) |v_c> (START_PRODUCT), or v_c.
// amp = 2^(-nb/2).
template <typename T>
__device__ __forceinline__ T start_value(int kind, int ns_log, int nb, uint64_t seed, uint32_t row,
                                         int c, int C, T amp) {
  if (c >= C) return T(0);
  uint32_t j, b;
  if (kind == START_SYSBATH) {
    const int m = c & ((1 << ns_log) - 1);
    j = (uint32_t)(c >> ns_log);
    if ((int)(row >> nb) != m) return T(0);
    b = row & ((1u << nb) - 1u);
  } else if (kind == START_PRODUCT) {
    const uint32_t m = row >> nb;
    b = row & ((1u << nb) - 1u);
    const T a = amp * amp_of<T>(ns_log);
    return (bath_bit(seed, (uint32_t)c, b) ^ bath_bit(seed ^ kSysSeedXor, (uint32_t)c, m)) ? -a : a;
  } else {
    j = (uint32_t)c;
    b = row;
  }
  return bath_bit(seed, j, b) ? -amp : amp;
}

#define GLOBAL_AS __attribute__((address_space(1)))
#define CONST_AS __attribute__((address_space(4)))

// 16-byte panel access in the global address space with a uniform base and a
// 32-bit row offset, so the compiler emits global loads/stores with an SGPR
// base and a VGPR offset.
template <typename V>
__device__ __forceinline__ V ldg(const V* base, uint32_t row) {
  return *(const GLOBAL_AS V*)((const GLOBAL_AS char*)base + (uint32_t)(row << 4));
}
template <typename V>
__device__ __forceinline__ void stg(V* base, uint32_t row, V v) {
  *(GLOBAL_AS V*)((GLOBAL_AS char*)base + (uint32_t)(row << 4)) = v;
}
// Streaming forms: a transform pass reads every vector once and its working
// set is several times the last-level cache, so loads carry the nontemporal
// hint.  Stores of the block R take it too; the basis vector written in the
// norm step (read again within the step) and the plain apply's first pass
// keep ordinary stores, which measured faster.  The hop-table kernels use
// the same forms for their pure streams (r and u_{j-1}), not for the partner
// tiles that neighbouring workgroups share.
template <typename V>
__device__ __forceinline__ V ldg_nt(const V* base, uint32_t row) {
  return __builtin_nontemporal_load((const GLOBAL_AS V*)((const GLOBAL_AS char*)base + (uint32_t)(row << 4)));
}
template <bool NT, typename V>
__device__ __forceinline__ void stg_stream(V* base, uint32_t row, V v) {
  GLOBAL_AS V* p = (GLOBAL_AS V*)((GLOBAL_AS char*)base + (uint32_t)(row << 4));
  if (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}
template <typename T>
__device__ __forceinline__ T ldg_s(const T* base, uint32_t row) {
  return ((const GLOBAL_AS T*)base)[row];
}
// Strided transform tiles whose row runs are shorter than a cache line share
// lines with their neighbours (which run on the same XCD): there the hint
// would evict lines before the neighbours use them, so NT is false.  The
// choice is a template parameter: a run-time select around every access
// costs the common case about 8 %.
template <bool NT, typename V>
__device__ __forceinline__ V ldg_sel(const V* base, uint32_t row) {
  if constexpr (NT) return ldg_nt(base, row);
  else return ldg(base, row);
}
template <bool NT, typename V>
__device__ __forceinline__ void stg_sel(V* base, uint32_t row, V v) {
  if constexpr (NT) stg_stream<true>(base, row, v);
  else stg(base, row, v);
}

// Segment descriptors are read-only during a kernel: read them through the
// constant address space so uniform fields come in with scalar loads.
typedef Seg CSeg;
__device__ __forceinline__ const CONST_AS CSeg& cseg(const Seg* segs, int i) {
  return ((const CONST_AS CSeg*)segs)[i];
}

__device__ __forceinline__ float fma_s(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_s(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename V>
__device__ __forceinline__ V fma_v(V a, V b, V c) {
  V r;
#pragma unroll
  for (int e = 0; e < (int)(sizeof(V) / sizeof(a[0])); ++e) r[e] = fma_s(a[e], b[e], c[e]);
  return r;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum NV per-lane values over the workgroup in a fixed tree; threads 0..NV-1
// receive the totals.  lds: 4*NV doubles.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds, double* tot) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) lds[wave * NV + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    const int t = threadIdx.x;
    *tot = ((lds[t] + lds[NV + t]) + lds[2 * NV + t]) + lds[3 * NV + t];
  }
}

// Sum the lane values v over the workgroup and store them at plane `plane`
// (XP_*), row tile rt, columns panel0 * W .. + W - 1, times scale.
template <int W>
__device__ __forceinline__ void put_plane(const CONST_AS Seg& sg, int plane, int rt, int panel0, double (&v)[W],
                                          double* red, double scale = 1.0) {
  double tot;
  block_sum<W>(v, red, &tot);
  if (threadIdx.x < W)
    sg.part[((uint64_t)plane * sg.x_tiles + rt) * sg.cpad + panel0 * W + threadIdx.x] = tot * scale;
}

// per-column scalars of the recurrence for panel s of a tile (uniform loads)
template <typename T, int S>
__device__ __forceinline__ typename PanelT<T>::V scur_of(const CONST_AS double* st, int cp, int panel0,
                                                         int s, bool plain) {
  typename PanelT<T>::V v;
#pragma unroll
  for (int e = 0; e < PanelT<T>::W; ++e)
    v[e] = plain ? T(1) : (T)st[ST_SCUR * cp + (panel0 + s) * PanelT<T>::W + e];
  return v;
}
template <typename T, int S>
__device__ __forceinline__ typename PanelT<T>::V bps_of(const CONST_AS double* st, int cp, int panel0,
                                                        int s) {
  typename PanelT<T>::V v;
#pragma unroll
  for (int e = 0; e < PanelT<T>::W; ++e) v[e] = (T)st[ST_BPS * cp + (panel0 + s) * PanelT<T>::W + e];
  return v;
}

// The tile of this workgroup: binary search of blockIdx.x in the segments'
// tile_base offsets (uniform, scalar loads), then slab-major inside the
// segment so the workgroups in flight share one group of panels.
template <bool APPLY>
__device__ __forceinline__ Tile tile_of(const Seg* segs, int nseg) {
  const CONST_AS Seg* cs = (const CONST_AS Seg*)segs;
  const int b = (int)blockIdx.x;
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((APPLY ? cs[mid].ap_base : cs[mid].tile_base) <= b) lo = mid;
    else hi = mid - 1;
  }
  const int lt = b - (APPLY ? cs[lo].ap_base : cs[lo].tile_base);
  const int nrt = cs[lo].n_row_tiles;
  const int sl = lt / nrt, rt = lt - sl * nrt;
  return Tile{lo, (uint32_t)rt * (uint32_t)kBlock, sl * cs[lo].S, rt};
}

template <typename T>
__device__ __forceinline__ T* slot_ptr(const CONST_AS Seg& sg, int j) {
  const int idx = sg.ring ? ((j - 1) & 1) : (j - 1);
  return (T*)sg.Q + (uint64_t)idx * sg.blk;
}

// ---------------------------------------------------------------------------
// diagonal of H: sum_t c_t (1 - 2 parity(idx & mask_t)), accumulated in FP64
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_diag(const DiagTerm* __restrict__ terms, int nt,
                                                 T* __restrict__ diag, uint32_t dim, int tiled_lrb) {
  const uint32_t e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= dim) return;
  // tiled_lrb >= 0: entries in the order of the transform's strided tiles
  // (entry rt * 4096 + tau holds the row ((tau >> lrb) << 12) | (rt << lrb) |
  // (tau mod 2^lrb)), so each tile reads one contiguous 4096-entry block
  uint32_t row = e;
  if (tiled_lrb >= 0) {
    const uint32_t tau = e & ((1u << kXzTileBits) - 1u), rt = e >> kXzTileBits;
    row = ((tau >> tiled_lrb) << kXzTileBits) | (rt << tiled_lrb) | (tau & ((1u << tiled_lrb) - 1u));
  }
  double d = 0.0;
  for (int t = 0; t < nt; ++t) {
    const uint32_t par = __builtin_popcount(row & terms[t].mask) & 1u;
    d += par ? -terms[t].c : terms[t].c;
  }
  diag[e] = (T)d;
}

// ---------------------------------------------------------------------------
// state initialisation: phase 0 = fresh Lanczos run, 1 = regeneration pass
// ---------------------------------------------------------------------------
__global__ void k_init_state(const Seg* __restrict__ segs, int phase) {
  const Seg& sg = segs[blockIdx.x];
  const int c = blockIdx.y * 64 + threadIdx.x;
  if (c >= sg.cpad) return;
  const int cp = sg.cpad;
  for (int i = 0; i < ST_COUNT; ++i) sg.st[i * cp + c] = 0.0;
  sg.st[ST_FROZEN * cp + c] = (c >= sg.C) ? 1.0 : 0.0;
  sg.stepc[c] = 1;
  if (phase == 0) sg.kc[c] = (c >= sg.C) ? 0 : sg.k;
}

// ---------------------------------------------------------------------------
// norm kernel: u_j = r - (alpha_{j-1} s_{j-1}) u_{j-1}  (j >= 2) or the start
// block (j = 1); partial sums of |u_j|^2; in the regeneration pass also
// psi_b = fma(y_{b,j}, u_j, psi_b).  S = panels per lane (exact).
// ---------------------------------------------------------------------------
template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_norm(const Seg* __restrict__ segs, int nseg) {
  using V = typename PanelT<T>::V;
  constexpr int W = PanelT<T>::W;
  __shared__ double lds[4 * S * W];
  const Tile t = tile_of<false>(segs, nseg);
  const CONST_AS CSeg& sg = cseg(segs, t.seg);
  const int j = sg.stepc[0];
  if (j > sg.k) return;
  const int cp = sg.cpad;
  const uint32_t dim = 1u << sg.nbits;
  const uint64_t pstride = (uint64_t)dim;

  V* ucur = (V*)slot_ptr<T>(sg, j) + (uint64_t)t.panel0 * pstride;
  const V* uprev = (j > 1) ? (const V*)slot_ptr<T>(sg, j - 1) + (uint64_t)t.panel0 * pstride : nullptr;
  const V* rv = (const V*)sg.R + (uint64_t)t.panel0 * pstride;
  const bool regen = sg.mode == MODE_REGEN;
  const T amp = amp_of<T>(sg.nb);
  const CONST_AS double* st = (const CONST_AS double*)sg.st;

  V acur[S];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int e = 0; e < W; ++e) acur[s][e] = (T)st[ST_ACUR * cp + (t.panel0 + s) * W + e];

  double dsum[S * W];
#pragma unroll
  for (int i = 0; i < S * W; ++i) dsum[i] = 0.0;

  for (int rr = 0; rr < sg.rpl; ++rr) {
    const uint32_t row = t.row0 + rr * kBlock + threadIdx.x;
    if (row >= dim) break;
    V u[S];
    if (j == 1) {
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int e = 0; e < W; ++e)
          u[s][e] = start_value<T>(sg.start_kind, sg.ns_log, sg.nb, sg.seed, row, (t.panel0 + s) * W + e,
                                   sg.C, amp);
    } else {
      V r[S], up[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        r[s] = ldg_nt(rv + s * pstride, row);
        up[s] = ldg_nt(uprev + s * pstride, row);
      }
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int e = 0; e < W; ++e) u[s][e] = fma_s(-acur[s][e], up[s][e], r[s][e]);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      stg(ucur + s * pstride, row, u[s]);
#pragma unroll
      for (int e = 0; e < W; ++e) dsum[s * W + e] += (double)u[s][e] * (double)u[s][e];
    }
    if (regen) {
      const CONST_AS T* yt = (const CONST_AS T*)sg.ytab;
      for (int b = 0; b < sg.n_beta; ++b) {
        V* pb = (V*)sg.psi + (uint64_t)b * (sg.blk / W) + (uint64_t)t.panel0 * pstride;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          V old;
          if (j == 1) {
#pragma unroll
            for (int e = 0; e < W; ++e) old[e] = T(0);
          } else {
            old = ldg(pb + s * pstride, row);
          }
          V nw;
#pragma unroll
          for (int e = 0; e < W; ++e) {
            const T y = yt[((uint64_t)b * sg.k + (j - 1)) * cp + (t.panel0 + s) * W + e];
            nw[e] = fma_s(y, u[s][e], old[e]);
          }
          stg(pb + s * pstride, row, nw);
        }
      }
    }
  }
  double tot;
  block_sum<S * W>(dsum, lds, &tot);
  if (threadIdx.x < S * W) sg.part[(uint64_t)t.rtile * cp + t.panel0 * W + threadIdx.x] = tot;
}

// ---------------------------------------------------------------------------
// apply kernel: r = s_j (H u_j) - (beta_{j-1} s_{j-1}) u_{j-1}, partial sums of
// <u_j, r>.  MODE_PLAIN: Y = H X with X = Q, Y = R.
//
// A workgroup owns a tile of 256 consecutive rows (one per lane) and S panels
// (S*W columns).  Every off-diagonal term maps the tile onto one partner tile
// (the flip bits above the tile, fhi) permuted inside by the low flip bits
// (flo).  The hops are grouped by fhi on the host.  For a partner tile that
// several hops share, the workgroup loads it once -- a coalesced 16-byte load
// per lane and panel -- into LDS, and every hop of the group reads its operand
// from LDS at lane ^ flo; the load of the next group's tile is issued before
// the current group's FMAs (double-buffered LDS), so one barrier per group
// separates the two.  Hops whose partner tile is shared by fewer than
// kFatGroup hops skip the staging and gather directly.  Hop coefficients come
// from scalar loads.
// ---------------------------------------------------------------------------
template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_apply(const Seg* __restrict__ segs, int nseg) {
  using V = typename PanelT<T>::V;
  constexpr int W = PanelT<T>::W;
  __shared__ V tl[2][S][kBlock];
  __shared__ double lds[4 * S * W];
  const Tile t = tile_of<true>(segs, nseg);
  const CONST_AS CSeg& sg = cseg(segs, t.seg);
  const bool plain = sg.mode == MODE_PLAIN;
  int j = 1;
  if (!plain) {
    j = sg.stepc[0];
    if (j > sg.k) return;
  }
  const int cp = sg.cpad;
  const uint32_t dim = 1u << sg.nbits;
  const uint64_t pstride = (uint64_t)dim;
  const V* ub = (plain ? (const V*)sg.Q : (const V*)slot_ptr<T>(sg, j)) + (uint64_t)t.panel0 * pstride;
  const V* uprev = (!plain && j > 1) ? (const V*)slot_ptr<T>(sg, j - 1) + (uint64_t)t.panel0 * pstride
                                     : nullptr;
  V* out = (V*)sg.R + (uint64_t)t.panel0 * pstride;
  const CONST_AS GHop<T>* hp = (const CONST_AS GHop<T>*)sg.hops;
  const CONST_AS HopGroup* gr = (const CONST_AS HopGroup*)sg.groups;
  const int ng = sg.ngroups;
  const T* dg = (const T*)sg.diag;
  const bool dots = sg.mode == MODE_LANCZOS;
  const CONST_AS double* st = (const CONST_AS double*)sg.st;

  const uint32_t lane = threadIdx.x;
  const uint32_t row = t.row0 + lane;
  const bool valid = row < dim;
  const uint32_t wbase = __builtin_amdgcn_readfirstlane(row & ~63u);

  V xc[S], acc[S], xnext[S];
  const T d = valid ? ldg_s(dg, row) : T(0);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    if (valid) {
      xc[s] = ldg(ub + s * pstride, row);
    } else {
#pragma unroll
      for (int e = 0; e < W; ++e) xc[s][e] = T(0);
    }
    acc[s] = d * xc[s];
    xnext[s] = xc[s];            // group 0 is the own tile
  }

  // next group that contributes to this tile: a tile-uniform group whose
  // coefficients all vanish for this tile is skipped (no load, no barrier)
  const uint32_t tbase = t.row0;
  auto next_active = [&](int g) -> int {
    for (; g < ng; ++g) {
      if (!gr[g].tile_uniform) return g;
      const int h0 = gr[g].start, n1 = gr[g].n1;
      for (int h = h0; h < h0 + n1; ++h) {
        const T c = (__builtin_popcount(tbase & hp[h].m) & 1u) ? hp[h].cd : hp[h].cs;
        if (c != T(0)) return g;
      }
    }
    return ng;
  };

  int buf = 0;
  for (int g = 0; g < ng; ++buf) {
    const int b = buf & 1;
    const int gn = next_active(g + 1);
#pragma unroll
    for (int s = 0; s < S; ++s) tl[b][s][lane] = xnext[s];
    __syncthreads();
    if (gn < ng && valid) {
      const uint32_t p = row ^ gr[gn].fhi;
#pragma unroll
      for (int s = 0; s < S; ++s) xnext[s] = ldg(ub + s * pstride, p);
    }
    if (valid) {
      const int h0 = gr[g].start, n0 = gr[g].n0, n1 = gr[g].n1, n2 = gr[g].n2;
      // state-independent coefficients, U hops at a time: all U*S operand
      // reads are issued before the FMAs that consume them
      constexpr int U = 4;
      int h = h0;
      for (; h + U <= h0 + n0; h += U) {
        uint32_t q[U];
        T c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          q[u] = lane ^ hp[h + u].flo;
          c[u] = hp[h + u].cs;
        }
        V a[U][S];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int s = 0; s < S; ++s) a[u][s] = tl[b][s][q[u]];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int s = 0; s < S; ++s) acc[s] += c[u] * a[u][s];
        __builtin_amdgcn_sched_group_barrier(0x0100, U * S, 0);
        __builtin_amdgcn_sched_group_barrier(0x0002, U * S * W, 0);
      }
      for (; h < h0 + n0; ++h) {
        const uint32_t q = lane ^ hp[h].flo;
        const T c = hp[h].cs;
#pragma unroll
        for (int s = 0; s < S; ++s) acc[s] += c * tl[b][s][q];
      }
      // coefficient uniform over the wave; zero ones skipped
      for (; h < h0 + n0 + n1; ++h) {
        const T c = (__builtin_popcount(wbase & hp[h].m) & 1u) ? hp[h].cd : hp[h].cs;
        if (c == T(0)) continue;
        const uint32_t q = lane ^ hp[h].flo;
#pragma unroll
        for (int s = 0; s < S; ++s) acc[s] += c * tl[b][s][q];
      }
      // per-row coefficient, two hops at a time
      const int hend = h0 + n0 + n1 + n2;
      for (; h + 2 <= hend; h += 2) {
        const uint32_t q0 = lane ^ hp[h].flo, q1 = lane ^ hp[h + 1].flo;
        V a0[S], a1[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
          a0[s] = tl[b][s][q0];
          a1[s] = tl[b][s][q1];
        }
        const T c0 = (__builtin_popcount(row & hp[h].m) & 1u) ? hp[h].cd : hp[h].cs;
        const T c1 = (__builtin_popcount(row & hp[h + 1].m) & 1u) ? hp[h + 1].cd : hp[h + 1].cs;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          acc[s] += c0 * a0[s];
          acc[s] += c1 * a1[s];
        }
        __builtin_amdgcn_sched_group_barrier(0x0100, 2 * S, 0);
        __builtin_amdgcn_sched_group_barrier(0x0002, 2 * S * W + 8, 0);
      }
      if (h < hend) {
        const T c = (__builtin_popcount(row & hp[h].m) & 1u) ? hp[h].cd : hp[h].cs;
        const uint32_t q = lane ^ hp[h].flo;
#pragma unroll
        for (int s = 0; s < S; ++s) acc[s] += c * tl[b][s][q];
      }
    }
    g = gn;
  }

  // hops whose partner tile few hops share: coalesced gathers straight from
  // memory, U at a time so U*S loads are in flight
  if (valid) {
    const CONST_AS GHop<T>* th = (const CONST_AS GHop<T>*)sg.thin;
    const int e0 = sg.nt0, e1 = e0 + sg.nt1, e2 = e1 + sg.nt2;
    constexpr int U = S >= 4 ? 4 : 8;
    int h = 0;
    for (; h + U <= e0; h += U) {
      V x[U][S];
      T c[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t p = row ^ th[h + u].flo;
        c[u] = th[h + u].cs;
#pragma unroll
        for (int s = 0; s < S; ++s) x[u][s] = ldg(ub + s * pstride, p);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int s = 0; s < S; ++s) acc[s] += c[u] * x[u][s];
      __builtin_amdgcn_sched_group_barrier(0x0020, U * S, 0);
      __builtin_amdgcn_sched_group_barrier(0x0002, U * S * W, 0);
    }
    for (; h < e0; ++h) {
      const uint32_t p = row ^ th[h].flo;
      const T c = th[h].cs;
#pragma unroll
      for (int s = 0; s < S; ++s) acc[s] += c * ldg(ub + s * pstride, p);
    }
    // wave-uniform coefficient: zero ones skipped
    for (; h < e1; ++h) {
      const T c = (__builtin_popcount(wbase & th[h].m) & 1u) ? th[h].cd : th[h].cs;
      if (c == T(0)) continue;
      const uint32_t p = row ^ th[h].flo;
#pragma unroll
      for (int s = 0; s < S; ++s) acc[s] += c * ldg(ub + s * pstride, p);
    }
    for (; h + 2 <= e2; h += 2) {
      V x0[S], x1[S];
      const uint32_t p0 = row ^ th[h].flo, p1 = row ^ th[h + 1].flo;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        x0[s] = ldg(ub + s * pstride, p0);
        x1[s] = ldg(ub + s * pstride, p1);
      }
      const T c0 = (__builtin_popcount(row & th[h].m) & 1u) ? th[h].cd : th[h].cs;
      const T c1 = (__builtin_popcount(row & th[h + 1].m) & 1u) ? th[h + 1].cd : th[h + 1].cs;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        acc[s] += c0 * x0[s];
        acc[s] += c1 * x1[s];
      }
    }
    if (h < e2) {
      const uint32_t p = row ^ th[h].flo;
      const T c = (__builtin_popcount(row & th[h].m) & 1u) ? th[h].cd : th[h].cs;
#pragma unroll
      for (int s = 0; s < S; ++s) acc[s] += c * ldg(ub + s * pstride, p);
    }
  }

  double dq[S * W];
#pragma unroll
  for (int i = 0; i < S * W; ++i) dq[i] = 0.0;
  if (valid) {
    V up[S];
    if (uprev) {
#pragma unroll
      for (int s = 0; s < S; ++s) up[s] = ldg_nt(uprev + s * pstride, row);
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      V r = scur_of<T, S>(st, cp, t.panel0, s, plain) * acc[s];
      if (uprev) {
        const V bp = bps_of<T, S>(st, cp, t.panel0, s);
#pragma unroll
        for (int e = 0; e < W; ++e) r[e] = fma_s(-bp[e], up[s][e], r[e]);
      }
      stg_stream<true>(out + s * pstride, row, r);
      if (dots) {
#pragma unroll
        for (int e = 0; e < W; ++e) dq[s * W + e] = (double)xc[s][e] * (double)r[e];
      }
    }
  }
  if (!dots) return;
  double tot;
  block_sum<S * W>(dq, lds, &tot);
  if (threadIdx.x < S * W) sg.part[(uint64_t)t.rtile * cp + t.panel0 * W + threadIdx.x] = tot;
}

// ---------------------------------------------------------------------------
// apply on bit-set tiles (Seg::wide): the product (MODE_PLAIN) or product and
// recurrence of k_apply for hop-table operators on kWideBits sites or more.
//
// A tile is the 2^kWideBits rows that differ only in the row bits B
// (Seg::wbits) and agree with the tile's base in all other bits.  A workgroup
// of kWideBlock lanes owns one tile of one panel; lane l holds the rows of
// tile index t = l + kWideBlock q (q < kWideRows) at row base | deposit(t, B).
// A hop with flip bits f maps tile index t to t ^ flo in the partner tile
// base ^ fhi (fhi = f & ~B, flo = f & B packed to B's positions).  The hops
// are grouped by fhi on the host, B chosen there to leave few distinct
// partner tiles.  A group's partner tile is staged in LDS at slot t (16-byte
// slots; the 8 lanes of a 128-byte phase read t ^ flo from one aligned group
// of 8 slots, so there are no bank conflicts); the next group's tile is
// loaded into registers while the current group's hops run.  The own tile
// (the hops inside it) comes last, so the diagonal term and <u_j, r> read
// the row's own value from LDS.  Hops whose partner tile no other hop reads
// are gathered directly from memory.
// ---------------------------------------------------------------------------
// the low bits of x deposited at the set bits of mask, lowest first
__device__ __forceinline__ uint32_t deposit_bits(uint32_t x, uint32_t mask) {
  uint32_t r = 0;
  for (uint32_t m = mask; m != 0u; m &= m - 1u, x >>= 1)
    if (x & 1u) r |= m & (0u - m);
  return r;
}

struct WTile {
  int32_t seg;
  uint32_t base;   // row bits outside B
  int32_t panel;
  int32_t tile;    // partial-sum row
};

// The tile of this workgroup: binary search of blockIdx.x in the segments'
// wp_base offsets, then panel-major inside the segment (the workgroups in
// flight share one panel, whose partner tiles the memory-side cache holds).
// Workgroups go round-robin to the 8 XCDs; inside a panel the k-th workgroup
// of each XCD takes consecutive tiles, so partner tiles whose bases differ in
// low tile bits are read through that XCD's L2.  A bijection on the panel's
// 2^(N - kWideBits) tiles (a multiple of 8 from N = kWideBits + 3 on).
__device__ __forceinline__ WTile wide_tile_of(const Seg* segs, int nseg) {
  const CONST_AS Seg* cs = (const CONST_AS Seg*)segs;
  const int b = (int)blockIdx.x;
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cs[mid].wp_base <= b) lo = mid;
    else hi = mid - 1;
  }
  const int tb = cs[lo].nbits - kWideBits;
  const int nt = 1 << tb;
  const int lt = b - cs[lo].wp_base;
  const int panel = lt >> tb;
  int tile = lt & (nt - 1);
  if (nt >= 8) tile = (tile & 7) * (nt >> 3) + (tile >> 3);
  const uint32_t outside = ~cs[lo].wbits & ((1u << cs[lo].nbits) - 1u);
  return WTile{lo, deposit_bits((uint32_t)tile, outside), panel, tile};
}

template <typename T>
__global__ __launch_bounds__(kWideBlock) void k_apply_wide(const Seg* __restrict__ segs, int nseg) {
  using V = typename PanelT<T>::V;
  constexpr int W = PanelT<T>::W;
  constexpr int R = kWideRows;
  constexpr int NW = kWideBlock / 64;
  __shared__ V tl[1 << kWideBits];
  __shared__ double lds[NW * W];
  const WTile t = wide_tile_of(segs, nseg);
  const CONST_AS CSeg& sg = cseg(segs, t.seg);
  const bool plain = sg.mode == MODE_PLAIN;
  int j = 1;
  if (!plain) {
    j = sg.stepc[0];
    if (j > sg.k) return;
  }
  const int cp = sg.cpad;
  const uint64_t pstride = (uint64_t)1 << sg.nbits;
  const V* ub = (plain ? (const V*)sg.Q : (const V*)slot_ptr<T>(sg, j)) + (uint64_t)t.panel * pstride;
  const V* uprev = (!plain && j > 1) ? (const V*)slot_ptr<T>(sg, j - 1) + (uint64_t)t.panel * pstride
                                     : nullptr;
  V* out = (V*)sg.R + (uint64_t)t.panel * pstride;
  const CONST_AS GHop<T>* hp = (const CONST_AS GHop<T>*)sg.hops;
  const CONST_AS HopGroup* gr = (const CONST_AS HopGroup*)sg.groups;
  const int ng = sg.ngroups;
  const T* dg = (const T*)sg.diag;
  const bool dots = sg.mode == MODE_LANCZOS;
  const CONST_AS double* st = (const CONST_AS double*)sg.st;

  const uint32_t B = sg.wbits;
  const uint32_t lane = threadIdx.x;
  const uint32_t lrow = t.base | deposit_bits(lane, B);
  // row q of the lane = lrow | dep[q]; dep[q] is uniform, so a per-row
  // coefficient parity(row & m) is parity(lrow & m) (per lane, once per hop)
  // flipped by the uniform parity(dep[q] & m)
  uint32_t dep[R], row[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    dep[q] = deposit_bits((uint32_t)(q * kWideBlock), B);
    row[q] = lrow | dep[q];
  }
  auto row_coefs = [&](uint32_t m, T cs, T cd, T (&c)[R]) {
    const bool p0 = __builtin_popcount(lrow & m) & 1u;
    const T ca = p0 ? cd : cs, cb = p0 ? cs : cd;
#pragma unroll
    for (int q = 0; q < R; ++q) c[q] = (__builtin_popcount(dep[q] & m) & 1u) ? cb : ca;
  };

  // next partner group (1 .. ng-1) that contributes to this tile: a
  // tile-uniform group whose coefficients all vanish here is skipped (no
  // load, no barrier); ng stands for the own tile (group 0), staged last so
  // that its values are still in LDS for the diagonal and the dot products
  auto next_active = [&](int g) -> int {
    for (; g < ng; ++g) {
      if (!gr[g].tile_uniform) return g;
      const int h0 = gr[g].start, n1 = gr[g].n1;
      for (int h = h0; h < h0 + n1; ++h) {
        const T c = (__builtin_popcount(t.base & hp[h].m) & 1u) ? hp[h].cd : hp[h].cs;
        if (c != T(0)) return g;
      }
    }
    return ng;
  };

  V acc[R], nx[R];
#pragma unroll
  for (int q = 0; q < R; ++q)
#pragma unroll
    for (int e = 0; e < W; ++e) acc[q][e] = T(0);
  int g = next_active(1);
  {
    const uint32_t f = g < ng ? gr[g].fhi : 0u;
#pragma unroll
    for (int q = 0; q < R; ++q) nx[q] = ldg(ub, row[q] ^ f);
  }

  // hops whose partner tile no other hop reads: gathered directly, two hops
  // (2R loads) in flight, while the first staged tile is on its way
  {
    const CONST_AS GHop<T>* th = (const CONST_AS GHop<T>*)sg.thin;
    const int e0 = sg.nt0, e1 = e0 + sg.nt1, e2 = e1 + sg.nt2;
    int h = 0;
    for (; h < e0; ++h) {
      const uint32_t f = th[h].flo;
      const T c = th[h].cs;
      V x[R];
#pragma unroll
      for (int q = 0; q < R; ++q) x[q] = ldg(ub, row[q] ^ f);
#pragma unroll
      for (int q = 0; q < R; ++q) acc[q] += c * x[q];
    }
    for (; h < e1; ++h) {
      const T c = (__builtin_popcount(t.base & th[h].m) & 1u) ? th[h].cd : th[h].cs;
      if (c == T(0)) continue;
      const uint32_t f = th[h].flo;
      V x[R];
#pragma unroll
      for (int q = 0; q < R; ++q) x[q] = ldg(ub, row[q] ^ f);
#pragma unroll
      for (int q = 0; q < R; ++q) acc[q] += c * x[q];
    }
    for (; h + 2 <= e2; h += 2) {
      const uint32_t f0 = th[h].flo, f1 = th[h + 1].flo;
      V x0[R], x1[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        x0[q] = ldg(ub, row[q] ^ f0);
        x1[q] = ldg(ub, row[q] ^ f1);
      }
      T c0[R], c1[R];
      row_coefs(th[h].m, th[h].cs, th[h].cd, c0);
      row_coefs(th[h + 1].m, th[h + 1].cs, th[h + 1].cd, c1);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        acc[q] += c0[q] * x0[q];
        acc[q] += c1[q] * x1[q];
      }
    }
    if (h < e2) {
      const uint32_t f = th[h].flo;
      V x[R];
#pragma unroll
      for (int q = 0; q < R; ++q) x[q] = ldg(ub, row[q] ^ f);
      T c[R];
      row_coefs(th[h].m, th[h].cs, th[h].cd, c);
#pragma unroll
      for (int q = 0; q < R; ++q) acc[q] += c[q] * x[q];
    }
  }

  for (;;) {
    const int cur = g < ng ? g : 0;
    const int gn = g < ng ? next_active(g + 1) : -1;
    __syncthreads();             // the previous group's reads of tl are done
#pragma unroll
    for (int q = 0; q < R; ++q) tl[lane + q * kWideBlock] = nx[q];
    __syncthreads();
    if (gn >= 0) {
      const uint32_t f = gn < ng ? gr[gn].fhi : 0u;
#pragma unroll
      for (int q = 0; q < R; ++q) nx[q] = ldg(ub, row[q] ^ f);
    }
    const int h0 = gr[cur].start, e0 = h0 + gr[cur].n0, e1 = e0 + gr[cur].n1, e2 = e1 + gr[cur].n2;
    int h = h0;
    for (; h < e0; ++h) {        // m = 0
      const uint32_t flo = hp[h].flo;
      const T c = hp[h].cs;
#pragma unroll
      for (int q = 0; q < R; ++q) acc[q] += c * tl[(lane + q * kWideBlock) ^ flo];
    }
    for (; h < e1; ++h) {        // coefficient uniform over the tile; zero ones skipped
      const T c = (__builtin_popcount(t.base & hp[h].m) & 1u) ? hp[h].cd : hp[h].cs;
      if (c == T(0)) continue;
      const uint32_t flo = hp[h].flo;
#pragma unroll
      for (int q = 0; q < R; ++q) acc[q] += c * tl[(lane + q * kWideBlock) ^ flo];
    }
    for (; h < e2; ++h) {        // per-row coefficient
      const uint32_t flo = hp[h].flo;
      V a[R];
#pragma unroll
      for (int q = 0; q < R; ++q) a[q] = tl[(lane + q * kWideBlock) ^ flo];
      T c[R];
      row_coefs(hp[h].m, hp[h].cs, hp[h].cd, c);
#pragma unroll
      for (int q = 0; q < R; ++q) acc[q] += c[q] * a[q];
    }
    if (gn < 0) break;
    g = gn;
  }

  double dq[W];
#pragma unroll
  for (int e = 0; e < W; ++e) dq[e] = 0.0;
  V up[R];
  if (uprev) {
#pragma unroll
    for (int q = 0; q < R; ++q) up[q] = ldg_nt(uprev, row[q]);
  }
  const V sc = scur_of<T, 1>(st, cp, t.panel, 0, plain);
  V bp;
  if (uprev) bp = bps_of<T, 1>(st, cp, t.panel, 0);
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const V x = tl[lane + q * kWideBlock];   // the own row, staged last
    V r = sc * (acc[q] + ldg_s(dg, row[q]) * x);
    if (uprev) {
#pragma unroll
      for (int e = 0; e < W; ++e) r[e] = fma_s(-bp[e], up[q][e], r[e]);
    }
    stg_stream<true>(out, row[q], r);
    if (dots) {
#pragma unroll
      for (int e = 0; e < W; ++e) dq[e] += (double)x[e] * (double)r[e];
    }
  }
  if (!dots) return;
  // fixed-order sum over the workgroup's NW waves
#pragma unroll
  for (int e = 0; e < W; ++e) dq[e] = wave_sum(dq[e]);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int e = 0; e < W; ++e) lds[wave * W + e] = dq[e];
  }
  __syncthreads();
  if (threadIdx.x < W) {
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) tot += lds[w * W + threadIdx.x];
    sg.part[(uint64_t)t.tile * cp + t.panel * W + threadIdx.x] = tot;
  }
}

// ---------------------------------------------------------------------------
// Transform apply for operators whose off-diagonal part has only X-type terms
// (XX couplings and x-fields, no YY): in the Hadamard basis such a term is
// diagonal, so H = D_Z + W D_X W with W the unnormalised Walsh-Hadamard
// transform on all N bits and D_X (with the 2^-N of W^2 folded in) the X-term
// energies.  Each workgroup transforms a 4096-row tile in registers and LDS,
// over the low 12 row bits (W_lo, contiguous tiles) or the high N - 12 bits
// (W_hi, tiles of 2^(24-N)-row runs at every high-bit value); W = W_hi W_lo.
// The plain product Y = H X takes three such passes (k_apply_xz); a Lanczos
// step keeps its basis in the low-bit Hadamard basis and takes two
// (k_xz_lanczos).  Intermediate results live in the output block R, which
// each workgroup rewrites only at its own rows.
//
// A tile is 4096 elements indexed by a 12-bit coordinate tau; lane l holds 16
// of them in registers q.  Three arrangements: 0: tau = q*256 + l (q = bits
// 8..11); 1: tau = l*16 + q (q = bits 0..3); 2: q = bits 4..7, l = bits 0..3
// and 8..11.  Butterflies act on register bits; an LDS round trip changes the
// arrangement.  The LDS slot of tau is tau + (tau >> 4) (one 16-byte pad per
// 16 slots): in every arrangement it is a per-lane base plus a constant per
// register (an instruction offset), and the 16 lanes of each group of a
// 16-byte access fall on distinct banks (slot mod 16 = lane + const).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t xz_tau(int arr, uint32_t l, int q) {
  return arr == 0 ? (uint32_t)q * 256u + l
       : arr == 1 ? (l << 4) | (uint32_t)q
                  : (l & 15u) | ((uint32_t)q << 4) | ((l >> 4) << 8);
}
// tau + (tau >> 4) for tau = xz_tau(arr, l, q), as base(l) + const(q)
__device__ __forceinline__ uint32_t xz_slot(int arr, uint32_t l, int q) {
  return arr == 0 ? (l + (l >> 4)) + (uint32_t)q * 272u
       : arr == 1 ? l * 17u + (uint32_t)q
                  : ((l & 15u) + (l >> 4) * 272u) + (uint32_t)q * 17u;
}
constexpr int kXzLdsSlots = (1 << kXzTileBits) + (1 << (kXzTileBits - 4));

// butterflies (a, b) -> (a + b, a - b) over the register bits set in mask
template <typename V>
__device__ __forceinline__ void xz_bfly(V (&v)[kXzRegs], int mask) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (!((mask >> k) & 1)) continue;
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) {
      if (q & (1 << k)) continue;
      const V a = v[q], b = v[q | (1 << k)];
      v[q] = a + b;
      v[q | (1 << k)] = a - b;
    }
  }
}

template <typename V>
__device__ __forceinline__ void xz_rearrange(V (&v)[kXzRegs], V* lds, int from, int to) {
  const uint32_t l = threadIdx.x;
#pragma unroll
  for (int q = 0; q < kXzRegs; ++q) lds[xz_slot(from, l, q)] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kXzRegs; ++q) v[q] = lds[xz_slot(to, l, q)];
  __syncthreads();
}

__device__ __forceinline__ Tile xz_tile_of(const Seg* segs, int nseg, int b, bool strided = false) {
  const CONST_AS Seg* cs = (const CONST_AS Seg*)segs;
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cs[mid].x_base <= b) lo = mid;
    else hi = mid - 1;
  }
  int lt = b - cs[lo].x_base;
  const int nrt = cs[lo].x_tiles;
  if (strided && cs[lo].nbits > kXzTileBits + 9 && cs[lo].nbits <= kXzDeepMaxBits) {
    // more than 9 high bits: a strided tile reads runs of fewer than 8 rows
    // (under 128 bytes), and 128 / (16 * 2^lrb) neighbouring tiles share each
    // cache line.  Workgroups go round-robin to the 8 XCDs, so the k-th
    // workgroup of each XCD takes consecutive tiles: lines shared by
    // neighbours meet in one XCD's L2 instead of being fetched by several.
    // A bijection on the segment's tiles (a multiple of 8: at least 1024).
    const int n = nrt * cs[lo].P;
    lt = (lt & 7) * (n >> 3) + (lt >> 3);
  }
  const int sl = lt / nrt, rt = lt - sl * nrt;
  return Tile{lo, (uint32_t)rt << kXzTileBits, sl, rt};
}

template <typename V>
__device__ __forceinline__ void xz_low_transform(V (&v)[kXzRegs], V* lds) {
  xz_bfly(v, 0xF);                 // bits 8..11
  xz_rearrange(v, lds, 0, 1);
  xz_bfly(v, 0xF);                 // bits 0..3
  xz_rearrange(v, lds, 1, 2);
  xz_bfly(v, 0xF);                 // bits 4..7
  xz_rearrange(v, lds, 2, 0);
}

// W_hi D_X W_hi on a strided tile held in arrangement 0.  The row's high bits
// are the tau bits lrb..11: 8..11 (arrangement 0), those of 4..7 at or above
// lrb (arrangement 2) and, in DEEP tiles (more than 8 high bits, lrb < 4),
// those of 0..3 at or above lrb (arrangement 1).  D_X is stored in row order
// for shallow operators (read through row_of) and in the strided tiles' own
// order for deep ones (tile rt's 4096 entries in tau order from rt * 4096).
// QUAD: qf[e] += sum over the tile of D z^2 (z = W_hi v, column e), the
// lane's share of <v, W_hi D W_hi v>.
template <typename T, typename V>
__device__ __forceinline__ V xz_scale_quad(T d, V z, double* qf, bool quad) {
  constexpr int W = sizeof(V) / sizeof(T);
  if (quad) {
#pragma unroll
    for (int e = 0; e < W; ++e) qf[e] += (double)d * ((double)z[e] * (double)z[e]);
  }
  return d * z;
}

template <bool DEEP, bool QUAD = false, typename T, typename V, typename RowOf>
__device__ __forceinline__ void xz_high_transform(V (&v)[kXzRegs], V* lds, const T* dx, uint32_t rt, int lrb,
                                                  RowOf row_of, double* qf = nullptr) {
  constexpr int W = sizeof(V) / sizeof(T);
  const uint32_t l = threadIdx.x;
  xz_bfly(v, 0xF);
  xz_rearrange(v, lds, 0, 2);
  if constexpr (!DEEP) {
    const int m2 = 0xF & ~((1 << (lrb - 4)) - 1);
    xz_bfly(v, m2);
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) v[q] = xz_scale_quad(ldg_s(dx, row_of(xz_tau(2, l, q))), v[q], qf, QUAD);
    xz_bfly(v, m2);
  } else {
    const int m1 = 0xF & ~((1 << lrb) - 1);
    xz_bfly(v, 0xF);
    xz_rearrange(v, lds, 2, 1);
    xz_bfly(v, m1);
    // arrangement 1: lane l holds tau = 16 l .. 16 l + 15, contiguous in D_X
    const V* dv = (const V*)(dx + ((uint64_t)rt << kXzTileBits) + 16u * l);
#pragma unroll
    for (int g = 0; g < kXzRegs / W; ++g) {
      const V dd = ldg(dv, (uint32_t)g);
#pragma unroll
      for (int e = 0; e < W; ++e) v[g * W + e] = xz_scale_quad(dd[e], v[g * W + e], qf, QUAD);
    }
    xz_bfly(v, m1);
    xz_rearrange(v, lds, 1, 2);
    xz_bfly(v, 0xF);
  }
  xz_rearrange(v, lds, 2, 0);
  xz_bfly(v, 0xF);
}

// The YY twist T = diag(t(idx)), t = (-1)^floor(popcount(idx)/2): Y_i Y_j =
// T X_i X_j T for every pair, so the YY couplings are T W D_Y W T.
__device__ __forceinline__ bool yy_twist_neg(uint32_t row) { return (__builtin_popcount(row) >> 1) & 1u; }

template <typename T, typename V>
__device__ __forceinline__ void yy_twist(V (&v)[kXzRegs], uint32_t row0, T scale) {
  const uint32_t l = threadIdx.x;
#pragma unroll
  for (int q = 0; q < kXzRegs; ++q) {
    const bool neg = yy_twist_neg(row0 + xz_tau(0, l, q));
    v[q] = (neg ? -scale : scale) * v[q];
  }
}

// In-place strided pass buf = W_hi D W_hi buf on the strided tile t of a
// segment (the row map and cache hints of the strided passes below); QUAD as
// in xz_high_transform.
template <typename T, bool DEEP, bool QUAD = false>
__device__ __forceinline__ void xz_strided_inplace(const CONST_AS CSeg& sg, const Tile& t, typename PanelT<T>::V* buf,
                                                   const T* dd, typename PanelT<T>::V* lds, double* qf = nullptr) {
  using V = typename PanelT<T>::V;
  const uint32_t l = threadIdx.x;
  const int hb = sg.nbits - kXzTileBits;
  const int lrb = kXzTileBits - hb;
  const uint32_t lrm = (1u << lrb) - 1u;
  const uint32_t base = (uint32_t)t.rtile << lrb;
  auto row_of = [&](uint32_t tau) -> uint32_t {
    return ((tau >> lrb) << kXzTileBits) | (base + (tau & lrm));
  };
  V v[kXzRegs];
  auto run = [&](auto nt_tag) {
    constexpr bool NT = decltype(nt_tag)::value;
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) v[q] = ldg_sel<NT>((const V*)buf, row_of(xz_tau(0, l, q)));
    xz_high_transform<DEEP, QUAD>(v, lds, dd, t.rtile, lrb, row_of, qf);
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) stg_sel<NT>(buf, row_of(xz_tau(0, l, q)), v[q]);
  };
  if (!DEEP || lrb >= 3) run(std::true_type{});
  else run(std::false_type{});
}

// Transform over one group of high bits on a split tile held in arrangement
// 0: the group's g bits are the tau bits lrb..11 (lrb = 12 - g >= 4), so the
// butterflies act on arrangement 0 (tau bits 8..11) and on the bits of 4..7
// at or above lrb (arrangement 2), as in shallow tiles.  WITH_D: the sandwich
// W_G D W_G with D read in row order through row_of; otherwise W_G alone.
// QUAD (with WITH_D) as in xz_high_transform.
template <bool WITH_D, bool QUAD = false, typename T, typename V, typename RowOf>
__device__ __forceinline__ void xz_group_transform(V (&v)[kXzRegs], V* lds, const T* dd, int lrb, RowOf row_of,
                                                   double* qf = nullptr) {
  const uint32_t l = threadIdx.x;
  const int m2 = 0xF & ~((1 << (lrb - 4)) - 1);
  xz_bfly(v, 0xF);
  xz_rearrange(v, lds, 0, 2);
  xz_bfly(v, m2);
  if (WITH_D) {
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) v[q] = xz_scale_quad(ldg_s(dd, row_of(xz_tau(2, l, q))), v[q], qf, QUAD);
    xz_bfly(v, m2);
  }
  xz_rearrange(v, lds, 2, 0);
  if (WITH_D) xz_bfly(v, 0xF);
}

// Row of tau in a split tile of group A (B = false: bits 12 .. 12+a-1) or B
// (bits 12+a .. N-1) of a segment on nbits bits; the tile index rt holds the
// other group's bits above the g low-rest bits lrb..11 of the row.
struct SplitRows {
  int lrb;
  uint32_t lrm, fixed;
  int gshift;
  __device__ __forceinline__ SplitRows(int nbits, bool B, uint32_t rt) {
    const int a = xz_split_a(nbits);
    const int g = B ? nbits - kXzTileBits - a : a;
    lrb = kXzTileBits - g;
    lrm = (1u << lrb) - 1u;
    const uint32_t lowrest = rt & ((1u << g) - 1u), other = rt >> g;
    gshift = B ? kXzTileBits + a : kXzTileBits;
    fixed = (lowrest << lrb) | (other << (B ? kXzTileBits : kXzTileBits + a));
  }
  __device__ __forceinline__ uint32_t operator()(uint32_t tau) const {
    return ((tau >> lrb) << gshift) | fixed | (tau & lrm);
  }
};

// The strided passes of split segments (ops of launch_xz_split), in place.
template <typename T, int OP>
__global__ __launch_bounds__(kBlock) void k_xz_split(const Seg* __restrict__ segs, int nseg) {
  using V = typename PanelT<T>::V;
  constexpr int W = PanelT<T>::W;
  // FP64 Lanczos steps: the D_X / D_Y sandwiches give the XP_QX / XP_QY planes
  constexpr bool QUAD = sizeof(T) == 8 && (OP == 1 || OP == 3);
  __shared__ V lds[kXzLdsSlots];
  __shared__ double red[4 * W];
  const Tile t = xz_tile_of(segs, nseg, (int)blockIdx.x);
  const CONST_AS CSeg& sg = cseg(segs, t.seg);
  if (xz_geom(sg.nbits) != XG_SPLIT) return;
  if ((OP == 2 || OP == 3) && !sg.xy) return;
  if (sg.mode != MODE_PLAIN && sg.stepc[0] > sg.k) return;
  const uint64_t pstride = (uint64_t)1 << sg.nbits;
  constexpr bool B = OP == 1 || OP == 3;
  const SplitRows row_of(sg.nbits, B, (uint32_t)t.rtile);
  V* buf = (V*)(OP == 2 || OP == 3 ? sg.Y : sg.R) + (uint64_t)t.panel0 * pstride;
  const V* src = OP == 4 ? (const V*)sg.Q + (uint64_t)t.panel0 * pstride : buf;
  const uint32_t l = threadIdx.x;
  V v[kXzRegs];
#pragma unroll
  for (int q = 0; q < kXzRegs; ++q) v[q] = ldg_nt(src, row_of(xz_tau(0, l, q)));
  double qf[W];
#pragma unroll
  for (int e = 0; e < W; ++e) qf[e] = 0.0;
  xz_group_transform<B, QUAD>(v, lds, (const T*)(OP == 3 ? sg.dy : sg.dx), row_of.lrb, row_of, qf);
  if (QUAD && sg.mode == MODE_LANCZOS) put_plane<W>(sg, OP == 1 ? XP_QX : XP_QY, t.rtile, t.panel0, qf, red);
  if (OP == 4) {
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) v[q] = T(1 << kXzTileBits) * v[q];
  }
#pragma unroll
  for (int q = 0; q < kXzRegs; ++q) stg_stream<true>(buf, row_of(xz_tau(0, l, q)), v[q]);
}

// Plain transform apply Y = H X (MODE_PLAIN segments), H = D_Z + W D_X W:
// phase 0: R = W_lo X (contiguous tiles); phase 1: R = W_hi D_X W_hi R
// (strided tiles); phase 2: R = D_Z X + W_lo R (contiguous tiles).
// The same product on blocks kept in the orthogonal basis X^ = W_lo X / 64
// (W_lo W_lo = L I, L = 4096; the block Lanczos keeps its blocks there):
// phase 3: X^ = W_lo X / 64 in place (contiguous, once per run); phase 4:
// R = L W_hi D_X W_hi X^ (strided); phase 5: R = W_lo D_Z W_lo X^ / L + R
// (contiguous), so that R = (W_lo / 64) H X: two passes per product.
// Strided passes come in two instantiations: DEEP for operators of more than
// kXzShallowMaxBits bits (more than 8 high bits), the other for the rest;
// each leaves the other's segments alone.
template <typename T, int PHASE, bool DEEP>
__global__ __launch_bounds__(kBlock) void k_apply_xz(const Seg* __restrict__ segs, int nseg) {
  using V = typename PanelT<T>::V;
  __shared__ V lds[kXzLdsSlots];
  const Tile t = xz_tile_of(segs, nseg, (int)blockIdx.x, DEEP);
  const CONST_AS CSeg& sg = cseg(segs, t.seg);
  const uint64_t pstride = (uint64_t)1 << sg.nbits;
  const V* ub = (const V*)sg.Q + (uint64_t)t.panel0 * pstride;
  V* rb = (V*)sg.R + (uint64_t)t.panel0 * pstride;
  const uint32_t l = threadIdx.x;
  V v[kXzRegs];

  if (PHASE >= 6) {
    // the YY part (xy segments): T W D_Y W T X = T W_lo (W_hi D_Y W_hi) W_lo T X
    if (!sg.xy) return;
    V* yb = (V*)sg.Y + (uint64_t)t.panel0 * pstride;
    if (PHASE == 7) {
      if (xz_geom(sg.nbits) != (DEEP ? XG_DEEP : XG_SHALLOW)) return;
      xz_strided_inplace<T, DEEP>(sg, t, yb, (const T*)sg.dy, lds);
      return;
    }
    if (PHASE == 6 || PHASE == 9) {
      // 6: Y = W_lo T X;  9: Y = W_lo T W_lo X^ / 64 (= W_lo T X, X kept as X^)
#pragma unroll
      for (int q = 0; q < kXzRegs; ++q) v[q] = ldg_nt(ub, t.row0 + xz_tau(0, l, q));
      if (PHASE == 9) xz_low_transform(v, lds);
      yy_twist<T>(v, t.row0, PHASE == 9 ? T(1) / T(1 << (kXzTileBits / 2)) : T(1));
      xz_low_transform(v, lds);
#pragma unroll
      for (int q = 0; q < kXzRegs; ++q) stg_stream<true>(yb, t.row0 + xz_tau(0, l, q), v[q]);
      return;
    }
    // 8: R += T W_lo Y;  10: R += W_lo T W_lo Y / 64
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) v[q] = ldg_nt((const V*)yb, t.row0 + xz_tau(0, l, q));
    xz_low_transform(v, lds);
    yy_twist<T>(v, t.row0, PHASE == 10 ? T(1) / T(1 << (kXzTileBits / 2)) : T(1));
    if (PHASE == 10) xz_low_transform(v, lds);
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) {
      const uint32_t row = t.row0 + xz_tau(0, l, q);
      stg_stream<true>(rb, row, ldg_nt((const V*)rb, row) + v[q]);
    }
  } else if (PHASE == 3) {
    // contiguous tile, in place on X
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) v[q] = ldg_nt(ub, t.row0 + xz_tau(0, l, q));
    xz_low_transform(v, lds);
    const T sc = T(1) / T(1 << (kXzTileBits / 2));
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) stg((V*)ub, t.row0 + xz_tau(0, l, q), sc * v[q]);
  } else if (PHASE == 5) {
    // contiguous tile: the diagonal term in the transformed basis
    const T* dg = (const T*)sg.diag;
    V w[kXzRegs];
    T d[kXzRegs];
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) {
      const uint32_t row = t.row0 + xz_tau(0, l, q);
      v[q] = ldg_nt(ub, row);
      w[q] = ldg_nt((const V*)rb, row);
      d[q] = ldg_s(dg, row);
    }
    xz_low_transform(v, lds);
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) v[q] = d[q] * v[q];
    xz_low_transform(v, lds);
    const T inv_l = T(1) / T(1 << kXzTileBits);
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) stg_stream<true>(rb, t.row0 + xz_tau(0, l, q), inv_l * v[q] + w[q]);
  } else if (PHASE == 0 || PHASE == 2) {
    // contiguous tile: row = row0 + tau; arrangement 0 loads and stores coalesced
    const V* src = PHASE == 0 ? ub : (const V*)rb;
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) v[q] = ldg_nt(src, t.row0 + xz_tau(0, l, q));
    // phase 2: the diagonal term's operands are loaded while the tile is transformed
    V u[PHASE == 2 ? kXzRegs : 1];
    T d[PHASE == 2 ? kXzRegs : 1];
    if (PHASE == 2) {
      const T* dg = (const T*)sg.diag;
#pragma unroll
      for (int q = 0; q < kXzRegs; ++q) {
        u[q] = ldg_nt(ub, t.row0 + xz_tau(0, l, q));
        d[q] = ldg_s(dg, t.row0 + xz_tau(0, l, q));
      }
    }
    xz_low_transform(v, lds);
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q)
      stg_stream<PHASE != 0>(rb, t.row0 + xz_tau(0, l, q), PHASE == 0 ? v[q] : d[q] * u[q] + v[q]);
  } else {
    // strided tile: tau = hi * Lr + lr  ->  row = hi * 4096 + rt * Lr + lr,
    // hb = N - 12 high bits (4 <= hb <= 8 shallow, 9 <= hb <= 12 DEEP;
    // operators go up to kXzMaxBits), Lr = 2^(12 - hb) >= 1
    if (xz_geom(sg.nbits) != (DEEP ? XG_DEEP : XG_SHALLOW)) return;
    const int hb = sg.nbits - kXzTileBits;
    const int lrb = kXzTileBits - hb;
    const uint32_t lrm = (1u << lrb) - 1u;
    const uint32_t base = (uint32_t)t.rtile << lrb;
    auto row_of = [&](uint32_t tau) -> uint32_t {
      return ((tau >> lrb) << kXzTileBits) | (base + (tau & lrm));
    };
    // phase 1 transforms R in place; phase 4 reads X^ and scales by L
    const V* src = PHASE == 4 ? ub : (const V*)rb;
    auto run = [&](auto nt_tag) {
      constexpr bool NT = decltype(nt_tag)::value;
#pragma unroll
      for (int q = 0; q < kXzRegs; ++q) v[q] = ldg_sel<NT>(src, row_of(xz_tau(0, l, q)));
      xz_high_transform<DEEP>(v, lds, (const T*)sg.dx, t.rtile, lrb, row_of);
      if (PHASE == 4) {
#pragma unroll
        for (int q = 0; q < kXzRegs; ++q) v[q] = T(1 << kXzTileBits) * v[q];
      }
#pragma unroll
      for (int q = 0; q < kXzRegs; ++q) stg_sel<NT>(rb, row_of(xz_tau(0, l, q)), v[q]);
    };
    if (!DEEP || lrb >= 3) run(std::true_type{});
    else run(std::false_type{});
  }
}

// ---------------------------------------------------------------------------
// Lanczos step of the transform apply with the basis kept as u~ = W_lo u
// (W_lo: Hadamard transform over the 12 low row bits, W_lo W_lo = L I,
// L = 4096).  With W = W_hi W_lo and H = D_Z + W D_X W (D_X holding 2^-N):
//   W_lo (H u) = W_lo (D_Z u) + L W_hi D_X W_hi u~,
// so a step is one strided pass (high-bit transform, norm step fused) and one
// contiguous pass (low-bit transforms, recurrence): 8 vector streams instead
// of 10.  W_lo acts on bath bits only, so Gram matrices and bath partial
// traces of the basis are those of u times L; the recombination weights
// carry L^-1/2.
//   PASS 0 (once per run, contiguous tiles): R = W_lo x_1
//   PASS 1 (strided tiles): u~_j = R - (alpha s)_{j-1} u~_{j-1} -> slot j,
//     partial |u~_j|^2 / L, psi~_b += y_{b,j} u~_j (regeneration pass);
//     R = W_hi D_X W_hi u~_j
//   PASS 2 (contiguous tiles): w = s L R - (beta s)_{j-1} u~_{j-1};
//     u = W_lo u~_j / L; R = s W_lo (D_Z u) + w  (= W_lo r_j);
//     partial <u_j, r_j> = s sum d u^2 + <u~_j, w> / L
// FP64 steps move the recurrence (ZR below): pass 2 only leaves
// Z = W_lo D_Z u_j in Y, pass 1 of the next step starts from
// s L R + s Z - (beta s) u~_{j-1}, and <u_j, r_j> comes from the XP_* planes.
// Passes 3-5: the YY part (below).
// boff offsets blockIdx.x in the segments' transform tile numbering.
// ---------------------------------------------------------------------------
template <typename T, int PASS, bool REGEN, int GEOM>
__global__ __launch_bounds__(kBlock) void k_xz_lanczos(const Seg* __restrict__ segs, int nseg, int boff) {
  using V = typename PanelT<T>::V;
  constexpr int W = PanelT<T>::W;
  constexpr bool DEEP = GEOM == XG_DEEP;
  // FP64 steps split the recurrence differently (the contiguous pass then
  // reads one vector and writes one, in 210 VGPRs at two waves per SIMD):
  // ZR: the contiguous pass leaves Z = W_lo D_Z u_j in the block Y and the
  // next strided pass forms s Z + s L R - (beta s) u~_{j-1} there; XD: the
  // step's <u_j, r_j> from the XP_* planes.  FP32 steps keep the whole
  // recurrence and the dot product in the contiguous pass.
  constexpr bool ZR = sizeof(T) == 8;
  constexpr bool XD = ZR && !REGEN;
  __shared__ V lds[kXzLdsSlots];
  __shared__ double red[4 * 2 * W];
  const Tile t = xz_tile_of(segs, nseg, (int)blockIdx.x + boff, (PASS == 1 || PASS == 4) && DEEP);
  const CONST_AS CSeg& sg = cseg(segs, t.seg);
  // pass 1 comes in variants (the regeneration pass needs more registers;
  // one per strided geometry); each leaves the other variants' tiles alone.
  // Passes 3, 4 and 5 run on the segments with a YY part only (pass 4:
  // shallow and deep; split segments take launch_xz_split).
  if (PASS == 1 && ((sg.mode == MODE_REGEN) != REGEN || xz_geom(sg.nbits) != GEOM)) return;
  if ((PASS == 3 || PASS == 4 || PASS == 5) && !sg.xy) return;
  if (PASS == 4 && xz_geom(sg.nbits) != GEOM) return;
  const int j = PASS == 0 ? 1 : sg.stepc[0];
  if (j > sg.k) return;
  const int cp = sg.cpad;
  const uint64_t pstride = (uint64_t)1 << sg.nbits;
  const uint32_t l = threadIdx.x;
  const CONST_AS double* st = (const CONST_AS double*)sg.st;
  V* rb = (V*)sg.R + (uint64_t)t.panel0 * pstride;
  const V* uprev = j > 1 ? (const V*)slot_ptr<T>(sg, j - 1) + (uint64_t)t.panel0 * pstride : nullptr;
  const T inv_l = T(1) / T(1 << kXzTileBits);
  V v[kXzRegs];

  if (PASS == 0) {
    const T amp = amp_of<T>(sg.nb);
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q)
#pragma unroll
      for (int e = 0; e < W; ++e)
        v[q][e] = start_value<T>(sg.start_kind, sg.ns_log, sg.nb, sg.seed, t.row0 + xz_tau(0, l, q),
                                 t.panel0 * W + e, sg.C, amp);
    xz_low_transform(v, lds);
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) stg_stream<true>(rb, t.row0 + xz_tau(0, l, q), v[q]);
    return;
  }

  if (PASS == 1) {
    // strided tile: tau = hi * Lr + lr  ->  row = hi * 4096 + rt * Lr + lr,
    // hb = N - 12 high bits (4 <= hb <= 8 shallow, 9 <= hb <= 10 DEEP),
    // Lr = 2^(12 - hb) >= 4; split segments: a tile of group A (SplitRows)
    const int hb = sg.nbits - kXzTileBits;
    const SplitRows srows(sg.nbits, false, (uint32_t)t.rtile);
    const int lrb = GEOM == XG_SPLIT ? srows.lrb : kXzTileBits - hb;
    const uint32_t lrm = (1u << lrb) - 1u;
    const uint32_t base = (uint32_t)t.rtile << lrb;
    auto row_of = [&](uint32_t tau) -> uint32_t {
      if constexpr (GEOM == XG_SPLIT) return srows(tau);
      else return ((tau >> lrb) << kXzTileBits) | (base + (tau & lrm));
    };
    auto run = [&](auto nt_tag) {
      constexpr bool NT = decltype(nt_tag)::value;
      V* ucur = (V*)slot_ptr<T>(sg, j) + (uint64_t)t.panel0 * pstride;
      V acur;
#pragma unroll
      for (int e = 0; e < W; ++e) acur[e] = (T)st[ST_ACUR * cp + t.panel0 * W + e];
#pragma unroll
      for (int q = 0; q < kXzRegs; ++q) v[q] = ldg_sel<NT>((const V*)rb, row_of(xz_tau(0, l, q)));
      // dsum: |u~_j|^2; XD: dsum[W + e] = <u~_j, u~_{j-1}>
      double dsum[XD ? 2 * W : W];
#pragma unroll
      for (int e = 0; e < (XD ? 2 * W : W); ++e) dsum[e] = 0.0;
      if (ZR && uprev) {
        // W_lo r_{j-1} = s L R + s Z - (beta s) u~_{j-2}, with the scalars of
        // step j-1 (still in st), in the FP32 path's rounding order
        const V sc = scur_of<T, 1>(st, cp, t.panel0, 0, false);
        const V scl = sc * T(1 << kXzTileBits);
        const V bp = bps_of<T, 1>(st, cp, t.panel0, 0);
        const V* zb = (const V*)sg.Y + (uint64_t)t.panel0 * pstride;
        const V* upp = j > 2 ? (const V*)slot_ptr<T>(sg, j - 2) + (uint64_t)t.panel0 * pstride : nullptr;
#pragma unroll
        for (int q = 0; q < kXzRegs; ++q) {
          const uint32_t row = row_of(xz_tau(0, l, q));
          V w = scl * v[q];
          if (upp) {
            const V u2 = ldg_sel<NT>(upp, row);
#pragma unroll
            for (int e = 0; e < W; ++e) w[e] = fma_s(-bp[e], u2[e], w[e]);
          }
          const V z = ldg_sel<NT>(zb, row);
#pragma unroll
          for (int e = 0; e < W; ++e) v[q][e] = fma_s(sc[e], z[e], w[e]);
        }
      }
      if (uprev) {
#pragma unroll
        for (int q = 0; q < kXzRegs; ++q) {
          const V up = ldg_sel<NT>(uprev, row_of(xz_tau(0, l, q)));
#pragma unroll
          for (int e = 0; e < W; ++e) {
            v[q][e] = fma_s(-acur[e], up[e], v[q][e]);
            if (XD) dsum[W + e] += (double)v[q][e] * (double)up[e];
          }
        }
      }
#pragma unroll
      for (int q = 0; q < kXzRegs; ++q) {
        stg(ucur, row_of(xz_tau(0, l, q)), v[q]);
#pragma unroll
        for (int e = 0; e < W; ++e) dsum[e] += (double)v[q][e] * (double)v[q][e];
      }
      if (REGEN) {
        const CONST_AS T* yt = (const CONST_AS T*)sg.ytab;
        for (int b = 0; b < sg.n_beta; ++b) {
          V* pb = (V*)sg.psi + (uint64_t)b * (sg.blk / W) + (uint64_t)t.panel0 * pstride;
          V y;
#pragma unroll
          for (int e = 0; e < W; ++e) y[e] = yt[((uint64_t)b * sg.k + (j - 1)) * cp + t.panel0 * W + e];
#pragma unroll
          for (int q = 0; q < kXzRegs; ++q) {
            const uint32_t row = row_of(xz_tau(0, l, q));
            V old;
            if (j == 1) {
#pragma unroll
              for (int e = 0; e < W; ++e) old[e] = T(0);
            } else {
              old = ldg((const V*)pb, row);
            }
            V nw;
#pragma unroll
            for (int e = 0; e < W; ++e) nw[e] = fma_s(y[e], v[q][e], old[e]);
            stg(pb, row, nw);
          }
        }
      }
      double tot;
      block_sum<XD ? 2 * W : W>(dsum, red, &tot);
      if (threadIdx.x < W) {
        sg.part[(uint64_t)t.rtile * cp + t.panel0 * W + threadIdx.x] = tot * (double)inv_l;
      } else if (XD && threadIdx.x < 2 * W) {
        sg.part[((uint64_t)XP_C * sg.x_tiles + t.rtile) * cp + t.panel0 * W + threadIdx.x - W] =
            tot * (double)inv_l;
      }
      if constexpr (GEOM == XG_SPLIT) {
        xz_group_transform<false>(v, lds, (const T*)nullptr, lrb, row_of);
      } else {
        double qf[W];
#pragma unroll
        for (int e = 0; e < W; ++e) qf[e] = 0.0;
        xz_high_transform<DEEP, XD>(v, lds, (const T*)sg.dx, t.rtile, lrb, row_of, qf);
        if (XD) put_plane<W>(sg, XP_QX, t.rtile, t.panel0, qf, red);
      }
#pragma unroll
      for (int q = 0; q < kXzRegs; ++q) stg_sel<NT>(rb, row_of(xz_tau(0, l, q)), v[q]);
    };
    if (!DEEP || lrb >= 3) run(std::true_type{});
    else run(std::false_type{});
    return;
  }

  if (PASS == 3) {
    // contiguous tile: Y = W_lo T W_lo u~_j / L = W_lo T u_j
    const V* ub = (const V*)slot_ptr<T>(sg, j) + (uint64_t)t.panel0 * pstride;
    V* yb = (V*)sg.Y + (uint64_t)t.panel0 * pstride;
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) v[q] = ldg(ub, t.row0 + xz_tau(0, l, q));
    xz_low_transform(v, lds);
    yy_twist<T>(v, t.row0, T(1) / T(1 << kXzTileBits));
    xz_low_transform(v, lds);
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) stg_stream<true>(yb, t.row0 + xz_tau(0, l, q), v[q]);
    return;
  }
  if (PASS == 4) {
    // strided tile: Y = W_hi D_Y W_hi Y (FP64: and the XP_QY plane)
    constexpr bool QY = sizeof(T) == 8;
    double qf[W];
#pragma unroll
    for (int e = 0; e < W; ++e) qf[e] = 0.0;
    xz_strided_inplace<T, DEEP, QY>(sg, t, (V*)sg.Y + (uint64_t)t.panel0 * pstride, (const T*)sg.dy, lds, qf);
    if (QY && sg.mode == MODE_LANCZOS) put_plane<W>(sg, XP_QY, t.rtile, t.panel0, qf, red);
    return;
  }
  if (PASS == 5) {
    // contiguous tile: R += W_lo T W_lo Y / L, so that pass 2 finds
    // L R = L W_hi D_X W_hi u~_j + W_lo (T W D_Y W T u_j) in R
    const V* yb = (const V*)sg.Y + (uint64_t)t.panel0 * pstride;
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) v[q] = ldg_nt(yb, t.row0 + xz_tau(0, l, q));
    xz_low_transform(v, lds);
    yy_twist<T>(v, t.row0, inv_l);
    xz_low_transform(v, lds);
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) {
      const uint32_t row = t.row0 + xz_tau(0, l, q);
      stg_stream<true>(rb, row, ldg_nt((const V*)rb, row) + v[q]);
    }
    return;
  }

  // PASS 2: contiguous tile, row = row0 + tau
  const V* ub = (const V*)slot_ptr<T>(sg, j) + (uint64_t)t.panel0 * pstride;
  const T* dg = (const T*)sg.diag;
  if constexpr (ZR) {
    // FP64: Z = W_lo D_Z u_j into Y (the next strided pass completes the
    // recurrence) and the diagonal part of <u_j, r_j> (plane XP_A)
    T d[kXzRegs];
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) {
      const uint32_t row = t.row0 + xz_tau(0, l, q);
      v[q] = ldg_nt(ub, row);
      d[q] = ldg_s(dg, row);
    }
    double d2[W];
#pragma unroll
    for (int e = 0; e < W; ++e) d2[e] = 0.0;
    xz_low_transform(v, lds);      // L u
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) {
      const V u = v[q] * inv_l;
      v[q] = d[q] * u;             // D_Z u
#pragma unroll
      for (int e = 0; e < W; ++e) d2[e] += (double)u[e] * (double)v[q][e];
    }
    xz_low_transform(v, lds);      // W_lo D_Z u
    V* zb = (V*)sg.Y + (uint64_t)t.panel0 * pstride;
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) stg_stream<true>(zb, t.row0 + xz_tau(0, l, q), v[q]);
    if (XD && sg.mode == MODE_LANCZOS) put_plane<W>(sg, XP_A, t.rtile, t.panel0, d2, red);
    return;
  }
  V w[kXzRegs];
  T d[kXzRegs];
#pragma unroll
  for (int q = 0; q < kXzRegs; ++q) {
    const uint32_t row = t.row0 + xz_tau(0, l, q);
    v[q] = ldg_nt(ub, row);
    w[q] = ldg_nt((const V*)rb, row);
    d[q] = ldg_s(dg, row);
  }
  const V sc = scur_of<T, 1>(st, cp, t.panel0, 0, false);
  const V scl = sc * T(1 << kXzTileBits);
#pragma unroll
  for (int q = 0; q < kXzRegs; ++q) w[q] = scl * w[q];
  if (uprev) {
    const V bp = bps_of<T, 1>(st, cp, t.panel0, 0);
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q) {
      const V up = ldg_nt(uprev, t.row0 + xz_tau(0, l, q));
#pragma unroll
      for (int e = 0; e < W; ++e) w[q][e] = fma_s(-bp[e], up[e], w[q][e]);
    }
  }
  const bool dots = sg.mode == MODE_LANCZOS;
  double d1[W], d2[W];
#pragma unroll
  for (int e = 0; e < W; ++e) d1[e] = d2[e] = 0.0;
  if (dots) {
#pragma unroll
    for (int q = 0; q < kXzRegs; ++q)
#pragma unroll
      for (int e = 0; e < W; ++e) d1[e] += (double)v[q][e] * (double)w[q][e];
  }
  xz_low_transform(v, lds);        // L u
#pragma unroll
  for (int q = 0; q < kXzRegs; ++q) {
    const V u = v[q] * inv_l;
    v[q] = d[q] * u;               // D_Z u
    if (dots) {
#pragma unroll
      for (int e = 0; e < W; ++e) d2[e] += (double)u[e] * (double)v[q][e];
    }
  }
  xz_low_transform(v, lds);        // W_lo D_Z u
#pragma unroll
  for (int q = 0; q < kXzRegs; ++q) {
    V r;
#pragma unroll
    for (int e = 0; e < W; ++e) r[e] = fma_s(sc[e], v[q][e], w[q][e]);
    stg_stream<true>(rb, t.row0 + xz_tau(0, l, q), r);
  }
  if (!dots) return;
  double dq[W];
#pragma unroll
  for (int e = 0; e < W; ++e) dq[e] = (double)sc[e] * d2[e] + d1[e] * (double)inv_l;
  double tot;
  block_sum<W>(dq, red, &tot);
  if (threadIdx.x < W) sg.part[(uint64_t)t.rtile * cp + t.panel0 * W + threadIdx.x] = tot;
}

// ---------------------------------------------------------------------------
// Block Lanczos (Algorithm 1) on the DS start columns of each bath vector.
// A lane owns one row of CB = max(DS, W) consecutive columns (NG = CB / DS
// groups); every update mixes only the columns of one group.  Per-group
// partial sums of d_s x d_s products go to part[rt][g][DS*DS] (FP64, fixed
// order), reduced per group by k_block_reduce.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ typename PanelT<T>::V* blk_slot(const CONST_AS BSeg& bs, int j) {
  return (typename PanelT<T>::V*)bs.Q + (uint64_t)((j - 1) % 3) * (bs.blk / PanelT<T>::W);
}

template <typename T, int DS>
__global__ __launch_bounds__(kBlock) void k_block_update(const BSeg* __restrict__ bsp, int phase, int j) {
  using V = typename PanelT<T>::V;
  constexpr int W = PanelT<T>::W;
  constexpr int CB = DS > W ? DS : W;
  constexpr int NP = CB / W;
  constexpr int NG = CB / DS;
  constexpr int NE = DS * DS;
  __shared__ double lds[4 * NG * NE];
  const CONST_AS BSeg& bs = *(const CONST_AS BSeg*)bsp;
  const int rt = (int)blockIdx.x % bs.n_rt, cb = (int)blockIdx.x / bs.n_rt;
  const uint32_t dim = 1u << bs.nbits;
  const uint64_t ps = dim;
  const int p0 = cb * NP;
  const int g0 = cb * NG;
  const int G = bs.G;
  const CONST_AS double* mats = (const CONST_AS double*)bs.mats;
  auto mat = [&](int which, int i, int a, int b) -> T {
    return (T)mats[((uint64_t)which * G + g0 + i) * NE + a * DS + b];
  };
  V* qj = blk_slot<T>(bs, j) + (uint64_t)p0 * ps;
  V* qn = blk_slot<T>(bs, j + 1) + (uint64_t)p0 * ps;
  const V* qp = j > 1 ? (const V*)blk_slot<T>(bs, j - 1) + (uint64_t)p0 * ps : nullptr;
  V* rb = (V*)bs.R + (uint64_t)p0 * ps;
  double dq[NG * NE];
#pragma unroll
  for (int i = 0; i < NG * NE; ++i) dq[i] = 0.0;

  for (int rr = 0; rr < bs.rpl; ++rr) {
    const uint32_t row = ((uint32_t)rt * bs.rpl + rr) * kBlock + threadIdx.x;
    if (row >= dim) break;
    T x[CB], y[CB], out[CB];
    auto load = [&](const V* base, T (&dst)[CB]) {
#pragma unroll
      for (int pp = 0; pp < NP; ++pp) {
        const V v = ldg(base + pp * ps, row);
#pragma unroll
        for (int e = 0; e < W; ++e) dst[pp * W + e] = v[e];
      }
    };
    auto store = [&](V* base, const T (&src)[CB]) {
#pragma unroll
      for (int pp = 0; pp < NP; ++pp) {
        V v;
#pragma unroll
        for (int e = 0; e < W; ++e) v[e] = src[pp * W + e];
        stg(base + pp * ps, row, v);
      }
    };
    if (phase == BLK_A) {
      // Z = H q_j - q_{j-1} B_{j-1}^T ; A partials q_j^T Z
      load(rb, x);
      load(qj, y);
#pragma unroll
      for (int c = 0; c < CB; ++c) out[c] = x[c];
      if (qp) {
        T w[CB];
        load(qp, w);
#pragma unroll
        for (int i = 0; i < NG; ++i)
#pragma unroll
          for (int a = 0; a < DS; ++a)
#pragma unroll
            for (int b = 0; b < DS; ++b) out[i * DS + a] = fma_s(-w[i * DS + b], mat(BM_BPREV, i, a, b), out[i * DS + a]);
      }
      store(rb, out);
#pragma unroll
      for (int i = 0; i < NG; ++i)
#pragma unroll
        for (int a = 0; a < DS; ++a)
#pragma unroll
          for (int b = 0; b < DS; ++b)
            dq[i * NE + a * DS + b] += (double)y[i * DS + a] * (double)out[i * DS + b];
    } else if (phase == BLK_G) {
      // Z <- Z - q_j A_j ; Gram partials Z^T Z
      load(rb, x);
      load(qj, y);
#pragma unroll
      for (int i = 0; i < NG; ++i)
#pragma unroll
        for (int a = 0; a < DS; ++a) {
          T z = x[i * DS + a];
#pragma unroll
          for (int b = 0; b < DS; ++b) z = fma_s(-y[i * DS + b], mat(BM_A, i, b, a), z);
          out[i * DS + a] = z;
        }
      store(rb, out);
#pragma unroll
      for (int i = 0; i < NG; ++i)
#pragma unroll
        for (int a = 0; a < DS; ++a)
#pragma unroll
          for (int b = 0; b < DS; ++b)
            dq[i * NE + a * DS + b] += (double)out[i * DS + a] * (double)out[i * DS + b];
    } else {
      // phase 2: q_{j+1} = Z R^-1 (Gram partials for the second pass);
      // phase 3: q_{j+1} <- q_{j+1} R^-1
      load(phase == BLK_G2 ? (const V*)rb : (const V*)qn, x);
#pragma unroll
      for (int i = 0; i < NG; ++i)
#pragma unroll
        for (int a = 0; a < DS; ++a) {
          T z = T(0);
#pragma unroll
          for (int b = 0; b <= a; ++b) z = fma_s(x[i * DS + b], mat(BM_RINV, i, b, a), z);
          out[i * DS + a] = z;
        }
      store(qn, out);
      if (phase == BLK_G2) {
#pragma unroll
        for (int i = 0; i < NG; ++i)
#pragma unroll
          for (int a = 0; a < DS; ++a)
#pragma unroll
            for (int b = 0; b < DS; ++b)
              dq[i * NE + a * DS + b] += (double)out[i * DS + a] * (double)out[i * DS + b];
      }
    }
  }
  if (phase > BLK_G2) return;
  double tot;
  block_sum<NG * NE>(dq, lds, &tot);
  if (threadIdx.x < NG * NE) bs.part[((uint64_t)rt * G + g0) * NE + threadIdx.x] = tot;
}

// Cholesky G = R^T R (R upper triangular, row-major DS x DS); returns the
// smallest pivot R[i][i] (<= 0 or NaN when G is not positive definite).
template <int DS>
__device__ double small_chol(const double* g, double* r) {
  double mn = INFINITY;
  for (int i = 0; i < DS * DS; ++i) r[i] = 0.0;
  for (int i = 0; i < DS; ++i) {
    double d = g[i * DS + i];
    for (int k = 0; k < i; ++k) d -= r[k * DS + i] * r[k * DS + i];
    if (!(d > 0.0)) return d > 0.0 ? mn : (d == d ? 0.0 : d);
    const double rii = sqrt(d);
    r[i * DS + i] = rii;
    mn = fmin(mn, rii);
    for (int jj = i + 1; jj < DS; ++jj) {
      double v = g[i * DS + jj];
      for (int k = 0; k < i; ++k) v -= r[k * DS + i] * r[k * DS + jj];
      r[i * DS + jj] = v / rii;
    }
  }
  return mn;
}
// inverse of an upper-triangular R with positive diagonal
template <int DS>
__device__ void small_triinv(const double* r, double* ri) {
  for (int i = 0; i < DS * DS; ++i) ri[i] = 0.0;
  for (int c = 0; c < DS; ++c) {
    ri[c * DS + c] = 1.0 / r[c * DS + c];
    for (int i = c - 1; i >= 0; --i) {
      double v = 0.0;
      for (int k = i + 1; k <= c; ++k) v += r[i * DS + k] * ri[k * DS + c];
      ri[i * DS + c] = -v / r[i * DS + i];
    }
  }
}

// one workgroup per group: sum the row-tile partials (fixed order), then the
// small-matrix step of the phase
template <int DS>
__global__ __launch_bounds__(kBlock) void k_block_reduce(const BSeg* __restrict__ bsp, int phase, int j) {
  constexpr int NE = DS * DS;
  const BSeg& bs = *bsp;
  const int g = blockIdx.x, G = bs.G;
  __shared__ double red[kBlock];
  __shared__ double tot[NE];
  for (int e = 0; e < NE; ++e) {
    double acc = 0.0;
    for (int t = threadIdx.x; t < bs.n_rt; t += kBlock) acc += bs.part[((uint64_t)t * G + g) * NE + e];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) tot[e] = red[0];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  auto M = [&](int which) { return bs.mats + ((uint64_t)which * G + g) * NE; };
  double* sc = M(BM_SCALE);
  const bool frozen = sc[1] != 0.0;
  if (phase == BLK_A) {
    double* a = M(BM_A);
    double mx = sc[0];
    for (int p = 0; p < DS; ++p)
      for (int q = 0; q < DS; ++q) {
        const double v = frozen ? 0.0 : 0.5 * (tot[p * DS + q] + tot[q * DS + p]);
        a[p * DS + q] = v;
        bs.a_hist[((uint64_t)(j - 1) * G + g) * NE + p * DS + q] = v;
        mx = fmax(mx, fabs(v));
      }
    sc[0] = mx;
    return;
  }
  double r[NE], ri[NE];
  if (phase == BLK_G) {
    const double mn = frozen ? 0.0 : small_chol<DS>(tot, r);
    if (frozen || !(mn > bs.tau * sc[0])) {
      // breakdown: the block Krylov space closed (to the threshold) after j blocks
      if (!frozen) bs.kc[g] = j;
      sc[1] = 1.0;
      for (int i = 0; i < NE; ++i) M(BM_RINV)[i] = M(BM_R1)[i] = M(BM_BPREV)[i] = 0.0;
      return;
    }
    small_triinv<DS>(r, ri);
    for (int i = 0; i < NE; ++i) {
      M(BM_R1)[i] = r[i];
      M(BM_RINV)[i] = ri[i];
    }
    return;
  }
  // BLK_G2: second Cholesky pass; B_j = R2 R1
  if (frozen) {
    for (int i = 0; i < NE; ++i) M(BM_RINV)[i] = M(BM_BPREV)[i] = 0.0;
    return;
  }
  const double mn = small_chol<DS>(tot, r);
  if (!(mn > 0.0)) {
    bs.kc[g] = j;
    sc[1] = 1.0;
    for (int i = 0; i < NE; ++i) M(BM_RINV)[i] = M(BM_BPREV)[i] = 0.0;
    return;
  }
  small_triinv<DS>(r, ri);
  const double* r1 = M(BM_R1);
  double mx = sc[0];
  for (int p = 0; p < DS; ++p)
    for (int q = 0; q < DS; ++q) {
      double v = 0.0;
      for (int t = 0; t < DS; ++t) v += r[p * DS + t] * r1[t * DS + q];
      M(BM_BPREV)[p * DS + q] = v;
      bs.b_hist[((uint64_t)(j - 1) * G + g) * NE + p * DS + q] = v;
      mx = fmax(mx, fabs(v));
    }
  sc[0] = mx;
  for (int i = 0; i < NE; ++i) M(BM_RINV)[i] = ri[i];
}

// ---------------------------------------------------------------------------
// ground-space partial trace (low-temperature limit): one lane per bath index
// b, the DS system states m in registers, one pass over the stored blocks
// ---------------------------------------------------------------------------
template <typename T, int DS>
__global__ __launch_bounds__(kBlock) void k_ground_ptrace(const GPSeg* __restrict__ gpp) {
  using V = typename PanelT<T>::V;
  constexpr int W = PanelT<T>::W;
  constexpr int RMAX = 4;
  constexpr int NE = DS * DS;
  __shared__ double lds[4 * NE];
  const CONST_AS GPSeg& gp = *(const CONST_AS GPSeg*)gpp;
  const uint32_t db = 1u << gp.nb;
  const uint64_t dim = 1ull << gp.nbits;
  const int P = gp.cpad / W;
  const CONST_AS T* w = (const CONST_AS T*)gp.w;
  double acc[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) acc[i] = 0.0;
  for (int rr = 0; rr < gp.rpl; ++rr) {
    const uint32_t b = ((uint32_t)blockIdx.x * gp.rpl + rr) * kBlock + threadIdx.x;
    if (b >= db) break;
    T phi[RMAX][DS];
#pragma unroll
    for (int i = 0; i < RMAX; ++i)
#pragma unroll
      for (int m = 0; m < DS; ++m) phi[i][m] = T(0);
    for (int j = 0; j < gp.k; ++j) {
      const V* qj = (const V*)gp.Q + (uint64_t)j * (gp.blk / W);
      for (int p = 0; p < P; ++p) {
#pragma unroll
        for (int m = 0; m < DS; ++m) {
          const V v = ldg(qj + (uint64_t)p * dim, ((uint32_t)m << gp.nb) | b);
#pragma unroll
          for (int e = 0; e < W; ++e)
#pragma unroll
            for (int i = 0; i < RMAX; ++i)
              if (i < gp.R) phi[i][m] = fma_s(w[((uint64_t)j * gp.R + i) * gp.cpad + p * W + e], v[e], phi[i][m]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < RMAX; ++i)
      if (i < gp.R)
#pragma unroll
        for (int m = 0; m < DS; ++m)
#pragma unroll
          for (int n = 0; n < DS; ++n) acc[m * DS + n] += (double)phi[i][m] * (double)phi[i][n];
  }
  double tot;
  block_sum<NE>(acc, lds, &tot);
  if (threadIdx.x < NE) gp.part[(uint64_t)blockIdx.x * NE + threadIdx.x] = tot;
}

// ---------------------------------------------------------------------------
// reductions of the per-tile partial sums: one workgroup per (segment,
// column); lane i sums tiles i, i+256, ... and a fixed binary tree in LDS
// combines the lanes, so the order never depends on scheduling.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double column_total(const Seg& sg, int nrows, int c, double* lds) {
  double s = 0.0;
  for (int t = threadIdx.x; t < nrows; t += kBlock) s += sg.part[(uint64_t)t * sg.cpad + c];
  lds[threadIdx.x] = s;
  __syncthreads();
#pragma unroll
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
    __syncthreads();
  }
  return lds[0];
}

// beta_{j-1} = |u_j| (or |u_1| -> s_1 at j = 1), breakdown test, scales.
__global__ __launch_bounds__(kBlock) void k_red_beta(const Seg* __restrict__ segs) {
  const Seg& sg = segs[blockIdx.x];
  const int c = blockIdx.y;
  if (c >= sg.cpad) return;
  __shared__ double lds[kBlock];
  const double tot = column_total(sg, sg.nm_rows, c, lds);
  if (threadIdx.x != 0) return;
  const int j = sg.stepc[c];
  if (j > sg.k) return;
  const int cp = sg.cpad;
  double* st = sg.st;
  const bool frozen = st[ST_FROZEN * cp + c] != 0.0;
  double s, beff;
  if (sg.mode == MODE_REGEN) {
    s = sg.h_s[(uint64_t)(j - 1) * cp + c];
    beff = (j == 1) ? 0.0 : sg.h_beta[(uint64_t)(j - 2) * cp + c];
  } else if (j == 1) {
    beff = 0.0;
    s = frozen ? 0.0 : 1.0 / sqrt(tot);
    st[ST_RUNMAX * cp + c] = 0.0;
  } else {
    const double b = sqrt(tot);
    const double runmax = st[ST_RUNMAX * cp + c];
    if (frozen) {
      beff = 0.0;
      s = 0.0;
    } else if (!(b > sg.tau * runmax)) {
      st[ST_FROZEN * cp + c] = 1.0;
      sg.kc[c] = j - 1;
      beff = 0.0;
      s = 0.0;
    } else {
      st[ST_RUNMAX * cp + c] = fmax(runmax, b);
      beff = b;
      s = 1.0 / b;
    }
    sg.h_beta[(uint64_t)(j - 2) * cp + c] = beff;
  }
  if (sg.mode != MODE_REGEN) sg.h_s[(uint64_t)(j - 1) * cp + c] = s;
  const double sprev = (j == 1) ? 0.0 : st[ST_SCUR * cp + c];
  st[ST_BPS * cp + c] = beff * sprev;
  st[ST_SPREV * cp + c] = sprev;
  st[ST_SCUR * cp + c] = s;
}

// <u_j, r_j> of an FP64 transform step from its partial-sum planes (XP_*):
// per tile s_j (A + QX [+ QY]) - (beta s)_{j-1} C, then the fixed tree.
__device__ __forceinline__ double xdots_total(const Seg& sg, int c, double* lds) {
  const int cp = sg.cpad;
  const double sc = sg.st[ST_SCUR * cp + c], bp = sg.st[ST_BPS * cp + c];
  const uint64_t ps = (uint64_t)sg.x_tiles * cp;
  double s = 0.0;
  for (int t = threadIdx.x; t < sg.x_tiles; t += kBlock) {
    const double* p = sg.part + (uint64_t)t * cp + c;
    double q = p[XP_A * ps] + p[XP_QX * ps];
    if (sg.xy) q += p[XP_QY * ps];
    s += sc * q - bp * p[XP_C * ps];
  }
  lds[threadIdx.x] = s;
  __syncthreads();
#pragma unroll
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
    __syncthreads();
  }
  return lds[0];
}

// alpha_j = s_j <u_j, r>; weight alpha_j s_j for the next step; advance.
__global__ __launch_bounds__(kBlock) void k_red_alpha(const Seg* __restrict__ segs) {
  const Seg& sg = segs[blockIdx.x];
  const int c = blockIdx.y;
  if (c >= sg.cpad) return;
  __shared__ double lds[kBlock];
  const double tot = sg.xdots && sg.mode == MODE_LANCZOS ? xdots_total(sg, c, lds)
                                                         : column_total(sg, sg.ap_rows, c, lds);
  if (threadIdx.x != 0) return;
  const int j = sg.stepc[c];
  if (j > sg.k) return;
  const int cp = sg.cpad;
  double* st = sg.st;
  double a;
  if (sg.mode == MODE_REGEN) {
    a = sg.h_alpha[(uint64_t)(j - 1) * cp + c];
  } else {
    const bool frozen = st[ST_FROZEN * cp + c] != 0.0;
    a = frozen ? 0.0 : st[ST_SCUR * cp + c] * tot;
    st[ST_RUNMAX * cp + c] = fmax(st[ST_RUNMAX * cp + c], fabs(a));
    sg.h_alpha[(uint64_t)(j - 1) * cp + c] = a;
  }
  st[ST_ACUR * cp + c] = a * st[ST_SCUR * cp + c];
  sg.stepc[c] = j + 1;
}

// ---------------------------------------------------------------------------
// recombination psi_b = sum_j y'_{b,j} u_j (fused) and the per-bath-vector
// d_s x d_s Gram blocks, accumulated per lane over its rows in T and summed
// across lanes / tiles in FP64.
// ---------------------------------------------------------------------------
// PART 0: the whole d_s x d_s Gram (d_s <= 8).  d_s = 16 takes three
// launches over the column halves A = 0..7 and B = 8..15 of each bath
// vector: PART 1 the block AA, 2 the block AB, 3 the block BB (each block's
// products in registers; only the panels a block needs are read).
template <int DS, int PART> struct GramBlock {
  static constexpr int M0 = PART == 3 ? DS / 2 : 0;
  static constexpr int M1 = PART == 0 ? DS : (PART == 3 ? DS : DS / 2);
  static constexpr int N0 = PART == 2 || PART == 3 ? DS / 2 : 0;
  static constexpr int N1 = PART == 1 ? DS / 2 : DS;
  static constexpr bool TRI = PART != 2;  // a diagonal block: n >= m only
  static constexpr int NE = TRI ? (M1 - M0) * (M1 - M0 + 1) / 2 : (M1 - M0) * (N1 - N0);
  static constexpr int C0 = M0 < N0 ? M0 : N0, C1 = M1 > N1 ? M1 : N1;  // columns read
};

template <typename T, int DS, int NB, int PART>
__global__ __launch_bounds__(kBlock) void k_gram(const GSeg* __restrict__ gsegs,
                                                 const GTile* __restrict__ tiles, int beta0) {
  using V = typename PanelT<T>::V;
  using GB = GramBlock<DS, PART>;
  constexpr int W = PanelT<T>::W;
  constexpr int CB = DS > W ? DS : W;
  constexpr int NPAN = CB / W;
  constexpr int Q0 = GB::C0 / W, Q1 = (GB::C1 + W - 1) / W;  // panels read
  constexpr int NG = CB / DS;
  constexpr int NE = GB::NE;
  constexpr int NV = NB * NG * NE;
  extern __shared__ double smem[];
  double* lds = smem;                       // 4 * NV doubles
  T* ys = (T*)(smem + 4 * NV);              // [k][NB][CB]
  const GTile t = tiles[blockIdx.x];
  const GSeg& g = gsegs[t.seg];
  const uint32_t dim = 1u << g.nbits;
  const uint64_t pstride = dim;
  const int nb = (g.n_beta - beta0) < NB ? (g.n_beta - beta0) : NB;
  const int k = g.k, cp = g.cpad;
  const int col0 = t.cblock * CB;
  if (!g.from_psi) {
    const T* yt = (const T*)g.ytab;
    for (int i = threadIdx.x; i < k * NB * CB; i += kBlock) {
      const int jj = i / (NB * CB), rem = i % (NB * CB), b = rem / CB, cc = rem % CB;
      ys[i] = (b < nb) ? yt[((uint64_t)(beta0 + b) * k + jj) * cp + col0 + cc] : T(0);
    }
    __syncthreads();
  }
  T gacc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) gacc[i] = T(0);

  for (int rr = 0; rr < g.rpl; ++rr) {
    const uint32_t row = t.row0 + rr * kBlock + threadIdx.x;
    if (row >= dim) break;
    V psi[NB][NPAN];
    if (g.from_psi) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int q = Q0; q < Q1; ++q) {
          if (b < nb) {
            const V* pb = (const V*)g.Q + (uint64_t)(beta0 + b) * (g.blk / W) +
                          (uint64_t)(t.cblock * NPAN + q) * pstride;
            psi[b][q] = ldg_nt(pb, row);
          } else {
#pragma unroll
            for (int e = 0; e < W; ++e) psi[b][q][e] = T(0);
          }
        }
    } else {
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int q = 0; q < NPAN; ++q)
#pragma unroll
          for (int e = 0; e < W; ++e) psi[b][q][e] = T(0);
      for (int jj = 0; jj < k; ++jj) {
        const V* sb = (const V*)g.Q + (uint64_t)jj * (g.blk / W);
        V qv[NPAN];
#pragma unroll
        for (int q = Q0; q < Q1; ++q) qv[q] = ldg_nt(sb + (uint64_t)(t.cblock * NPAN + q) * pstride, row);
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int q = Q0; q < Q1; ++q)
#pragma unroll
            for (int e = 0; e < W; ++e)
              psi[b][q][e] = fma_s(ys[(jj * NB + b) * CB + q * W + e], qv[q][e], psi[b][q][e]);
      }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int gg = 0; gg < NG; ++gg) {
        int e = 0;
#pragma unroll
        for (int m = GB::M0; m < GB::M1; ++m)
#pragma unroll
          for (int n = GB::TRI ? m : GB::N0; n < GB::N1; ++n) {
            const int cm = gg * DS + m, cn = gg * DS + n;
            const T pm = psi[b][cm / W][cm % W], pn = psi[b][cn / W][cn % W];
            gacc[(b * NG + gg) * NE + e] = fma_s(pm, pn, gacc[(b * NG + gg) * NE + e]);
            ++e;
          }
      }
  }
  double gv[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) gv[i] = (double)gacc[i];
  double tot;
  block_sum<NV>(gv, lds, &tot);
  if (threadIdx.x < NV) {
    const int i = threadIdx.x;
    const int b = i / (NG * NE), gg = (i / NE) % NG, e = i % NE;
    const int jv = t.cblock * NG + gg;
    if (b < nb && jv < g.n_v) {
      int m, n;
      if (GB::TRI) {
        int rem = e;
        m = GB::M0;
        while (rem >= GB::M1 - m) { rem -= GB::M1 - m; ++m; }
        n = m + rem;
      } else {
        m = GB::M0 + e / (GB::N1 - GB::N0);
        n = GB::N0 + e % (GB::N1 - GB::N0);
      }
      double* o = g.gpart + ((((uint64_t)t.rtile * g.n_beta + beta0 + b) * g.n_v + jv) * DS) * DS;
      o[m * DS + n] = tot;
      o[n * DS + m] = tot;
    }
  }
}

// out[w] = sum over rows of part[row][w], rows summed in a fixed order.
__global__ __launch_bounds__(kBlock) void k_colsum(const double* __restrict__ part, int nrows,
                                                   int width, double* __restrict__ out) {
  __shared__ double lds[4][64];
  const int cl = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int w = blockIdx.x * 64 + cl;
  double s = 0.0;
  if (w < width)
    for (int r = grp; r < nrows; r += 4) s += part[(uint64_t)r * width + w];
  lds[grp][cl] = s;
  __syncthreads();
  if (grp == 0 && w < width) out[w] = ((lds[0][cl] + lds[1][cl]) + lds[2][cl]) + lds[3][cl];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_start_block(int ns_log, int nb, int C, uint64_t seed,
                                                        int kind, T* __restrict__ out,
                                                        uint32_t dim, int cpad) {
  using V = typename PanelT<T>::V;
  constexpr int W = PanelT<T>::W;
  const uint32_t row = blockIdx.x * kBlock + threadIdx.x;
  const int panel = blockIdx.y;
  if (row >= dim) return;
  const T amp = amp_of<T>(nb);
  V u;
#pragma unroll
  for (int e = 0; e < W; ++e) u[e] = start_value<T>(kind, ns_log, nb, seed, row, panel * W + e, C, amp);
  stg((V*)out + (uint64_t)panel * dim, row, u);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_diag(const DiagTerm* terms, int nt, T* diag, int nbits, hipStream_t st, bool xz_tiled) {
  const uint32_t dim = 1u << nbits;
  if (xz_tiled && xz_geom(nbits) != XG_DEEP) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_diag<T>, dim3((dim + kBlock - 1) / kBlock), dim3(kBlock), 0, st, terms, nt,
                     diag, dim, xz_tiled ? 2 * kXzTileBits - nbits : -1);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_norm(const Seg* segs, int nseg, int ntiles, int slab, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  switch (slab) {
    case 1: hipLaunchKernelGGL((k_norm<T, 1>), dim3(ntiles), dim3(kBlock), 0, st, segs, nseg); break;
    case 2: hipLaunchKernelGGL((k_norm<T, 2>), dim3(ntiles), dim3(kBlock), 0, st, segs, nseg); break;
    default: hipLaunchKernelGGL((k_norm<T, 4>), dim3(ntiles), dim3(kBlock), 0, st, segs, nseg); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply(const Seg* segs, int nseg, int ntiles, int slab, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  switch (slab) {
    case 1: hipLaunchKernelGGL((k_apply<T, 1>), dim3(ntiles), dim3(kBlock), 0, st, segs, nseg); break;
    case 2: hipLaunchKernelGGL((k_apply<T, 2>), dim3(ntiles), dim3(kBlock), 0, st, segs, nseg); break;
    default: hipLaunchKernelGGL((k_apply<T, 4>), dim3(ntiles), dim3(kBlock), 0, st, segs, nseg); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply_wide(const Seg* segs, int nseg, int ntiles, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_apply_wide<T>), dim3(ntiles), dim3(kWideBlock), 0, st, segs, nseg);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xz_split(int op, const Seg* segs, int nseg, int ntiles, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  const dim3 g(ntiles), b(kBlock);
  switch (op) {
    case 0: hipLaunchKernelGGL((k_xz_split<T, 0>), g, b, 0, st, segs, nseg); break;
    case 1: hipLaunchKernelGGL((k_xz_split<T, 1>), g, b, 0, st, segs, nseg); break;
    case 2: hipLaunchKernelGGL((k_xz_split<T, 2>), g, b, 0, st, segs, nseg); break;
    case 3: hipLaunchKernelGGL((k_xz_split<T, 3>), g, b, 0, st, segs, nseg); break;
    case 4: hipLaunchKernelGGL((k_xz_split<T, 4>), g, b, 0, st, segs, nseg); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xz_pass(int pass, const Seg* segs, int nseg, int ntiles, hipStream_t st, int geo) {
  if (ntiles <= 0) return hipSuccess;
  const dim3 g(ntiles), b(kBlock);
  const bool deep = geo == XG_DEEP;
  if (geo == XG_SPLIT && (pass == 1 || pass == 4 || pass == 7)) {
    // W_hi D W_hi = W_A (W_B D W_B) W_A as three passes
    const int ops[3][3] = {{0, 1, 0}, {4, 1, 0}, {2, 3, 2}};
    const int* o = ops[pass == 1 ? 0 : pass == 4 ? 1 : 2];
    for (int i = 0; i < 3; ++i) {
      const hipError_t e = launch_xz_split<T>(o[i], segs, nseg, ntiles, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if (pass == 0) hipLaunchKernelGGL((k_apply_xz<T, 0, false>), g, b, 0, st, segs, nseg);
  else if (pass == 1 && deep) hipLaunchKernelGGL((k_apply_xz<T, 1, true>), g, b, 0, st, segs, nseg);
  else if (pass == 1) hipLaunchKernelGGL((k_apply_xz<T, 1, false>), g, b, 0, st, segs, nseg);
  else if (pass == 2) hipLaunchKernelGGL((k_apply_xz<T, 2, false>), g, b, 0, st, segs, nseg);
  else if (pass == 3) hipLaunchKernelGGL((k_apply_xz<T, 3, false>), g, b, 0, st, segs, nseg);
  else if (pass == 4 && deep) hipLaunchKernelGGL((k_apply_xz<T, 4, true>), g, b, 0, st, segs, nseg);
  else if (pass == 4) hipLaunchKernelGGL((k_apply_xz<T, 4, false>), g, b, 0, st, segs, nseg);
  else if (pass == 5) hipLaunchKernelGGL((k_apply_xz<T, 5, false>), g, b, 0, st, segs, nseg);
  else if (pass == 6) hipLaunchKernelGGL((k_apply_xz<T, 6, false>), g, b, 0, st, segs, nseg);
  else if (pass == 7 && deep) hipLaunchKernelGGL((k_apply_xz<T, 7, true>), g, b, 0, st, segs, nseg);
  else if (pass == 7) hipLaunchKernelGGL((k_apply_xz<T, 7, false>), g, b, 0, st, segs, nseg);
  else if (pass == 8) hipLaunchKernelGGL((k_apply_xz<T, 8, false>), g, b, 0, st, segs, nseg);
  else if (pass == 9) hipLaunchKernelGGL((k_apply_xz<T, 9, false>), g, b, 0, st, segs, nseg);
  else if (pass == 10) hipLaunchKernelGGL((k_apply_xz<T, 10, false>), g, b, 0, st, segs, nseg);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xz_lanczos(int pass, bool regen, const Seg* segs, int nseg, int ntiles, int boff, hipStream_t st,
                             int geo) {
  if (ntiles <= 0) return hipSuccess;
  const dim3 g(ntiles), b(kBlock);
#define RDM_XZL(P, R, G) hipLaunchKernelGGL((k_xz_lanczos<T, P, R, G>), g, b, 0, st, segs, nseg, boff)
  if (pass == 0) RDM_XZL(0, false, XG_SHALLOW);
  else if (pass == 1) {
    if (regen && geo == XG_SPLIT) RDM_XZL(1, true, XG_SPLIT);
    else if (regen && geo == XG_DEEP) RDM_XZL(1, true, XG_DEEP);
    else if (regen) RDM_XZL(1, true, XG_SHALLOW);
    else if (geo == XG_SPLIT) RDM_XZL(1, false, XG_SPLIT);
    else if (geo == XG_DEEP) RDM_XZL(1, false, XG_DEEP);
    else RDM_XZL(1, false, XG_SHALLOW);
  } else if (pass == 2) RDM_XZL(2, false, XG_SHALLOW);
  else if (pass == 3) RDM_XZL(3, false, XG_SHALLOW);
  else if (pass == 4 && geo == XG_DEEP) RDM_XZL(4, false, XG_DEEP);
  else if (pass == 4 && geo == XG_SHALLOW) RDM_XZL(4, false, XG_SHALLOW);
  else if (pass == 5) RDM_XZL(5, false, XG_SHALLOW);
  else return hipErrorInvalidValue;
#undef RDM_XZL
  return hipGetLastError();
}

template <typename T>
hipError_t launch_block_update(const BSeg* bs, int ds, int phase, int j, int n_rt, int n_cb, hipStream_t st) {
  const dim3 grid(n_rt * n_cb), blk(kBlock);
  switch (ds) {
    case 2: hipLaunchKernelGGL((k_block_update<T, 2>), grid, blk, 0, st, bs, phase, j); break;
    case 4: hipLaunchKernelGGL((k_block_update<T, 4>), grid, blk, 0, st, bs, phase, j); break;
    default: hipLaunchKernelGGL((k_block_update<T, 8>), grid, blk, 0, st, bs, phase, j); break;
  }
  return hipGetLastError();
}

hipError_t launch_block_reduce(const BSeg* bs, int ds, int G, int phase, int j, hipStream_t st) {
  switch (ds) {
    case 2: hipLaunchKernelGGL((k_block_reduce<2>), dim3(G), dim3(kBlock), 0, st, bs, phase, j); break;
    case 4: hipLaunchKernelGGL((k_block_reduce<4>), dim3(G), dim3(kBlock), 0, st, bs, phase, j); break;
    default: hipLaunchKernelGGL((k_block_reduce<8>), dim3(G), dim3(kBlock), 0, st, bs, phase, j); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ground_ptrace(const GPSeg* gp, int ds, int n_tiles, hipStream_t st) {
  switch (ds) {
    case 2: hipLaunchKernelGGL((k_ground_ptrace<T, 2>), dim3(n_tiles), dim3(kBlock), 0, st, gp); break;
    case 4: hipLaunchKernelGGL((k_ground_ptrace<T, 4>), dim3(n_tiles), dim3(kBlock), 0, st, gp); break;
    default: hipLaunchKernelGGL((k_ground_ptrace<T, 8>), dim3(n_tiles), dim3(kBlock), 0, st, gp); break;
  }
  return hipGetLastError();
}

hipError_t launch_red_beta(const Seg* segs, int nseg, int cmax, hipStream_t st) {
  if (nseg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_red_beta, dim3(nseg, cmax), dim3(kBlock), 0, st, segs);
  return hipGetLastError();
}

hipError_t launch_red_alpha(const Seg* segs, int nseg, int cmax, hipStream_t st) {
  if (nseg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_red_alpha, dim3(nseg, cmax), dim3(kBlock), 0, st, segs);
  return hipGetLastError();
}

hipError_t launch_init_state(const Seg* segs, int nseg, int cmax, int phase, hipStream_t st) {
  if (nseg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_state, dim3(nseg, (cmax + 63) / 64), dim3(64), 0, st, segs, phase);
  return hipGetLastError();
}

template <typename T, int DS, int NB, int PART = 0>
static hipError_t launch_gram_t(const GSeg* gs, const GTile* tiles, int ntiles, int beta0, int k,
                                hipStream_t st) {
  constexpr int W = PanelT<T>::W;
  constexpr int CB = DS > W ? DS : W;
  constexpr int NG = CB / DS;
  constexpr int NE = GramBlock<DS, PART>::NE;
  constexpr int NV = NB * NG * NE;
  const size_t shm = 4 * NV * sizeof(double) + (size_t)k * NB * CB * sizeof(T);
  hipLaunchKernelGGL((k_gram<T, DS, NB, PART>), dim3(ntiles), dim3(kBlock), shm, st, gs, tiles, beta0);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gram(const GSeg* gs, const GTile* tiles, int ntiles, int ds, int nb_chunk,
                       int beta0, int k, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
#define RDM_G(DSV, NBV) \
  if (ds == DSV && nb_chunk == NBV) return launch_gram_t<T, DSV, NBV>(gs, tiles, ntiles, beta0, k, st);
  RDM_G(2, 1) RDM_G(2, 2) RDM_G(2, 4) RDM_G(4, 1) RDM_G(4, 2) RDM_G(4, 4)
  RDM_G(8, 1) RDM_G(8, 2)
#undef RDM_G
  if (ds == 16 && nb_chunk == 1) {
    hipError_t e = launch_gram_t<T, 16, 1, 1>(gs, tiles, ntiles, beta0, k, st);
    if (e == hipSuccess) e = launch_gram_t<T, 16, 1, 2>(gs, tiles, ntiles, beta0, k, st);
    if (e == hipSuccess) e = launch_gram_t<T, 16, 1, 3>(gs, tiles, ntiles, beta0, k, st);
    return e;
  }
  return hipErrorInvalidValue;
}

hipError_t launch_colsum(const double* part, int nrows, int width, double* out, hipStream_t st) {
  if (width <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_colsum, dim3((width + 63) / 64), dim3(kBlock), 0, st, part, nrows, width, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_start_block(int ns_log, int nb, int C, uint64_t seed, int kind, T* out, int nbits,
                              int cpad, hipStream_t st) {
  constexpr int W = PanelT<T>::W;
  const uint32_t dim = 1u << nbits;
  hipLaunchKernelGGL(k_start_block<T>, dim3((dim + kBlock - 1) / kBlock, cpad / W), dim3(kBlock), 0,
                     st, ns_log, nb, C, seed, kind, out, dim, cpad);
  return hipGetLastError();
}

template hipError_t launch_diag<float>(const DiagTerm*, int, float*, int, hipStream_t, bool);
template hipError_t launch_diag<double>(const DiagTerm*, int, double*, int, hipStream_t, bool);
template hipError_t launch_norm<float>(const Seg*, int, int, int, hipStream_t);
template hipError_t launch_norm<double>(const Seg*, int, int, int, hipStream_t);
template hipError_t launch_apply<float>(const Seg*, int, int, int, hipStream_t);
template hipError_t launch_apply<double>(const Seg*, int, int, int, hipStream_t);
template hipError_t launch_apply_wide<float>(const Seg*, int, int, hipStream_t);
template hipError_t launch_apply_wide<double>(const Seg*, int, int, hipStream_t);
template hipError_t launch_xz_pass<float>(int, const Seg*, int, int, hipStream_t, int);
template hipError_t launch_xz_split<float>(int, const Seg*, int, int, hipStream_t);
template hipError_t launch_xz_split<double>(int, const Seg*, int, int, hipStream_t);
template hipError_t launch_block_update<float>(const BSeg*, int, int, int, int, int, hipStream_t);
template hipError_t launch_ground_ptrace<float>(const GPSeg*, int, int, hipStream_t);
template hipError_t launch_ground_ptrace<double>(const GPSeg*, int, int, hipStream_t);
template hipError_t launch_block_update<double>(const BSeg*, int, int, int, int, int, hipStream_t);
template hipError_t launch_xz_pass<double>(int, const Seg*, int, int, hipStream_t, int);
template hipError_t launch_xz_lanczos<float>(int, bool, const Seg*, int, int, int, hipStream_t, int);
template hipError_t launch_xz_lanczos<double>(int, bool, const Seg*, int, int, int, hipStream_t, int);
template hipError_t launch_gram<float>(const GSeg*, const GTile*, int, int, int, int, int, hipStream_t);
template hipError_t launch_gram<double>(const GSeg*, const GTile*, int, int, int, int, int, hipStream_t);
template hipError_t launch_start_block<float>(int, int, int, uint64_t, int, float*, int, int, hipStream_t);
template hipError_t launch_start_block<double>(int, int, int, uint64_t, int, double*, int, int, hipStream_t);

}  // namespace rdm
