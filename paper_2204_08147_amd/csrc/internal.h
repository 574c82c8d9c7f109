// Internal declarations shared by the host driver and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/rdm.h"

namespace rdm {

constexpr int kBlock = 256;        // threads per workgroup (4 wave64)
constexpr int kMaxSlab = 4;        // most 16-byte panels one lane handles

// Per-column device state, index [ST_x * cpad + c] (FP64).
enum {
  ST_SCUR = 0,   // s_j: scale of the current stored vector, q_j = s_j u_j
  ST_SPREV,      // s_{j-1}
  ST_BPS,        // beta_{j-1} * s_{j-1}: weight of u_{j-1} in the recurrence
  ST_ACUR,       // alpha_j * s_j: weight of u_j when forming u_{j+1}
  ST_RUNMAX,     // running max of |alpha_i|, beta_i (breakdown scale)
  ST_FROZEN,     // 1 once the column hit breakdown (or is padding)
  ST_COUNT
};

enum { MODE_LANCZOS = 0, MODE_REGEN = 1, MODE_PLAIN = 2 };

// Partial-sum planes of the FP64 transform Lanczos step (Seg::xdots): plane p
// is rows [p * x_tiles, (p + 1) * x_tiles) of part, one row per tile.  The
// step's <u_j, r_j> = s_j (A + QX + QY) - (beta s)_{j-1} C is assembled from
//   XP_A:  sum d u^2, the diagonal part (contiguous pass; before it the
//          plane holds |u~_j|^2 / L for the norm)
//   XP_QX: <u~_j, W_hi D_X W_hi u~_j> as sum D_X z^2, z = W_hi u~_j (strided
//          pass of the X part)
//   XP_C:  <u~_j, u~_{j-1}> / L (strided pass, where u~_j is formed)
//   XP_QY: <u~_j, (W_lo T W_lo) Y / L> = <Y_in, W_hi D_Y W_hi Y_in> (strided
//          pass of the YY part)
// so that the contiguous pass needs neither R nor u~_{j-1} before its
// transforms (FP32 steps keep the fused form of the contiguous pass).
enum { XP_A = 0, XP_QX = 1, XP_C = 2, XP_QY = 3, XP_COUNT = 4 };
enum { START_SYSBATH = 0, START_BATH = 1, START_PRODUCT = 2 };

constexpr int kTileBits = 8;       // the apply stages 2^8 = kBlock-row partner tiles in LDS
constexpr int kXzTileBits = 12;    // transform apply: 4096-element tiles ...
constexpr int kXzRegs = 16;        // ... as kBlock lanes x 16 registers
constexpr int kXzMinBits = 16;     // operators on 16..28 bits can use the transform apply
constexpr int kXzMaxBits = 28;
// Geometry of the strided passes over the N - 12 high bits:
//   shallow (up to 20 bits): one pass, tiles of every high-bit value and runs
//     of at least 16 consecutive rows;
//   deep (21, 22 bits): one pass, runs of 8 or 4 rows (a third LDS exchange);
//   split (23 bits and more): the high bits in two groups A (bits 12 ..
//     12+a-1) and B (the rest), W_hi D W_hi = W_A (W_B D W_B) W_A as three
//     passes whose tiles keep runs of at least 16 rows.
constexpr int kXzShallowMaxBits = 20;
constexpr int kXzDeepMaxBits = 22;
enum { XG_SHALLOW = 0, XG_DEEP = 1, XG_SPLIT = 2 };
__host__ __device__ inline int xz_geom(int nbits) {
  return nbits <= kXzShallowMaxBits ? XG_SHALLOW : nbits <= kXzDeepMaxBits ? XG_DEEP : XG_SPLIT;
}
__host__ __device__ inline int xz_split_a(int nbits) { return (nbits - 12) / 2; }  // bits in group A
constexpr int kFatGroup = 3;       // partner tiles read by at least this many hops go through LDS
// Bit-set tiles (per-column Lanczos steps on hop-table operators of at least
// kWideBits sites): a tile is the 2^kWideBits rows that differ only in a
// chosen set B of row bits -- the four lowest always among them, so every 16
// lanes read 256 contiguous bytes -- and agree with the tile's base in all
// others.  A hop with flip bits f reads the partner tile base ^ (f & ~B); B is
// chosen per operator so that few distinct partner tiles remain.
constexpr int kWideBits = 12;
constexpr int kWideRows = 4;       // rows per lane
constexpr int kWideBlock = (1 << kWideBits) / kWideRows;  // lanes per workgroup
constexpr int kWideLowBits = 4;    // bits 0..3 are always in B
constexpr int kWideFat = 2;        // partner tiles read by at least two hops go through LDS

// One off-diagonal term of H as the apply sees it: row idx couples to the
// partner idx ^ f with coefficient c = (parity(idx & m) == 0) ? cs : cd.
// f is split into the bits above the 256-row tile (fhi, shared by the hop's
// group) and the bits inside it (flo).  An XX+YY pair has m = f, cs = jx - jy,
// cd = jx + jy; when cs == cd (or for a one-site x-field) m = 0.
template <typename T>
struct alignas(16) GHop {
  uint32_t flo;
  uint32_t m;
  T cs, cd;
};
// Hops sharing one partner tile (same fhi), stored contiguously in three kinds:
// n0 with m = 0, n1 whose tested bits are all >= 6 (the coefficient is uniform
// over a wave of 64 consecutive rows), n2 with a per-row coefficient.  In the
// tables of bit-set tiles fhi = f & ~B, flo is the partner's tile index
// offset (the bits of f & B compressed to B's positions), and the n1 hops
// test no bit of B (the coefficient is uniform over the tile).
struct HopGroup {
  uint32_t fhi;
  int32_t start;
  int32_t n0, n1, n2;
  int32_t tile_uniform;  // 1: only n1 hops, all tested bits >= 8, so every
                         // coefficient is uniform over a 256-row tile
  int32_t pad[2];
};
// Diagonal term: c * (1 - 2 * parity(idx & mask)).
struct DiagTerm {
  uint32_t mask;
  uint32_t pad;
  double c;
};

// One Lanczos problem inside a (possibly batched) launch.  Lives in device
// memory; all kernels read it with uniform loads.
struct Seg {
  const void* hops;    // GHop<T>[] of the LDS-staged groups
  const void* groups;  // HopGroup[ngroups]; group 0 has fhi = 0
  const void* thin;    // GHop<T>[] gathered directly (flo holds the full flip mask)
  const void* diag;
  int32_t ngroups;
  int32_t nt0, nt1, nt2;  // direct hops by kind (m = 0, wave-uniform, per-row)
  int32_t nbits;       // log2(dim)
  int32_t P;           // panels
  int32_t S;           // panels per lane in apply/norm
  int32_t rpl;         // rows per lane in apply/norm
  int32_t C;           // real columns
  int32_t cpad;        // P * panel width
  int32_t k;
  int32_t mode;        // MODE_*
  int32_t ring;        // 0: slot j is Q + (j-1)*blk; 1: slot j is Q + ((j-1)&1)*blk
  int32_t start_kind;  // START_*
  int32_t ns_log;      // log2 d_s for START_SYSBATH
  int32_t nb;          // bath bits (RNG index range)
  int32_t n_beta;      // psi blocks (MODE_REGEN)
  int32_t n_row_tiles; // partial-sum rows (= row tiles of kBlock rows)
  int32_t tile_base;   // first workgroup of this segment in a norm launch (hop-table segments)
  int32_t ap_base;     // first workgroup of this segment in a (256-row) apply launch
  int32_t ap_rows;     // partial-sum rows the apply writes (row tiles of its kind)
  int32_t nm_rows;     // partial-sum rows the norm step writes
  int32_t xz;          // 1: transform apply (D_Z + W D_X W [+ T W D_Y W T]), 0: hop tables
  int32_t x_tiles;     // transform apply: tiles of 2^kXzTileBits rows
  int32_t x_base;      // transform apply: first workgroup of this segment
  int32_t xy;          // transform apply with a YY part (D_Y, the block Y)
  int32_t xdots;       // FP64 transform Lanczos: <u_j, r_j> from the XP_* planes
  int32_t wide;        // 1: the apply takes bit-set tiles (hops / groups / thin and the
                       // counts above are then the bit-set tables)
  int32_t wp_base;     // first workgroup of this segment in a bit-set apply launch
  uint32_t wbits;      // the row bits B that vary inside a bit-set tile
  const void* dx;      // transform apply: D_X / 2^N in T (tile order above 20 bits)
  const void* dy;      // transform apply: D_Y / 2^N in T, same order (xy segments)
  void* Y;             // xy segments: one block of dim x cpad for the YY part
  uint64_t seed;
  uint64_t blk;        // elements per vector block = dim * cpad
  void* Q;
  void* R;
  void* psi;           // n_beta blocks (MODE_REGEN)
  const void* ytab;    // [n_beta][k][cpad] in T (MODE_REGEN)
  double* st;          // [ST_COUNT][cpad]
  double* h_alpha;     // [k][cpad]
  double* h_beta;      // [k][cpad]  entry j-1 holds beta_j (0 after breakdown)
  double* h_s;         // [k][cpad]  entry j-1 holds s_j
  double* part;        // [n_row_tiles][cpad]
  int32_t* stepc;      // [cpad] current step (1-based) per column
  int32_t* kc;         // [cpad] Krylov size after breakdown truncation
  double tau;
};

// Block Lanczos (Algorithm 1) on the d_s start columns of every bath vector:
// groups g = 0..G-1 of DS consecutive columns.  Per-group d_s x d_s matrices
// in mats[(BM_x * G + g) * DS * DS + a * DS + b] (row a, column b), FP64.
enum {
  BM_BPREV = 0,  // B_{j-1} (zero at j = 1 and after breakdown)
  BM_A,          // A_j
  BM_RINV,       // inverse Cholesky factor of the current QR pass
  BM_R1,         // Cholesky factor of the first QR pass
  BM_SCALE,      // [0]: running max |entry| of the A_i, B_i (breakdown scale), [1]: frozen
  BM_COUNT
};
enum { BLK_A = 0, BLK_G = 1, BLK_G2 = 2 };  // reduction phases
struct BSeg {
  void* Q;            // three ring slots of dim x cpad (panel layout): slot(j) = (j-1) % 3
  void* R;            // dim x cpad: H q_j, then Z
  double* part;       // [n_rt][G][DS*DS] per-row-tile partial sums
  double* mats;       // [BM_COUNT][G][DS*DS]
  double* a_hist;     // [k][G][DS*DS]  A_j
  double* b_hist;     // [k][G][DS*DS]  B_j (Q_{j+1} B_j = Z)
  int32_t* kc;        // [G] blocks before breakdown
  uint64_t blk;       // dim * cpad
  int32_t nbits, cpad, C, G, k;
  int32_t rpl;        // rows per lane: a row tile is kBlock * rpl rows
  int32_t n_rt, n_cb; // row tiles, column blocks of max(DS, panel width) columns
  double tau;
};

// Partial trace over the bath of the ground-space projector: for each bath
// index b the lane forms phi_i[m] = sum_j sum_c w[j][i][c] u_j[(m << nb) + b][c]
// for the R orthonormalised Ritz vectors phi_i and accumulates
// sum_i phi_i[m] phi_i[n] (FP64) into part[tile][DS*DS].
struct GPSeg {
  const void* Q;      // k stored Lanczos blocks of dim x cpad (panel layout)
  const void* w;      // [k][R][cpad] weights, in T
  double* part;       // [n_tiles][DS*DS]
  uint64_t blk;       // dim * cpad
  int32_t nbits, nb, cpad, k, R, rpl, n_tiles, pad;
};

// Work item of the apply / norm kernels, derived from blockIdx.x: segment s
// owns workgroups [tile_base, tile_base + n_row_tiles * P/S), slab-major.
struct Tile {
  int32_t seg;
  uint32_t row0;
  int32_t panel0;
  int32_t rtile;
};

// Segment of the Gram kernel.
struct GSeg {
  const void* Q;        // k slots (stored) or n_beta psi blocks
  const void* ytab;     // [n_beta][k][cpad]
  double* gpart;        // [n_row_tiles][n_beta][n_v][ds][ds]
  uint64_t blk;
  int32_t nbits, cpad, k, n_beta, n_v, ds_log, rpl, from_psi;
  int32_t n_row_tiles, pad;
};
struct GTile {
  int32_t seg;
  uint32_t row0;
  int32_t cblock;       // column block of width CB
  int32_t rtile;
};

// ---- kernel launchers (kernels.hip) ----
template <typename T>
hipError_t launch_diag(const DiagTerm* terms, int nt, T* diag, int nbits, hipStream_t st,
                       bool xz_tiled = false);
template <typename T>
hipError_t launch_norm(const Seg* segs, int nseg, int ntiles, int slab, hipStream_t st);
template <typename T>
hipError_t launch_apply(const Seg* segs, int nseg, int ntiles, int slab, hipStream_t st);
// the apply over the wide segments: ntiles = sum of 2^(nbits - kWideBits) * P
template <typename T>
hipError_t launch_apply_wide(const Seg* segs, int nseg, int ntiles, hipStream_t st);
// pass 0, 1 or 2 of the plain transform apply Y = H X (MODE_PLAIN segments
// with xz = 1); passes 3 (once: X^ = W_lo X / 64 in place), 4 and 5 the same
// product on blocks kept as X^, giving R = W_lo H X / 64; the strided pass
// (1, 4 or 7) on the segments of geometry geo only (split: as three
// launch_xz_split passes).  The YY part (xy segments, block Y as scratch): passes
// 6 (Y = W_lo T X), 7 (Y = W_hi D_Y W_hi Y), 8 (R += T W_lo Y) after 0-2, or
// 9 (Y = W_lo T W_lo X^ / 64), 7, 10 (R += W_lo T W_lo Y / 64) after 4-5
template <typename T>
hipError_t launch_xz_pass(int pass, const Seg* segs, int nseg, int ntiles, hipStream_t st, int geo = XG_SHALLOW);
// The strided passes of split segments (three launches for one strided pass
// of the other geometries): op 0: R = W_A R; 1: R = W_B D_X W_B R; 2: Y =
// W_A Y; 3: Y = W_B D_Y W_B Y; 4: R = L W_A X (X the block Q, L = 4096).
template <typename T>
hipError_t launch_xz_split(int op, const Seg* segs, int nseg, int ntiles, hipStream_t st);
// Lanczos step over the segments with xz = 1, basis kept in the low-bit
// Hadamard basis: pass 0 = start block (once per run), 1 = norm step + high
// transform (split segments: the norm step and W_A only), 2 = low transforms
// + recurrence.  Pass 1 runs on the MODE_REGEN segments if regen, else on the
// others, and on the segments of geometry geo only.  boff: first transform
// tile.
template <typename T>
hipError_t launch_xz_lanczos(int pass, bool regen, const Seg* segs, int nseg, int ntiles, int boff,
                             hipStream_t st, int geo = XG_SHALLOW);
// Recombination weights of a segment whose basis is kept as W_lo u: L^-1/2
constexpr double kXzBasisScale = 1.0 / (1 << (kXzTileBits / 2));
// Lanczos-step passes of the YY part (xy segments): 3 = Y <- W_lo T W_lo u~ / L
// (contiguous), 4 = Y <- W_hi D_Y W_hi Y (strided; deep variant as for pass 1),
// 5 = R <- R + W_lo T W_lo Y / L (contiguous), before pass 2
hipError_t launch_red_beta(const Seg* segs, int nseg, int cmax, hipStream_t st);
hipError_t launch_red_alpha(const Seg* segs, int nseg, int cmax, hipStream_t st);
hipError_t launch_init_state(const Seg* segs, int nseg, int cmax, int phase, hipStream_t st);
template <typename T>
hipError_t launch_gram(const GSeg* gs, const GTile* tiles, int ntiles, int ds, int nb_chunk,
                       int beta0, int k, hipStream_t st);
hipError_t launch_colsum(const double* part, int nrows, int width, double* out, hipStream_t st);
// block Lanczos: one launch of the update kernel for step j (phase BLK_A:
// Z = H q_j - q_{j-1} B^T and A partials; BLK_G: Z -= q_j A and Gram partials;
// BLK_G2: q_{j+1} = Z R^-1 and Gram partials; 3: q_{j+1} = q_{j+1} R^-1), and
// the per-group reduction + small-matrix step of a phase
template <typename T>
hipError_t launch_block_update(const BSeg* bs, int ds, int phase, int j, int n_rt, int n_cb, hipStream_t st);
hipError_t launch_block_reduce(const BSeg* bs, int ds, int G, int phase, int j, hipStream_t st);
template <typename T>
hipError_t launch_ground_ptrace(const GPSeg* gp, int ds, int n_tiles, hipStream_t st);
template <typename T>
hipError_t launch_start_block(int ns_log, int nb, int C, uint64_t seed, int kind, T* out,
                              int nbits, int cpad, hipStream_t st);

// Bath-site sign correlations of the random bath vectors: for bath vectors
// j < nv and bath bits p < nb, the integer sum over b of s_b s_(b xor 2^p)
// (s_b = +-1 the signs of v_j), as per-block partials
// part[(j * nblk + blk) * nb + p], nblk = bath_sx_blocks(nb).
int bath_sx_blocks(int nb);
hipError_t launch_bath_sx(uint64_t seed, int nb, int nv, long long* part, hipStream_t st);

}  // namespace rdm
