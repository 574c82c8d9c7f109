// Host-side structures of the library (not part of the ABI).
#pragma once

#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "internal.h"

namespace rdm {

// A named range on the calling thread's roctx stack (shown by rocprofv3
// --marker-trace; a few nanoseconds when no tool is attached).
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

// Thread-local error message behind rdm_last_error().
void set_error(const std::string& msg);
const char* last_error();

#define RDM_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::rdm::set_error(std::string(#call) + ": " + hipGetErrorString(e_));             \
      return RDM_E_DEVICE;                                                             \
    }                                                                                  \
  } while (0)

// Compiled term tables of one operator (H_t or H_b) on nbits sites.
struct OpTables {
  int nbits = 0;
  std::vector<DiagTerm> diag;
  std::vector<uint32_t> uf;   // uniform-coefficient hops
  std::vector<double> uc;
  std::vector<uint32_t> pf, pm;  // parity-dependent hops
  std::vector<double> pcs, pcd;
  // grouped form used by the apply kernel (see GHop / HopGroup)
  std::vector<uint32_t> g_flo, g_m;
  std::vector<double> g_cs, g_cd;
  std::vector<HopGroup> groups;
  // hops of partner tiles used fewer than kFatGroup times: gathered directly
  std::vector<uint32_t> t_f, t_m;
  std::vector<double> t_cs, t_cd;
  int nt[3] = {0, 0, 0};
  // the same two forms for bit-set tiles (kWideBits sites and more): tile bits
  // wbits; wide when products with the operator use them
  bool wide = false;
  uint32_t wbits = 0;
  std::vector<uint32_t> w_flo, w_m;
  std::vector<double> w_cs, w_cd;
  std::vector<HopGroup> wgroups;
  std::vector<uint32_t> wt_f, wt_m;
  std::vector<double> wt_cs, wt_cd;
  int wnt[3] = {0, 0, 0};
  // transform apply (kXzMinBits..kXzMaxBits bits): D_X terms (XX couplings
  // and x-fields) and D_Y terms (YY couplings), coefficients already scaled
  // by 2^-nbits; xy when there are D_Y terms
  bool xz = false, xy = false;
  std::vector<DiagTerm> xterms, yterms;
};

// Device copy of an operator's tables in one precision.
struct OpDevice {
  bool ready = false;
  int device = -1;
  void* hops = nullptr;
  void* groups = nullptr;
  void* thin = nullptr;
  int nt[3] = {0, 0, 0};
  void* diag = nullptr;
  void* dterms = nullptr;
  int ngroups = 0;
  // bit-set tile tables (wide operators)
  bool wide = false;
  uint32_t wbits = 0;
  void* whops = nullptr;
  void* wgroups = nullptr;
  void* wthin = nullptr;
  int wngroups = 0;
  int wnt[3] = {0, 0, 0};
  bool xz = false, xy = false;
  void* dx = nullptr;      // D_X / 2^N (transform apply); strided-tile order above 20 bits
  void* dy = nullptr;      // D_Y / 2^N, same order (operators with YY couplings)
  void* xterms = nullptr;
  void* yterms = nullptr;
};

}  // namespace rdm

struct rdm_hamiltonian {
  int n_s = 0, n_b = 0, n = 0;
  int apply = RDM_APPLY_AUTO;    // apply kind requested at creation
  std::vector<rdm_coupling> couplings;
  std::vector<double> hx, hz;
  rdm::OpTables op[2];           // [0] H_t, [1] H_b
  mutable std::mutex mu;
  mutable rdm::OpDevice dev[2][2];  // [which][precision]
};

namespace rdm {

// Device tables of h for (which, precision), built on first use on the
// current device (synchronous).
rdm_status get_device_op(const rdm_hamiltonian* h, int which, int precision, hipStream_t st,
                         const OpDevice** out);
// The same tables if they are already resident on the current device,
// RDM_E_INVALID otherwise (never builds or allocates).
rdm_status find_device_op(const rdm_hamiltonian* h, int which, int precision, const OpDevice** out);

// Symmetric tridiagonal eigenproblem by implicit QR with Wilkinson shifts.
// Fills theta (n) and zrow = first row of the eigenvector matrix (n), and
// keeps the rotation sequence so that S w (S = eigenvectors) can be formed
// later by replaying it.
struct TridiagEig {
  int n = 0;
  std::vector<double> theta, zrow;
  std::vector<int32_t> rot_i;
  std::vector<double> rot_c, rot_s;
  bool ok = true;
  void solve(const double* alpha, const double* beta, int n);
  // y = S diag(g) S^T e_1 for g_i given.
  void apply_fn(const double* g, double* y) const;
  // apply_fn for nf weight vectors g (nf x n, row-major) -> y (nf x n)
  void apply_fn_multi(int nf, const double* g, double* y) const;
  // w <- S^T w for nf vectors stored interleaved (w[i * nf + f])
  void apply_st_multi(int nf, double* w) const;
  // y = S diag(g) S^T x for any x (n).
  void apply_fn_vec(const double* g, const double* x, double* y) const;
  // eigenvector i (column i of S), n entries
  void eigvec(int i, double* y) const;
};

// Eigensystem of a dense symmetric matrix through Householder reduction to
// tridiagonal form (A = P T P^T) and TridiagEig on T, kept in the form the
// leading b x b block of f(A) needs: Z = S^T P_b^T (n x b; P_b the first b
// rows of P, S the eigenvectors of T), so that quad() forms
// E_b^T f(A) E_b = Z^T diag(f(theta)) Z for f(x) = exp(-beta (x - e0)).
struct DenseSymEig {
  int n = 0, b = 0;
  std::vector<double> z;  // Z, row-major n x b
  TridiagEig te;
  bool ok = true;
  void solve(const double* a, int n, int b);  // a: row-major n x n, symmetric; 1 <= b <= n
  double min_eig() const;
  void quad(double beta, double e0, double* f) const;  // f: b x b row-major
};

// Eigendecomposition of a small symmetric matrix (cyclic Jacobi, n <= 16):
// a (row-major n x n) -> eigenvalues w (ascending) and eigenvectors v (columns).
void sym_eig_small(int n, const double* a, double* w, double* v);

}  // namespace rdm
