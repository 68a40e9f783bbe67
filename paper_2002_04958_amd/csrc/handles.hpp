// Opaque handle types behind the C ABI.
#pragma once
#include <cstdint>
#include <map>
#include <memory>
#include <utility>
#include <vector>

#include "setup.hpp"
#include "solve.hpp"
#include "spmv.hpp"

struct amg_hierarchy {
  mgd::Ctx* ctx = nullptr;
  amg_params prm{};
  mgd::SetupHierarchy H;
  std::unique_ptr<mgd::Union<double>> u64;  // built on first use
  std::unique_ptr<mgd::Union<float>> u32;
  mgd::DBuf<float> in32, out32;
  int n = 0;
  double setup_ms = 0;

  mgd::Union<double>* union64();
  mgd::Union<float>* union32();
  // FP64 in/out apply regardless of the stored precision
  void apply(const double* r, double* z, int cycles);
};

namespace mgd {

// Glue descriptors for a group of independent scalar solves.
struct SegOut {
  int seg;              // destination segment of the result
  const double* coef;   // accumulate coef o x into s (or nullptr)
};

// A scalar matrix inverted by Jacobi iterations (option #1 of Section 3.4):
// its CSR arrays and its diagonal, FP64.
struct JacMember {
  const int* rp;
  const int* ci;
  const double* v;
  const double* d;
};

// `sweeps` Jacobi iterations from zero for `nm` members at once (member-major
// vectors of N); tmp holds nm * N values of T.
template <typename T>
void jacobi_run(Ctx* c, int N, const JacMember* tab, int nm, int sweeps, double nnz, const T* b,
                T* x, T* tmp);

// Option #3 for a set of scalar inverses (one batched step, or a single
// inverse): V-cycles z <- z + V(r), r = b - A z, each member until
// ||r|| < tol ||b|| or maxc cycles (member-major vectors of N).
template <typename T>
struct TolSolve {
  std::vector<int> roles;   // inverse role of each member
  DBuf<JacMember> mats;     // each member's level-0 matrix (FP64, natural order)
  DBuf<T> r, t;             // residual and V-cycle output, members x N
  DBuf<int> active;         // members still iterating
  DBuf<double> part, sums;  // reduction partials (members x nb) and per-member sums
  int nb = 0;
  double nnz = 0;           // entries of all members' matrices
};

template <typename T>
struct Group {
  // one inverse set over several scalar matrices: members [0, n_amg) run
  // V-cycles (batched union or one hierarchy per member), the rest Jacobi
  std::unique_ptr<Union<T>> batched;
  std::vector<Union<T>*> seq;
  std::vector<int> roles;   // hierarchy index of each member, V-cycle members first
  int n_amg = 0;
  int cycles = 1;
  DBuf<T> in, out;          // members x N, member-major
  DBuf<SegIn> in_tab;
  DBuf<SegOut> out_tab;
  std::unique_ptr<TolSolve<T>> tol;  // option #3 for the V-cycle members, or null
  DBuf<JacMember> jac_tab;  // members [n_amg, roles.size())
  int jac_sweeps = 0;
  double jac_nnz = 0;       // entries of all Jacobi members
  DBuf<T> jac_tmp;
  void run(Ctx* c, int N);
};

template <typename T>
struct PcExec {
  Group<T> grp;                    // the batched step
  DBuf<T> a_in, a_out, b_in, b_out;  // single-hierarchy vectors
  DBuf<double> s, res;             // FP64 scratch
  std::vector<DBuf<JacMember>> jac_one;  // per role, for single Jacobi inverses
  DBuf<T> jac_tmp1;
  std::vector<std::unique_ptr<TolSolve<T>>> tol_one;  // per role, single option #3 inverses
  DBuf<T> o4_w, o4_s, o4_t, o4_u;  // option #4 iterate and work vectors
  DBuf<SegIn> seg_tab;             // {E, no coupling}, {I, no coupling}: single inputs
};

}  // namespace mgd

struct block_precond {
  mgd::Ctx* ctx = nullptr;
  block_params prm{};
  int G = 0, N = 0;
  // owned copy of the (possibly transposed) system
  std::vector<mgd::Csr<double>> blocks;
  mgd::DBuf<double> d_gE, d_Eg, d_EI, d_IE;
  mgd::BlockSysDev sys{};
  // scalar hierarchies by role: g < G groups, G: E, G+1: I, G+2: PCTL coarse; mono: 0
  std::vector<std::unique_ptr<amg_hierarchy>> hier;
  std::vector<int> cycles;  // per role
  // PCTL
  mgd::DBuf<double> p;      // (G+1) N: p_1..p_G, p_I
  std::vector<int> p_cycles;
  // adaptive strategy (Section 3.5): Definition 1 counts, neglected couplings
  std::vector<int> cnt_gE, cnt_Eg;
  int cnt_EI = 0, cnt_IE = 0;
  std::vector<uint8_t> weak_gE, weak_Eg;
  int weak_EI = 0, weak_IE = 0;
  bool from_E_weak = false;         // every row block's coupling to E neglected (D_gE, D_IE)
  bool into_E_weak = false;         // every coupling in E's row neglected (D_Eg, D_EI)
  bool groups_from_E_weak = false;  // every D_gE neglected
  bool into_E_weak_groups = false;  // every D_Eg neglected
  // option #1 per role (Definition 2 count, -1 where not evaluated)
  std::vector<int> wd_count;
  std::vector<uint8_t> jacobi;
  std::vector<mgd::DBuf<double>> jac_diag;
  // option #3 inner solves (inner_tol > 0): roles solved to the tolerance and
  // the V-cycles each used in the last apply (-1 for fixed-count roles)
  std::vector<uint8_t> tol_role;
  std::vector<int> inner_cycles;
  std::unique_ptr<mgd::PcExec<double>> x64;
  std::unique_ptr<mgd::PcExec<float>> x32;
  // graph cache keyed by (r, z)
  std::map<std::pair<const void*, void*>, hipGraphExec_t> graphs;
  // whole flexible-GMRES steps (apply, matvec, Gram-Schmidt) keyed by every
  // pointer and size their launches use
  std::map<std::vector<uintptr_t>, hipGraphExec_t> step_graphs;
  // GMRES steps with Schur2: the block matvec of z overlaps the last E solve
  hipStream_t ovl_stream = nullptr;
  hipEvent_t ovl_fork = nullptr, ovl_join = nullptr;
  const mgd::BlockSysDev* ovl_S = nullptr;  // set for one apply: split matvec of z into ovl_y
  double* ovl_y = nullptr;
  bool ovl_forked = false;
  // GMRES steps whose apply starts with w_E* = A_E^{-1} r_E: that solve for
  // the next basis vector runs at the end of a step, beside the rest of its
  // Gram-Schmidt update (fs_fork/fs_join order the update on ovl_stream).
  // first_stage: 0 whole apply, 1 only that solve, 2 the apply without it
  hipEvent_t fs_fork = nullptr, fs_join = nullptr;
  int first_stage = 0;
  hipStream_t aux = nullptr;  // graph stream when the context stream is the null stream
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  int inverses_last = 0, matvecs_last = 0;
  double setup_ms = 0;
  ~block_precond();
};
