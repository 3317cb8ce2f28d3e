// Shared declarations of the host side of the H.psi library.
#pragma once
#include <cstdint>
#include <string>
#include <vector>
#include <array>
#include <map>
#include <unordered_map>
#include "../../include/dmrg.h"

namespace dmrg {

void set_error(const std::string &msg);

// device memory through the plan's allocator (caller's callbacks or hipMalloc)
void *plan_dalloc(dmrg_plan_t *p, size_t bytes);
void plan_dfree(dmrg_plan_t *p, void *ptr);

struct Error {
  int code;
  std::string msg;
};

// ------------------------------------------------------------ Wigner (wigner.cpp)
double cg(int j1, int m1, int j2, int m2, int J, int M);   // doubled arguments
double w6j(int a, int b, int c, int d, int e, int f);
double w9j(int j1, int j2, int j, int k1, int k2, int k, int j1p, int j2p, int jp);
double ctilde(int j1, int j2, int j, int k1, int k2, int k, int j1p, int j2p, int jp);

// memoised C~ (Eq. 4); the three roles mirror the paper's W9j(l), W9j(r), W9j(h)
struct CtildeTable {
  std::unordered_map<uint64_t, double> cache;
  double get(int j1, int j2, int j, int k1, int k2, int k, int j1p, int j2p, int jp);
};

// ------------------------------------------------------------ families
enum Fam { F_H = 0, F_C, F_A0, F_A1, F_B0, F_B1, F_S, F_P0, F_P1, F_Q0, F_Q1, N_FAM };
extern const int FAM_TWO_K[N_FAM];
extern const int FAM_DN[N_FAM];
extern const int FAM_PAR[N_FAM];

struct BlockModel {
  int role = 0;            // 0 left, 1 right
  int n_orb = 0, p = 0, lo = 0, hi = 0;
  std::vector<dmrg_sector_t> sec;
  std::vector<int64_t> sec_off;          // unused by blocks, kept for symmetry
  std::vector<dmrg_oprec_t> rec;
  const double *data = nullptr;
  int64_t data_len = 0;
  std::vector<std::vector<std::array<int, 2>>> labels;   // per family
  std::vector<std::map<std::array<int, 2>, int>> label_pos;
  std::unordered_map<int64_t, int> rec_index;           // (fam,row,col) -> record
  int n_orbitals() const { return hi - lo; }
  int find_rec(int fam, int row, int col) const {
    auto it = rec_index.find(((int64_t)fam * 1000003 + row) * 1000003 + col);
    return it == rec_index.end() ? -1 : it->second;
  }
  int pos(int fam, int x, int y = -1) const {
    auto it = label_pos[fam].find({x, y});
    return it == label_pos[fam].end() ? -1 : it->second;
  }
};

int build_block(BlockModel &b, int role, const dmrg_problem_t &pr, Error &err);

// ------------------------------------------------------------ site algebra
struct SiteFamily {
  std::vector<int> adj;    // elementary tensors: 0 = a+, 1 = a~
  std::vector<int> inter;  // intermediate doubled ranks (left-to-right coupling)
  int k2 = 0, parity = 0;
  double red[3][3];        // <b||T||a>, multiplets 0 empty, 1 single, 2 double
};

struct SiteAlgebra {
  std::vector<SiteFamily> fams;
  std::map<std::pair<std::vector<int>, std::vector<int>>, int> index;
  int get(const std::vector<int> &adj, const std::vector<int> &inter);
};

// ------------------------------------------------------------ operator table
// Operator on one partition: identity, block family (adjoint or not), or a
// site family.
struct PT {
  int kind = 0;   // 0 identity, 1 block family, 2 site family
  int id = 0;     // family id (kind 1) or site-family index (kind 2)
  int adj = 0;
  int k2 = 0;
  int par = 0;
  bool operator<(const PT &o) const {
    return std::tie(kind, id, adj, k2) < std::tie(o.kind, o.id, o.adj, o.k2);
  }
  bool operator==(const PT &o) const {
    return kind == o.kind && id == o.id && adj == o.adj && k2 == o.k2;
  }
};

struct RowKey {
  PT t[4];
  int K2 = 0;
  bool operator<(const RowKey &o) const {
    for (int i = 0; i < 4; i++) {
      if (t[i] < o.t[i]) return true;
      if (o.t[i] < t[i]) return false;
    }
    return K2 < o.K2;
  }
};

struct PosAlpha { int pA, pD; double alpha; };

struct Row {
  RowKey key;
  std::vector<PosAlpha> pos;   // sorted by (pA, pD)
};

int build_rows(const dmrg_problem_t &pr, const BlockModel &L, const BlockModel &R,
               SiteAlgebra &site, std::vector<Row> &rows, Error &err);

// ------------------------------------------------------------ wavefunction blocks
struct PsiBlock {
  int iL, l, SLl, r, iR, SrR;
  int dL, dR;
  int64_t off;
};

void psi_blocks(const BlockModel &L, const BlockModel &R, int n_elec, int two_s,
                std::vector<PsiBlock> &out, int64_t &size);

// ------------------------------------------------------------ sector tasks
// One sector task (Eq. 3 row) with its position list: Y_F += v * alpha_p *
// op(A[recA, pA]) X_E op(D[recD, pD])^T, op = transpose for adjoint families.
struct Task {
  int row;
  int E, F;            // wavefunction block indices (input, output)
  int recA, recD;      // records, -1 for identity
  int adjA, adjD;
  double v;            // sector value incl. site elements, C~ factors, signs
  int dress = -1;      // >= 0: D comes from dressed record `dress` (positions j)
};

// A dressed right-block record: for operator-table rows with two position
// indices (one per block) the sum over the right-block index is done once,
//   Dt[j] = sum_t alpha_t D[rec][pD_t]  for the t belonging to left position j,
// turning sum_{i,k} alpha_ik A_i X D_k^T into sum_i A_i X Dt_i^T.
struct Dress {
  int rec = 0;                 // source record of the right block
  int rows = 0, cols = 0;      // block shape (same as the source record)
  int npos = 0;                // dressed positions (distinct left positions)
  std::vector<int> start;      // [npos+1] ranges into src_pos / src_alpha
  std::vector<int> src_pos;
  std::vector<double> src_alpha;
  int64_t off = 0;             // offset in the dressed-data array
};

struct Tasks {
  std::vector<PsiBlock> blocks;
  int64_t size = 0;
  std::vector<Row> rows;
  std::vector<Task> tasks;
  SiteAlgebra site;
  double flops = 0.0;
  std::vector<Dress> dress;
  int64_t dress_len = 0;       // elements of the dressed-data array
};

// host evaluation of the dressed records (test paths); out has dress_len entries
void dress_on_host(const Tasks &T, const BlockModel &R, std::vector<double> &out);

int build_tasks_for_problem(const dmrg_problem_t &pr, BlockModel &L, BlockModel &R,
                            Tasks &T, Error &err);

}  // namespace dmrg
