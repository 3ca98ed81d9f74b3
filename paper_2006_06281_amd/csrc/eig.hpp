// Eigen-prep of Fast CPD (Section III, eq. 16 and eq. 19): interfaces.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include <condition_variable>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace fcpd {

struct EigLayout {
  size_t end = 0;
  int n = 0;        // working width of the randomized solver (columns)
  int Mdense = 0;   // dense Jacobi size (0 when not used)
  size_t omega = 0, Z = 0, Q = 0, G = 0, R = 0, V = 0, ritz = 0, misc = 0, phi = 0, chol = 0;
};

// Columns the randomized solver can carry (K + oversample <= this).
int eig_topk_max_cols();
// Eigenpairs FULL mode may hold for M model points.
int eig_full_capacity(int M);
EigLayout eig_layout(int M, int mode, int K, int oversample, size_t start);

// One matrix of a grouped Jacobi solve (device-visible descriptor).
struct JacMember {
  double* A;               // n x n symmetric, destroyed (diag -> eigenvalues)
  double* V;               // n x n eigenvectors (rows of rotations applied)
  const double* normtot;   // |A|_F^2
  double* prm[2];          // per-pair rotation parameters of two steps
  int* state;              // {rotated in this sweep, active}
  int n;
  int nblk;                // block Jacobi: column blocks (even), else 0
  double* q;               // block Jacobi: Q of every pair (nblk / 2 x 64 x 64)
  int* qflag;              // block Jacobi: pairs that rotated in the step
};

// Collects the Jacobi solves of eigen-preps that run in parallel host
// threads (one stream each) and runs each collection as grouped launches:
// a thread's solve waits until every thread still inside its eigen-prep has
// submitted one or left; the last to arrive runs the group for all.
class JacobiBatcher {
 public:
  struct Req {
    double* A;
    double* V;
    int n;
    double* vals;
    int* perm;
    int* state;
    double* scratch;  // norm partials [0..64), their sum [64], two rotation buffers
    double* qscratch = nullptr;  // the block variant's scratch, if the caller has one
    hipStream_t st;
    hipEvent_t ready = nullptr;
    int rc = 0;
    std::string msg;
    bool done = false;
  };
  JacobiBatcher(JacMember* dev_members, int* dev_flags, int cap)
      : dev_members_(dev_members), dev_flags_(dev_flags), cap_(cap) {}
  void begin(int threads);  // threads that will each call solve() or leave()
  void leave();             // the calling thread's eigen-prep is over
  int solve(Req* r);        // blocks until r is solved; 0 ok, 1 no convergence, 2 device error

 private:
  void run_locked();
  JacMember* dev_members_;
  int* dev_flags_;
  int cap_;
  int live_ = 0;
  std::vector<Req*> pending_;
  std::mutex mu_;
  std::condition_variable cv_;
};

struct EigRun {
  const void* X;       // P4<float> or P4<double> model points
  bool x_is_double;
  int M;
  double beta;
  int mode, K, oversample, power_iters;
  uint64_t seed;
  const double* omega; // nullable (TOPK)
  char* ws;
  const EigLayout* L;
  double* U64;         // out: M x Kcap (row-major, M x K used)
  double* lam;         // out: Kcap
  int Kcap;
  hipStream_t st;
  JacobiBatcher* jb = nullptr;  // nullable: group the Jacobi solves with other threads'
};
// 0 ok, 1 numerical failure, 2 device error, 3 unsupported.
int eig_prepare_run(const EigRun& r, int* K_out, std::string* msg);

template <typename T> void convert_u_launch(const double* U64, T* U, size_t n, hipStream_t st);

// G = (A^T B + B^T A) / 2 for M x n row-major FP64 A, B (fixed-order
// reduction over row chunks; partials: gram_partial_doubles(M, n) doubles).
size_t gram_partial_doubles(int M, int n);
void gram_sym_launch(const double* A, const double* B, int M, int n, double* G, double* partials,
                     hipStream_t st);

}  // namespace fcpd
