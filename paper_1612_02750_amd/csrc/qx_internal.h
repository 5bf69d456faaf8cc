// Internal definitions shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace qx {

// ------------------------------------------------------------------ complex

template <typename R>
struct alignas(2 * sizeof(R)) cplx {
  R re, im;
};

// ----------------------------------------------------------------- geometry

// Lattice geometry in the form the kernels use: extents, half volume and the
// checkerboard-index strides of the y, z and t neighbours.
struct Geo {
  int L0, L1, L2, L3;
  int hv;        // V / 2
  int Lh;        // L0 / 2
  int s1, s2, s3;  // Lh, Lh*L1, Lh*L1*L2
  int anti_t;    // antiperiodic time boundary
  int stream_links;  // load links non-temporally (set per launch by the host)
};

// Links bigger than this do not fit the Infinity Cache next to the vectors
// and are streamed past the caches when one wavefront group reads each link.
constexpr size_t kStreamLinkBytes = (size_t)256 << 20;

// ------------------------------------------------------------ solver state

// Phase of one source in the solver state machine.
enum Phase : int {
  PH_RUN = 0,    // inner iterations proceed
  PH_RU = 1,     // waiting for a reliable update (x_hi += x_lo, FP64 residual)
  PH_RU2 = 2,    // FP64 residual computed, not converged: finish the update
  PH_DONE = 3    // finished (status says how)
};

enum RuReason : int { RU_DROP = 0, RU_INIT = 1, RU_FINAL = 2 };

// Per-source solver state, resident in device memory.
struct SrcState {
  double m2;        // mass squared
  double rho;       // |r|^2 of the current recurrence
  double pAp;       // Re <p, A p>
  double alpha, beta;
  double rmax;      // max |r| since the last reliable update
  double bnorm2;    // |b|^2
  double stop2;     // (tol_stop * |b|)^2
  double delta;     // reliable-update trigger
  double relres;    // last FP64 true relative residual
  int phase;
  int reason;       // RuReason of a pending update
  int status;       // QX_* status
  int iters, updates, max_iter;
  int pend;         // p is still to be replaced by r + beta p (done by the next p pass)
  int have_rr;      // |r|^2 partials of the last x/r update await the beta step (fused engine)
  int xpend;        // x_lo still lacks alpha p of the last x/r step (launch-per-pass and
                    // persistent engines: the next p pass or reliable update adds it)
};

// One system of a solver launch: a lattice, its links in the inner precision
// and in FP64, and the bases of its vectors inside the workspace.
// Stencil launches give each system nblk blocks of 64 sites (blocks
// [blk0, blk0 + nblk)); vector (BLAS) launches give each of its sources
// vtiles blocks of 256 complex elements (blocks [vblk0, vblk0 + nsrc*vtiles)).
struct SysDesc {
  Geo g;
  int nsrc;    // sources of this system
  int src0;    // index of its first source in the SrcState array
  int blk0, nblk;
  int vblk0, vtiles;
  const void* links_lo;
  const void* links_hi;
  void* vlo;        // inner precision: x_lo, r, p, Ap (even), t (odd), p', r'; each [nsrc][3][hv]
  void* vhi;        // FP64: x_hi, r_hi, b (even), t_hi (odd); each [nsrc][3][hv]
  double* partials;    // per-block partial sums of the stencil passes: [nsrc][nblk]
  double* partials_v;  // per-tile partial sums of the vector passes: [nsrc][vtiles]
  double* partials_x;  // two-launch sequence: Re<r, Ap>, |Ap|^2, |r|^2 partials, [3][nsrc][nblk]
};

// Grid barrier of the persistent solver kernel (zeroed before first use).
struct GridSync {
  unsigned count;   // blocks arrived at the current barrier
  unsigned gen;     // barrier generation
  unsigned error;   // set when a barrier wait timed out
  unsigned pad[61];
};

constexpr int kTile = 64;     // sites per stencil block
constexpr int kVTile = 256;   // complex elements per vector block

constexpr int kMaxSys = 64;

}  // namespace qx
