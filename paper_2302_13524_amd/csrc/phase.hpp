// Phase-offset correction from defocus images (Sec. 2.3), FP64 device code.
#pragma once
#include <stdint.h>

namespace tmk {

struct PhaseDims {
  int P, N, Nd, nf1, nf2;
};

struct PhaseOptics {
  double lambda, ps, NA, z;
};

// Pupil band: h vanishes outside the pupil, so only the spectrum bins with
// signed frequencies s1 in [s1lo, s1lo + B1), s2 in [s2lo, s2lo + B2) carry
// the field through the model. When the box is small (B1, B2 <= 16) the
// evaluation uses pruned transforms over the box instead of full line FFTs.
struct PhaseBand {
  int on;                  // 1: band evaluation, 0: full separable FFTs
  int s1lo, B1, s2lo, B2;  // the box
  int RA, CH;              // field rows per workgroup of the spectrum pass, their blocks (CH RA = nf1)
  int G, CPW, NXB;         // image pass: threads per column, columns per workgroup, column blocks
};

// Device workspace for one problem (all device pointers).
struct PhaseWork {
  double* c;      // [Nd][P] complex (2 doubles)  c_n = TM_est e^{j theta_n}
  double* h;      // [nf1][nf2] complex kernel
  double* A;      // [Nd][nf1][nf2] complex field-grid scratch
  double* B;      // [Nd][2nf1][2nf2] complex image-grid scratch
  double* gpart;  // [Nd] per-image objective
  double* w;      // [slices][P] complex partial sums of the gradient gather
  double* gval;   // [1] objective
  int32_t* inv;   // [nf1 nf2] row index of each field pixel, -1 outside the rows
  int* skip;      // [1] set to 1 when the L-BFGS solve has ended: evaluation kernels return at once
  int* chk;       // [3] pixel check: problem bits (1 outside the grid, 2 repeated), smallest row of each
  double* Sp;     // band: [Nd][CH][16][16] complex, box spectrum partials per block of field rows
  double* V;      // band: [Nd][column blocks][16][16] complex, adjoint box spectrum partials
  double* Wn;     // band: [Nd][P] complex, conj(c_n) (A_n^H a_n r_n) at the pixels
  double* dpart;  // [4 ceil(P / 256)] dvec^T grad over pixels 64 i .. 64 i + 63 (phase_eval with dvec)
  PhaseBand band; // host-side plan
};

size_t phase_work_bytes(const PhaseDims& d);
// Band plan for these optics (host computation of the pupil's support);
// enable = 0 forces the full separable path.
PhaseBand phase_band_plan(const PhaseDims& d, const PhaseOptics& o, int enable);
void phase_work_carve(void* base, const PhaseDims& d, PhaseWork* w);

// c[n][p] = sum_k theta[n][k] tm_est[p][k] (c_n = TM_est e^{j theta_n}): FP32
// inputs, FP64 products and sums, K split into phase_cgemm_slices(d) chunks
// whose partials (part: slices x Nd x P complex) are added in a fixed order.
int phase_cgemm_slices(const PhaseDims& d);
int phase_cgemm(const PhaseDims& d, const void* theta, const void* tm, double* part, double* c, void* stream);

// The kernel table h, the pixel map and the solve flag (c is formed by the
// caller). Returns hipError_t.
int phase_setup(const PhaseDims& d, const PhaseOptics& o, const void* tm_est, const void* theta,
                const int32_t* pix, PhaseWork& w, void* stream);
// g(phi) into w.gval[0] and dg/dphi into grad[P]; with dvec (else null) also
// the partial sums of dvec^T grad over each 64 pixels into w.dpart.
int phase_eval(const PhaseDims& d, const int32_t* pix, const float* Id, const double* phi,
               double* grad, PhaseWork& w, const double* tw64, void* stream, const double* dvec = nullptr);

// |A_n e^{j phi}|^2 into I_out [Nd][2nf1][2nf2] (float).
int phase_images(const PhaseDims& d, const int32_t* pix, const double* phi, float* I_out, PhaseWork& w,
                 const double* tw64, void* stream);

// L-BFGS helpers over phi (single-workgroup kernels).
struct PhaseLb {
  double* phi;    // [P]
  double* g;      // [P] gradient at phi
  double* gt;     // [P] gradient at trial
  double* gb;     // [P] gradient at the best trial kept while the step grows
  double* phit;   // [P] trial point
  double* d;      // [P]
  double* S;      // [m][P]
  double* Y;      // [m][P]
  double* sc;     // [phase_lb_state_doubles(m)] iteration state (see phase_kernels.hip)
  const double* dpart;  // [(P + 63) / 64] partials of d^T gt from the evaluation at the trial
};
int phase_lb_state_doubles(int m);
// Device-controlled iterations (see phase_kernels.hip): init after the first
// evaluation, then per iteration phase_lb_iter (decide on the pending trial,
// new direction or halved step, trial point) and the evaluation at phit.
int phase_lb_init(PhaseLb& L, int P, int m, int iters, const double* gval, int* skip, const int* chk,
                  void* stream);
int phase_lb_iter(PhaseLb& L, int P, int m, int iters, double ftol, const double* gval, int* skip, void* stream);
// phi (unless the pixel check failed) to phi_out, and rec[0..6] = f, accepted
// iterations, evaluations, solve ended, pixel check bits, first rows (device).
int phase_lb_finish(const PhaseLb& L, const PhaseWork& w, int P, double* phi_out, double* rec, void* stream);

}  // namespace tmk
