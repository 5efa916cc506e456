// Device evaluation of the analytic e, f, psi families used as synthetic
// workloads, the compact right-hand side operator F = (prod_l H_{alpha_l}) f
// (eq. eq2.2, Appendix A), and small utility kernels.
#pragma once
#include "common.h"

#define RSFDE_MAXMODES 8
#define RSFDE_MC_STRIDE 32  // per-axis manufactured-source coefficients

struct FieldDev {
  int kind;
  int K;                     // sine modes per axis
  int a;                     // manufactured exponent
  int pad;
  double c[4];
  double norm;               // sum |amp| (SINE_FIELD)
  const double* amp;         // K^d amplitudes, k_1 fastest
  const double* sintab[3];   // sin((k+1) pi x_{i,j}) at [k*(N_i+2) + j], closure index j
  const double* mc;          // manufactured: per axis [left(13), right(13), sigma] at axis*32
  const double* ax[3];       // per-axis factor tables (AX_* rows of N_i+2 entries, closure index)
};

// Rows of the per-axis tables: every factor of the separable fields that depends
// on one coordinate only, evaluated once per closure point of the axis with the
// same expression the point-wise evaluation would use.
enum : int { AX_E = 0, AX_U = 1, AX_RIESZ = 2, AX_PSI = 3, AX_ROWS = 4 };

struct GridDev {
  int d;
  int closure;               // 1: closure grid (N_i+2 points), 0: interior
  int N[3];                  // interior sizes
  double lo[3], h[3];
  double kappa[3];
  double inv[3];             // 1 / (points per axis of this grid), for index splitting
  int64_t size;
};

// (quotient, remainder) of r by n for r < 2^32, from the reciprocal inv = 1/n and
// one correction step (no integer division).
__device__ __forceinline__ unsigned split_u32(unsigned r, unsigned n, double inv, unsigned* rem) {
  unsigned q = (unsigned)((double)r * inv);
  if ((unsigned long long)q * n > r) --q;
  else if ((unsigned long long)(q + 1) * n <= r) ++q;
  *rem = r - q * n;
  return q;
}

// Time factors of the field families, evaluated once per launch on the host.
struct TimeF {
  double cos_t, exp_mt;
};

// one instance's field evaluation and its source operator, for batched launches
struct FieldJob {
  FieldDev e, f;
  GridDev g;
  int which, pad;
  double* out;
};
struct FJob {
  const double* fcl;
  GridDev g;
  double al[3];
  double* F;
};

hipError_t fields_eval(const FieldDev& e, const FieldDev& f, int which, const GridDev& g, double t,
                       double* out, hipStream_t s);
// jobs and start in device memory; block b of the launch works on the job whose
// block range start[s] .. start[s+1) holds b (blocks of 256 threads)
hipError_t fields_eval_batched(const FieldJob* jobs, const int* start, int n, int64_t nblocks,
                               double t, hipStream_t s);
hipError_t compute_F_batched(const FJob* jobs, const int* start, int n, int64_t nblocks,
                             hipStream_t s);
hipError_t fields_sintab(int K, int Ncl, double lo, double h, double* tab, hipStream_t s);
// per-axis tables for axis `axis` of the closure grid g (E, F, psi as registered)
hipError_t fields_axis_tables(const FieldDev& e, const FieldDev& f, const FieldDev& psi,
                              const GridDev& g, int axis, double* tab, hipStream_t s);
hipError_t compute_F(const double* fcl, const GridDev& interior, const double* alpha, double* F,
                     hipStream_t s);
hipError_t minmax_reset(double* mm, hipStream_t s);
hipError_t minmax_accum(const double* e, int64_t n, double* mm, double* partial, unsigned* counter,
                        hipStream_t s);
hipError_t convert_f64_f32(const double* in, float* out, int64_t n, hipStream_t s);
hipError_t fill_f64(double* x, int64_t n, double v, hipStream_t s);
