// 3D multigrid without the z synthesis (the comparison solver): plan layout
// shared by the host driver (mg3d.cpp) and the kernels (mg3d.hip).
#pragma once

#include <vector>

#include "internal.h"

namespace mbp {

struct Mg3Level {
    int xl = 0;           // x-y level of the FFT path's hierarchy
    int xyc = 0;          // the next coarser 3D level coarsens x-y (else x-y is kept)
    int zc = 0;           // the next coarser 3D level halves z (else z is kept)
    int even_xy = 0;      // every block has even x and y counts (x-y children in pairs)
    int xy22 = 1;         // an x-y coarsening step from here halves both x and y (not semicoarsened)
    int blk_off = 0;      // first DBlock of the x-y level in the block table
    int tile_off = 0;     // first x-y tile of the level
    int ntiles = 0;
    int nz = 0;           // cells along z on this level
    double idz2 = 0.0;    // 1 / dz_l^2
    long long plane = 0;  // x-y cells
    long long ncell = 0;  // nz * plane
    double* f = nullptr;  // rhs (levels >= 1)
    double* p = nullptr;  // iterate (levels >= 1)
    double* q = nullptr;  // second buffer of the out-of-place sweeps
};

struct Mg3Plan {
    int nlev = 0;
    std::vector<Mg3Level> lev;
    int zlo = 0, zhi = 0;  // MBP_* conditions at the two z ends
    double alpha = 0.0;    // Helmholtz term
    double omega = 6.0 / 7.0;  // Jacobi weight (optimal smoothing of the 3D 7-point stencil)
    int nc = 0;            // coarsest x-y cells
    // device tables (one allocation)
    DBlock* d_blk = nullptr;
    int* d_int = nullptr;
    double* d_dbl = nullptr;
    int4* d_tiles = nullptr;
    double* d_cwl = nullptr;
    double* d_cwr = nullptr;
    double* d_cmu = nullptr;
    int2* d_cmap = nullptr;   // coarsest plane cell -> {packed offset at z = 0, z stride}
    double* d_vz = nullptr;   // coarsest z eigenvectors, nzc x nzc (column m = mode m)
    double* d_muz = nullptr;  // their eigenvalues
    double* d_xhat = nullptr; // nzc x nc scratch of the coarsest solve
    double* d_area0 = nullptr;
    double mu_min = 0.0;      // smallest non-null |eigenvalue| of the coarsest operator (error test)
    double* d_part = nullptr; // per-workgroup partial sums, two arrays of (finest tiles x nz)
    double* d_scal = nullptr; // [0..1] cycle residual^2 and |p|^2; [2] rhs mean; [3..4] a residual
                              // evaluation (residual^2, |p|^2); [5] p mean
    double* q0 = nullptr;     // second finest buffer
};

// One sweep; returns the number of workgroups (the count of partial sums
// written to part[0, n) and part[n, 2n) when part is given).
long long m3_jacobi(const Mg3Plan& M, int l, const double* pin, double* pout, const double* f, double fshift,
                    bool zero, double* part, hipStream_t s);
void m3_residual_norm(const Mg3Plan& M, const double* p, const double* f, double fshift, bool zero, double* part,
                      double* out, hipStream_t s);
void m3_total(const double* part, long long n, double scale, double* out, hipStream_t s);
void m3_restrict(const Mg3Plan& M, int l, const double* p, const double* f, double fshift, double* fc,
                 hipStream_t s);
void m3_prolong(const Mg3Plan& M, int l, const double* pc, double* pf, hipStream_t s);
void m3_coarse(const Mg3Plan& M, const double* f, double* p, hipStream_t s);
void m3_area_sum(const Mg3Plan& M, const double* x, double* part, double* out, double scale, hipStream_t s);
void m3_sub(double* x, long long n, const double* mean, hipStream_t s);
void m3_copy(const double* a, double* b, long long n, hipStream_t s);

}  // namespace mbp
