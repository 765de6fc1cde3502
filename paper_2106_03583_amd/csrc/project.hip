// Pressure projection around the Poisson solve: the fractional step of
// Eqs. (3)-(6) on the staggered grid (Sec. 2; velocities on cell faces),
//     rhs = D u* / (gamma dt),   L_h Phi = rhs,   u = u* - gamma dt G Phi,
// after which D u vanishes to the solver's tolerance (the check of Sec. 4.1).
// D is the finite-volume divergence (face flux differences over the cell
// width) and G the face gradient, so D G = L_h with the boundary rules of
// the solver: a Neumann face keeps its velocity (G Phi = 0), a Dirichlet face
// sees the mirrored ghost -Phi one cell width away, a joined or periodic face
// the partner's cell at half the two widths.  A face shared by two blocks is
// stored (and updated) in both.
//
// Face fields are packed block after block: u (nz, ny, nx + 1), v (nz, ny + 1,
// nx), w (nz, ny, nx) for periodic z (face k - 1/2, cyclic) else (nz + 1, ny, nx).
#include "internal.h"

namespace mbp {

namespace {

__device__ __forceinline__ int xcd_remap_pj(int g, int n) {
    int x = g & 7, l = g >> 3;
    int per = n >> 3, rem = n & 7;
    return x * per + min(x, rem) + l;
}

struct PjArgs {
    const DBlock* B;  // finest-level blocks
    const int4* tiles;
    int ntiles;
    const double* dp;
    const int* pt;    // per block {dcx, dcy, gx, gy, rows before, columns before}
    int nz, nzw;      // cells and z faces per column
    double dz;
    int zper, zlo, zhi;
};

__device__ __forceinline__ long long uoff(const PjArgs& a, const DBlock& b, int bi) {
    return (long long)a.nz * (b.off + a.pt[6 * bi + 4]);
}
__device__ __forceinline__ long long voff(const PjArgs& a, const DBlock& b, int bi) {
    return (long long)a.nz * (b.off + a.pt[6 * bi + 5]);
}
__device__ __forceinline__ long long woff(const PjArgs& a, const DBlock& b) { return (long long)a.nzw * b.off; }
__device__ __forceinline__ long long coff(const PjArgs& a, const DBlock& b) { return (long long)a.nz * b.off; }

}  // namespace

// out = scale * D(u, v, w) on every cell.
__global__ void __launch_bounds__(256)
k_divergence(PjArgs a, const double* __restrict__ u, const double* __restrict__ v, const double* __restrict__ w,
             double scale, double* __restrict__ out) {
    const int k = blockIdx.y;
    const int4 t = a.tiles[xcd_remap_pj(blockIdx.x, a.ntiles)];
    const int bi = t.x;
    const DBlock b = a.B[bi];
    const int i = t.y + threadIdx.x;
    if (i >= b.nx) return;
    const double* dcx = a.dp + a.pt[6 * bi + 0];
    const double* dcy = a.dp + a.pt[6 * bi + 1];
    const double* ub = u + uoff(a, b, bi);
    const double* vb = v + voff(a, b, bi);
    const double* wb = w + woff(a, b);
    const int k1 = a.zper ? (k + 1) % a.nz : k + 1;
    const double idz = 1.0 / a.dz;
    for (int r = threadIdx.y; r < kTileY; r += kRowsPerPass) {
        const int j = t.z + r;
        if (j >= b.ny) break;
        const long long ui = ((long long)k * b.ny + j) * (b.nx + 1) + i;
        const long long vi = ((long long)k * (b.ny + 1) + j) * b.nx + i;
        const long long wi = ((long long)k * b.ny + j) * b.nx + i;
        const long long wi1 = ((long long)k1 * b.ny + j) * b.nx + i;
        const double d = (ub[ui + 1] - ub[ui]) / dcx[i] + (vb[vi + b.nx] - vb[vi]) / dcy[j] + (wb[wi1] - wb[wi]) * idz;
        out[coff(a, b) + ((long long)k * b.ny + j) * b.nx + i] = scale * d;
    }
}

namespace {

// Phi at (k, jj, ii) of block b, where (ii, jj) may be one cell outside along
// one axis: the partner's cell across a joined face, the mirrored ghost -Phi
// across a Dirichlet wall (a Neumann wall's face coefficient is zero).
__device__ __forceinline__ double phi_at(const PjArgs& a, const double* __restrict__ phi, const DBlock& b, int k,
                                         int ii, int jj) {
    int f = -1;
    if (ii < 0) f = XM;
    else if (ii >= b.nx) f = XP;
    else if (jj < 0) f = YM;
    else if (jj >= b.ny) f = YP;
    if (f < 0) return phi[coff(a, b) + ((long long)k * b.ny + jj) * b.nx + ii];
    const int nb = b.nbr[f];
    if (nb >= 0) {
        const DBlock& n = a.B[nb];
        const int ni = f == XM ? n.nx - 1 : f == XP ? 0 : ii;
        const int nj = f == YM ? n.ny - 1 : f == YP ? 0 : jj;
        return phi[coff(a, n) + ((long long)k * n.ny + nj) * n.nx + ni];
    }
    const int ci = min(max(ii, 0), b.nx - 1), cj = min(max(jj, 0), b.ny - 1);
    return -phi[coff(a, b) + ((long long)k * b.ny + cj) * b.nx + ci];
}

}  // namespace

// u -= gdt G Phi on every face of the block: each cell updates its lower x,
// y and z faces, the last cell of a row / column / z column also the upper
// one.  Faces with a zero coefficient (Neumann walls) are left untouched.
__global__ void __launch_bounds__(256)
k_gradient_update(PjArgs a, const double* __restrict__ phi, double gdt, double* __restrict__ u,
                  double* __restrict__ v, double* __restrict__ w) {
    const int k = blockIdx.y;
    const int4 t = a.tiles[xcd_remap_pj(blockIdx.x, a.ntiles)];
    const int bi = t.x;
    const DBlock b = a.B[bi];
    const int i = t.y + threadIdx.x;
    if (i >= b.nx) return;
    const double* gx = a.dp + a.pt[6 * bi + 2];
    const double* gy = a.dp + a.pt[6 * bi + 3];
    double* ub = u + uoff(a, b, bi);
    double* vb = v + voff(a, b, bi);
    double* wb = w + woff(a, b);
    const double idz = 1.0 / a.dz;
    for (int r = threadIdx.y; r < kTileY; r += kRowsPerPass) {
        const int j = t.z + r;
        if (j >= b.ny) break;
        const double pc = phi[coff(a, b) + ((long long)k * b.ny + j) * b.nx + i];
        const long long urow = ((long long)k * b.ny + j) * (b.nx + 1);
        // x faces i - 1/2 (and nx - 1/2 + 1 for the last column)
        if (gx[i] != 0.0) ub[urow + i] -= gdt * gx[i] * (pc - phi_at(a, phi, b, k, i - 1, j));
        if (i == b.nx - 1 && gx[b.nx] != 0.0)
            ub[urow + b.nx] -= gdt * gx[b.nx] * (phi_at(a, phi, b, k, b.nx, j) - pc);
        // y faces
        const long long vcol = (long long)k * (b.ny + 1) * b.nx + i;
        if (gy[j] != 0.0) vb[vcol + (long long)j * b.nx] -= gdt * gy[j] * (pc - phi_at(a, phi, b, k, i, j - 1));
        if (j == b.ny - 1 && gy[b.ny] != 0.0)
            vb[vcol + (long long)b.ny * b.nx] -= gdt * gy[b.ny] * (phi_at(a, phi, b, k, i, b.ny) - pc);
        // z faces (uniform spacing)
        const long long plane = (long long)b.ny * b.nx, cell = (long long)j * b.nx + i;
        if (a.zper) {
            const int km = (k + a.nz - 1) % a.nz;
            const double pm = phi[coff(a, b) + km * plane + cell];
            wb[k * plane + cell] -= gdt * idz * (pc - pm);
        } else {
            if (k > 0) {
                const double pm = phi[coff(a, b) + (k - 1) * plane + cell];
                wb[k * plane + cell] -= gdt * idz * (pc - pm);
            } else if (a.zlo == MBP_DIRICHLET) {
                wb[cell] -= gdt * idz * (pc + pc);
            }
            if (k == a.nz - 1 && a.zhi == MBP_DIRICHLET) wb[(long long)a.nz * plane + cell] -= gdt * idz * (-pc - pc);
        }
    }
}

namespace {
PjArgs pj_args(const mbp_plan* P) {
    const Level& L = P->levels[0];
    const bool per = P->g.zkind == Z_PP;
    return PjArgs{P->d_blk + L.blk_off, P->d_tiles + L.tile_off, L.ntiles, P->d_dbl, P->d_int + P->proj_tab,
                  P->g.nz, per ? P->g.nz : P->g.nz + 1, P->g.dz, per ? 1 : 0, P->g.zlo, P->g.zhi};
}
}  // namespace

void velocity_offsets(const mbp_plan* P, int64_t* uo, int64_t* vo, int64_t* wo) {
    const int nz = P->g.nz, nzw = P->g.zkind == Z_PP ? nz : nz + 1;
    int64_t a = 0, c = 0, e = 0;
    for (int b = 0; b <= P->g.nb; ++b) {
        if (uo) uo[b] = a;
        if (vo) vo[b] = c;
        if (wo) wo[b] = e;
        if (b == P->g.nb) break;
        const int64_t nx = P->g.nx[b], ny = P->g.ny[b];
        a += int64_t(nz) * ny * (nx + 1);
        c += int64_t(nz) * (ny + 1) * nx;
        e += int64_t(nzw) * ny * nx;
    }
}

void launch_divergence(const mbp_plan* P, const double* u, const double* v, const double* w, double scale,
                       double* out, hipStream_t s) {
    const Level& L = P->levels[0];
    hipLaunchKernelGGL(k_divergence, dim3(L.ntiles, P->g.nz), dim3(kTileX, kRowsPerPass), 0, s, pj_args(P), u, v, w,
                       scale, out);
}

void launch_gradient_update(const mbp_plan* P, const double* phi, double gdt, double* u, double* v, double* w,
                            hipStream_t s) {
    const Level& L = P->levels[0];
    hipLaunchKernelGGL(k_gradient_update, dim3(L.ntiles, P->g.nz), dim3(kTileX, kRowsPerPass), 0, s, pj_args(P), phi,
                       gdt, u, v, w);
}

}  // namespace mbp
