// Host-side plan construction: validation, connectivity, multigrid levels,
// coefficient and transfer tables, colour parities, the coarsest-level
// eigen-decomposition and the z-transform tables.  No HIP call is made here,
// so mbp_plan_check works without a GPU.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.h"

namespace mbp {

void options_default(mbp_options* o) {
    o->precision = MBP_FP64;
    o->nu1 = 1;
    o->nu2 = 1;
    o->max_cycles = 100;
    o->flags = 0;
    o->etol = 0.0;
    o->inner = 4;
    o->march = 0;
    o->smoother = MBP_SMOOTHER_DEFAULT;
    o->helmholtz = 0.0;
}

// Hyperbolic-tangent face clustering (Sec. 3.1, Table 2 caption).  Two-sided:
// x(s) = (1 + tanh(a (s - 1/2)) / tanh(a/2)) / 2; lower-end clustering:
// x(s) = 1 + tanh(a (s - 1)) / tanh(a); upper-end: x(s) = tanh(a s) / tanh(a).
int grid_tanh(int n, double lmin, double lmax, int type, double factor, double* out) {
    if (n < 1 || !out || !(lmax > lmin) || !std::isfinite(lmin) || !std::isfinite(lmax) ||
        !(factor >= 0.0) || !std::isfinite(factor) || type < -1 || type > 1)
        return MBP_ERR_INVALID;
    for (int i = 0; i <= n; ++i) {
        double s = double(i) / n, x;
        if (factor == 0.0)
            x = s;
        else if (type == 0)
            x = 0.5 * (1.0 + std::tanh(factor * (s - 0.5)) / std::tanh(0.5 * factor));
        else if (type == -1)
            x = 1.0 + std::tanh(factor * (s - 1.0)) / std::tanh(factor);
        else
            x = std::tanh(factor * s) / std::tanh(factor);
        if (i == 0) x = 0.0;
        if (i == n) x = 1.0;
        out[i] = lmin + (lmax - lmin) * x;
    }
    return MBP_OK;
}

namespace {

bool fail(std::string* err, const std::string& msg) {
    if (err) *err = msg;
    return false;
}

bool increasing(const double* f, int n1) {
    if (!f) return false;
    for (int i = 0; i < n1; ++i)
        if (!std::isfinite(f[i])) return false;
    for (int i = 1; i < n1; ++i)
        if (!(f[i] > f[i - 1])) return false;
    return true;
}

bool validate(const mbp_block_desc* blocks, int nb, const mbp_synth_desc* z, Geometry& g,
              std::string* err) {
    if (!blocks || nb < 1 || nb > 4096) return fail(err, "need 1..4096 blocks");
    if (!z) return fail(err, "missing z descriptor");
    if (z->nz < 2 || (z->nz & 1) || z->nz > 4096) return fail(err, "nz must be even, 2..4096");
    if (!(z->lz > 0.0) || !std::isfinite(z->lz)) return fail(err, "lz must be positive");
    int lo = z->bc_lo, hi = z->bc_hi;
    if (lo == MBP_PERIODIC && hi == MBP_PERIODIC)
        g.zkind = Z_PP;
    else if (lo == MBP_NEUMANN && hi == MBP_NEUMANN)
        g.zkind = Z_NN;
    else if (lo == MBP_DIRICHLET && hi == MBP_DIRICHLET)
        g.zkind = Z_DD;
    else if (lo == MBP_NEUMANN && hi == MBP_DIRICHLET)
        g.zkind = Z_ND;
    else if (lo == MBP_DIRICHLET && hi == MBP_NEUMANN)
        g.zkind = Z_DN;
    else
        return fail(err, "invalid z condition pair");
    g.nz = z->nz;
    g.lz = z->lz;
    g.dz = z->lz / z->nz;
    g.zlo = lo;
    g.zhi = hi;
    g.nb = nb;
    g.lo0.resize(nb); g.lo1.resize(nb); g.hi0.resize(nb); g.hi1.resize(nb);
    g.nx.resize(nb); g.ny.resize(nb); g.xf.resize(nb); g.yf.resize(nb);
    g.bc.resize(nb); g.nbr.resize(nb);
    for (int i = 0; i < nb; ++i) {
        const mbp_block_desc& b = blocks[i];
        if (b.hi[0] < b.lo[0] || b.hi[1] < b.lo[1]) return fail(err, "block with hi < lo");
        int64_t nx = int64_t(b.hi[0]) - b.lo[0] + 1, ny = int64_t(b.hi[1]) - b.lo[1] + 1;
        if (nx > (1 << 16) || ny > (1 << 16)) return fail(err, "block too large");
        g.lo0[i] = b.lo[0]; g.lo1[i] = b.lo[1]; g.hi0[i] = b.hi[0]; g.hi1[i] = b.hi[1];
        g.nx[i] = int(nx);
        g.ny[i] = int(ny);
        if (!increasing(b.xf, int(nx) + 1) || !increasing(b.yf, int(ny) + 1))
            return fail(err, "face coordinates must be finite and increasing");
        g.xf[i].assign(b.xf, b.xf + nx + 1);
        g.yf[i].assign(b.yf, b.yf + ny + 1);
        for (int f = 0; f < 4; ++f) {
            if (b.bc[f] < MBP_DIRICHLET || b.bc[f] > MBP_PERIODIC)
                return fail(err, "unknown face condition");
            g.bc[i][f] = b.bc[f];
            g.nbr[i][f] = -1;
        }
    }
    // overlapping blocks in index space
    for (int i = 0; i < nb; ++i)
        for (int k = i + 1; k < nb; ++k) {
            bool ox = g.lo0[i] <= g.hi0[k] && g.lo0[k] <= g.hi0[i];
            bool oy = g.lo1[i] <= g.hi1[k] && g.lo1[k] <= g.hi1[i];
            if (ox && oy) return fail(err, "blocks overlap in index space");
        }
    // connectivity: each joined face has exactly one partner over the same
    // tangential range (Sec. 3.1)
    for (int i = 0; i < nb; ++i)
        for (int f = 0; f < 4; ++f) {
            int kind = g.bc[i][f];
            if (kind != MBP_CONNECT && kind != MBP_PERIODIC) continue;
            int axis = f / 2;
            int tlo_i = axis == 0 ? g.lo1[i] : g.lo0[i];
            int thi_i = axis == 0 ? g.hi1[i] : g.hi0[i];
            int found = -1, count = 0;
            for (int k = 0; k < nb; ++k) {
                int tlo_k = axis == 0 ? g.lo1[k] : g.lo0[k];
                int thi_k = axis == 0 ? g.hi1[k] : g.hi0[k];
                if (tlo_k != tlo_i || thi_k != thi_i) continue;
                if (g.bc[k][f ^ 1] != kind) continue;
                if (kind == MBP_CONNECT) {
                    if (k == i) continue;
                    int alo_i = axis == 0 ? g.lo0[i] : g.lo1[i];
                    int ahi_i = axis == 0 ? g.hi0[i] : g.hi1[i];
                    int alo_k = axis == 0 ? g.lo0[k] : g.lo1[k];
                    int ahi_k = axis == 0 ? g.hi0[k] : g.hi1[k];
                    bool lower = (f & 1) == 0;
                    if (lower ? (ahi_k + 1 != alo_i) : (ahi_i + 1 != alo_k)) continue;
                }
                found = k;
                ++count;
            }
            if (count != 1)
                return fail(err, "block " + std::to_string(i) + " face " + std::to_string(f) +
                                     ": needs exactly one partner, found " + std::to_string(count));
            g.nbr[i][f] = found;
        }
    for (int i = 0; i < nb; ++i)
        for (int f = 0; f < 4; ++f) {
            int k = g.nbr[i][f];
            if (k >= 0 && g.nbr[k][f ^ 1] != i) return fail(err, "connectivity not symmetric");
            if (k < 0) continue;
            const std::vector<double>& a = f < 2 ? g.yf[i] : g.xf[i];
            const std::vector<double>& c = f < 2 ? g.yf[k] : g.xf[k];
            if (a.size() != c.size()) return fail(err, "joined faces differ in cell count");
            if (g.bc[i][f] == MBP_CONNECT) {
                double scale = std::max(std::fabs(a.front()), std::fabs(a.back())) + (a.back() - a.front());
                for (size_t t = 0; t < a.size(); ++t)
                    if (std::fabs(a[t] - c[t]) > 1e-12 * scale)
                        return fail(err, "joined faces are not congruent");
            }
        }
    g.dirichlet_xy = false;
    for (int i = 0; i < nb; ++i)
        for (int f = 0; f < 4; ++f)
            if (g.bc[i][f] == MBP_DIRICHLET) g.dirichlet_xy = true;
    bool zd = g.zlo == MBP_DIRICHLET || g.zhi == MBP_DIRICHLET;
    g.singular = !g.dirichlet_xy && !zd;
    return true;
}

std::vector<double> coarsen_faces(const std::vector<double>& f) {
    int n = int(f.size()) - 1, nc = n / 2;
    std::vector<double> c(nc + 1);
    for (int I = 0; I < nc; ++I) c[I] = f[2 * I];
    c[nc] = f[n];
    return c;
}

}  // namespace

// Symmetric eigen-decomposition by cyclic Jacobi rotations (A is overwritten;
// V receives the eigenvectors as columns, row-major n x n).
void jacobi_eig(std::vector<double>& A, int n, std::vector<double>& V, std::vector<double>& w) {
    V.assign(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) V[size_t(i) * n + i] = 1.0;
    auto a = [&](int i, int j) -> double& { return A[size_t(i) * n + j]; };
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += a(i, j) * a(i, j);
                if (i != j) off += a(i, j) * a(i, j);
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = a(p, q);
                if (std::fabs(apq) < 1e-300) continue;
                double app = a(p, p), aqq = a(q, q);
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    double akp = a(k, p), akq = a(k, q);
                    a(k, p) = c * akp - s * akq;
                    a(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = a(p, k), aqk = a(q, k);
                    a(p, k) = c * apk - s * aqk;
                    a(q, k) = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double vkp = V[size_t(k) * n + p], vkq = V[size_t(k) * n + q];
                    V[size_t(k) * n + p] = c * vkp - s * vkq;
                    V[size_t(k) * n + q] = s * vkp + c * vkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = a(i, i);
}

namespace {

std::vector<int> fft_radices(int m) {
    std::vector<int> r;
    while (m % 8 == 0) { r.push_back(8); m /= 8; }
    while (m % 4 == 0) { r.push_back(4); m /= 4; }
    while (m % 2 == 0) { r.push_back(2); m /= 2; }
    for (int p = 3; m > 1; p += 2)
        while (m % p == 0) { r.push_back(p); m /= p; }
    return r;
}

}  // namespace

// Modal shifts of Eq. (9), sigma_q = lambda_q / dz^2 - alpha, with alpha >= 0
// the Helmholtz term of the implicit-diffusion systems (Sec. 2; the diagonal
// changes every Runge-Kutta substep, footnote of Sec. 3.3.1).  Also the lower
// bound |mu + sigma_q| >= sabs_q of the mode's non-null eigenvalue magnitudes
// used by the error test: a plane without Dirichlet faces has the constant
// mode (mu = 0), so its smallest magnitude is |sigma_q| unless sigma_q = 0
// (the null mode, removed by the gauge), where it is mu0.  The problem is
// singular only without Dirichlet conditions and with alpha = 0.
void plan_set_shifts(mbp_plan* P) {
    const Geometry& g = P->g;
    const int nz = g.nz;
    const double alpha = P->opt.helmholtz;
    P->shift.resize(nz);
    P->sabs.resize(nz);
    for (int q = 0; q < nz; ++q) {
        const long double s = (long double)P->lambda[q] / ((long double)g.dz * g.dz) - alpha;
        P->shift[q] = double(s);
        const double as = std::fabs(P->shift[q]);
        P->sabs[q] = g.dirichlet_xy ? P->mu0 + as : (as > 0.0 ? as : P->mu0);
    }
    const bool zd = g.zlo == MBP_DIRICHLET || g.zhi == MBP_DIRICHLET;
    P->g.singular = !g.dirichlet_xy && !zd && alpha == 0.0;
}

int build_plan_host(const mbp_block_desc* blocks, int nblocks, const mbp_synth_desc* z,
                    const mbp_options* opt, mbp_plan* P, std::string* err) {
    return build_plan_host_limits(blocks, nblocks, z, opt, 64 * 1024, P, err);
}

int build_plan_host_limits(const mbp_block_desc* blocks, int nblocks, const mbp_synth_desc* z,
                           const mbp_options* opt, int64_t lds_limit, mbp_plan* P, std::string* err,
                           bool uniform_levels) {
    P->lds_limit = lds_limit;
    if (!validate(blocks, nblocks, z, P->g, err)) return MBP_ERR_INVALID;
    Geometry& g = P->g;
    if (opt) {
        P->opt = *opt;
        if (P->opt.precision != MBP_FP64 && P->opt.precision != MBP_MIXED) {
            if (err) *err = "unknown precision";
            return MBP_ERR_INVALID;
        }
        if (P->opt.nu1 < 0 || P->opt.nu2 < 0 || P->opt.nu1 + P->opt.nu2 < 1 || P->opt.nu1 > 8 ||
            P->opt.nu2 > 8 || P->opt.max_cycles < 1) {
            if (err) *err = "bad smoothing counts or max_cycles";
            return MBP_ERR_INVALID;
        }
        if (P->opt.inner == 0) P->opt.inner = 4;
        if (P->opt.inner < 1 || P->opt.inner > 8) {
            if (err) *err = "bad inner cycle count";
            return MBP_ERR_INVALID;
        }
        if (P->opt.march != 0 && P->opt.march != 1) {
            if (err) *err = "bad pre-smoothing form";
            return MBP_ERR_INVALID;
        }
        if (P->opt.smoother != MBP_SMOOTHER_DEFAULT && P->opt.smoother != MBP_SMOOTHER_RBGS) {
            if (err) *err = "unknown smoother";
            return MBP_ERR_INVALID;
        }
        if (!(P->opt.helmholtz >= 0.0) || !std::isfinite(P->opt.helmholtz)) {
            if (err) *err = "Helmholtz shift must be finite and >= 0";
            return MBP_ERR_INVALID;
        }
    } else {
        options_default(&P->opt);
    }
    const int nb = g.nb;
    const int nz = g.nz;

    // ---- modal shifts (Table 1): lambda_q = 2 (cos(2 pi k_q / n) - 1) ----
    P->lambda.resize(nz);
    P->shift.resize(nz);
    for (int q = 0; q < nz; ++q) {
        long double k;
        switch (g.zkind) {
            case Z_PP: k = q; break;
            case Z_NN: k = 0.5L * q; break;
            case Z_DD: k = 0.5L * (q + 1); break;
            default: k = 0.25L * (2 * q + 1); break;
        }
        long double lam = 2.0L * (std::cos(2.0L * 3.14159265358979323846264338327950288L * k / nz) - 1.0L);
        if (g.zkind == Z_PP && q == 0) lam = 0.0L;
        if (g.zkind == Z_NN && q == 0) lam = 0.0L;
        P->lambda[q] = double(lam);
    }

    // ---- multigrid levels.  Each step coarsens the direction(s) with the
    //      smaller mean cell width, as PFMG picks its semicoarsening direction
    //      (Sec. 3.3.1): x alone when the mean x width is below the mean y
    //      width over sqrt(2), y alone in the opposite case, both otherwise.
    //      Uniform steps (every block takes each step) unless they leave too
    //      large a coarsest plane, see below.  Per-class steps: blocks joined
    //      across a y face share their x cells, so they halve x together;
    //      blocks joined across an x face halve y together.  Each such class
    //      halves a direction while its blocks have at least 4 cells along
    //      it; a thinner class then merges its 2 or 3 cells into one while
    //      other classes go on halving, where that direction is its cells'
    //      strongly coupled one.  A thin block thus does not hold back the
    //      rest of the plane; the hierarchy ends when no class can halve the
    //      chosen direction(s).  Odd counts merge their last three cells ----
    std::vector<int> xcls(nb), ycls(nb);
    {
        auto find = [](std::vector<int>& u, int a) {
            while (u[a] != a) a = u[a] = u[u[a]];
            return a;
        };
        for (int b = 0; b < nb; ++b) xcls[b] = ycls[b] = b;
        for (int b = 0; b < nb; ++b)
            for (int f = 0; f < 4; ++f) {
                const int k = g.nbr[b][f];
                if (k < 0) continue;
                std::vector<int>& u = f < 2 ? ycls : xcls;  // x faces tie y cells, y faces x cells
                const int ra = find(u, b), rb = find(u, k);
                if (ra != rb) u[std::max(ra, rb)] = std::min(ra, rb);
            }
        for (int b = 0; b < nb; ++b) {
            xcls[b] = find(xcls, b);
            ycls[b] = find(ycls, b);
        }
    }
    auto build_levels = [&](bool uniform) {
        P->levels.clear();
        {
            Level L;
            L.nb = nb;
            L.nx = g.nx;
            L.ny = g.ny;
            L.xf = g.xf;
            L.yf = g.yf;
            P->levels.push_back(L);
        }
        while (P->levels.size() < 24) {
            Level& F = P->levels.back();
            if (!uniform) {
                // per-class steps end once the plane fits an exact solve of
                // a few hundred cells: deeper, thin blocks left one or two
                // cells wide beside far coarser neighbours made the cycle
                // slow (268 V-cycles on one layout, 67 when stopped here)
                // or even divergent
                int64_t cells = 0;
                for (int b = 0; b < nb; ++b) cells += int64_t(F.nx[b]) * F.ny[b];
                if (cells <= 256) break;
            }
            double wx = 0.0, wy = 0.0;
            int64_t cellsx = 0, cellsy = 0;
            // per class (indexed by its representative): every block has at
            // least 4 cells along the direction (halve), or 2-3 (merge into one
            // cell, taken only while another class halves that direction, so a
            // thin block follows its neighbours one step further)
            std::vector<char> canx(nb, 1), cany(nb, 1), mrgx(nb, 1), mrgy(nb, 1);
            for (int b = 0; b < nb; ++b) {
                if (F.nx[b] < 4) canx[xcls[b]] = 0;
                if (F.ny[b] < 4) cany[ycls[b]] = 0;
                // (a periodic wrap keeps at least two cells)
                if (F.nx[b] < 2 || g.bc[b][XM] == MBP_PERIODIC || g.bc[b][XP] == MBP_PERIODIC) mrgx[xcls[b]] = 0;
                if (F.ny[b] < 2 || g.bc[b][YM] == MBP_PERIODIC || g.bc[b][YP] == MBP_PERIODIC) mrgy[ycls[b]] = 0;
                wx += F.xf[b].back() - F.xf[b].front();
                wy += F.yf[b].back() - F.yf[b].front();
                cellsx += F.nx[b];
                cellsy += F.ny[b];
            }
            const double hx = wx / double(cellsx), hy = wy / double(cellsy);
            // halving the smaller width alone brings the ratio closer to 1 once
            // it exceeds sqrt(2)
            const double r2 = 0.70710678118654752440;
            const bool dirx = !(hy < r2 * hx), diry = !(hx < r2 * hy);
            bool halvex = false, halvey = false;
            for (int b = 0; b < nb; ++b) {
                halvex = halvex || (dirx && canx[xcls[b]]);
                halvey = halvey || (diry && cany[ycls[b]]);
            }
            // a merge must leave the block's cells no more anisotropic than
            // they would be without it: the merged direction has to be the
            // block's strongly coupled one (width below the other direction's
            // next-level width over sqrt(2)), as the direction rule itself asks
            for (int b = 0; b < nb; ++b) {
                const double wxb = (F.xf[b].back() - F.xf[b].front()) / F.nx[b];
                const double wyb = (F.yf[b].back() - F.yf[b].front()) / F.ny[b];
                const double wxn = (dirx && canx[xcls[b]]) ? 2.0 * wxb : wxb;
                const double wyn = (diry && cany[ycls[b]]) ? 2.0 * wyb : wyb;
                if (!(wxb < r2 * wyn)) mrgx[xcls[b]] = 0;
                if (!(wyb < r2 * wxn)) mrgy[ycls[b]] = 0;
            }
            std::vector<char> bx(nb), by(nb);
            bool any = false, allx = true, ally = true;
            for (int b = 0; b < nb; ++b) {
                const bool hxb = dirx && canx[xcls[b]], hyb = diry && cany[ycls[b]];
                bx[b] = hxb || (!uniform && halvex && !canx[xcls[b]] && mrgx[xcls[b]]);
                by[b] = hyb || (!uniform && halvey && !cany[ycls[b]] && mrgy[ycls[b]]);
                any = any || bx[b] || by[b];
                allx = allx && hxb;
                ally = ally && hyb;
            }
            if (!any) break;
            if (uniform && ((dirx && !allx) || (diry && !ally))) break;
            F.cx = allx ? 1 : 0;
            F.cy = ally ? 1 : 0;
            Level C;
            C.nb = nb;
            C.nx.resize(nb);
            C.ny.resize(nb);
            C.xf.resize(nb);
            C.yf.resize(nb);
            for (int b = 0; b < nb; ++b) {
                C.xf[b] = bx[b] ? coarsen_faces(F.xf[b]) : F.xf[b];
                C.yf[b] = by[b] ? coarsen_faces(F.yf[b]) : F.yf[b];
                C.nx[b] = int(C.xf[b].size()) - 1;
                C.ny[b] = int(C.yf[b].size()) - 1;
            }
            P->levels.push_back(C);
        }
    };
    // Every block takes each step (the hierarchy ends when one block cannot)
    // unless that leaves more than 256 coarsest cells: then each class of
    // blocks steps on its own, down to 256 cells.  Per-class steps converge
    // slower on layouts whose thin blocks stay one or two cells wide while
    // their neighbours coarsen, while a large coarsest plane costs the plan
    // an O(n^3) eigen-decomposition (seconds at a few hundred cells, minutes
    // near 2048).
    auto coarsest = [&]() {
        int64_t cells = 0;
        for (int b = 0; b < nb; ++b) cells += int64_t(P->levels.back().nx[b]) * P->levels.back().ny[b];
        return cells;
    };
    build_levels(true);
    if (!uniform_levels && coarsest() > 256) build_levels(false);
    P->nlev = int(P->levels.size());
    for (Level& L : P->levels) {
        L.off.resize(nb + 1);
        L.off[0] = 0;
        for (int b = 0; b < nb; ++b) L.off[b + 1] = L.off[b] + L.nx[b] * L.ny[b];
        L.plane = L.off[nb];
    }
    P->plane0 = P->levels[0].plane;
    if (P->plane0 > (int64_t(1) << 30)) {
        if (err) *err = "plane too large";
        return MBP_ERR_INVALID;
    }
    P->ncells = P->plane0 * nz;
    P->coarse_n = int(P->levels.back().plane);
    if (P->coarse_n > 2048) {
        if (err) *err = "coarsest plane exceeds 2048 cells (cells too anisotropic to coarsen further)";
        return MBP_ERR_INVALID;
    }
    P->block_off.resize(nb + 1);
    P->block_off[0] = 0;
    for (int b = 0; b < nb; ++b)
        P->block_off[b + 1] = P->block_off[b] + int64_t(nz) * g.nx[b] * g.ny[b];

    // ---- tables ----
    P->hblk.clear();
    P->hint.clear();
    P->hdbl.clear();
    P->htiles.clear();
    auto push_d = [&](const std::vector<double>& v) {
        int o = int(P->hdbl.size());
        P->hdbl.insert(P->hdbl.end(), v.begin(), v.end());
        return o;
    };
    auto push_i = [&](const std::vector<int>& v) {
        int o = int(P->hint.size());
        P->hint.insert(P->hint.end(), v.begin(), v.end());
        return o;
    };
    for (int l = 0; l < P->nlev; ++l) {
        Level& L = P->levels[l];
        L.blk_off = int(P->hblk.size());
        L.dp_begin = int(P->hdbl.size());
        L.ip_begin = int(P->hint.size());
        // colour parity: a breadth-first walk makes joined neighbours differ
        std::vector<int> par(nb, -1);
        for (int s = 0; s < nb; ++s) {
            if (par[s] >= 0) continue;
            par[s] = 0;
            std::vector<int> stack{s};
            while (!stack.empty()) {
                int b = stack.back();
                stack.pop_back();
                for (int f = 0; f < 4; ++f) {
                    int k = g.nbr[b][f];
                    if (k < 0 || par[k] >= 0) continue;
                    int n;
                    if (f == XP) n = L.nx[b];
                    else if (f == XM) n = L.nx[k];
                    else if (f == YP) n = L.ny[b];
                    else n = L.ny[k];
                    par[k] = (par[b] + n) & 1;
                    stack.push_back(k);
                }
            }
        }
        for (int b = 0; b < nb; ++b) {
            DBlock d{};
            d.nx = L.nx[b];
            d.ny = L.ny[b];
            d.off = L.off[b];
            for (int f = 0; f < 4; ++f) {
                d.nbr[f] = g.nbr[b][f];
                d.bc[f] = g.bc[b][f];
            }
            d.par = par[b];
            // an odd cell count around a periodic wrap cannot be two-coloured:
            // its last column / row is relaxed in two extra passes
            d.oddwrap = 0;
            if (g.bc[b][XP] == MBP_PERIODIC && g.nbr[b][XP] == b && (L.nx[b] & 1)) d.oddwrap |= 1;
            if (g.bc[b][YP] == MBP_PERIODIC && g.nbr[b][YP] == b && (L.ny[b] & 1)) d.oddwrap |= 2;
            if (d.oddwrap) L.oddwrap = true;
            // coefficients along each axis
            for (int axis = 0; axis < 2; ++axis) {
                const std::vector<double>& F = axis == 0 ? L.xf[b] : L.yf[b];
                int n = int(F.size()) - 1;
                std::vector<double> dc(n), cc(n), co(3 * n, 0.0);
                for (int i = 0; i < n; ++i) {
                    dc[i] = F[i + 1] - F[i];
                    cc[i] = 0.5 * (F[i + 1] + F[i]);
                }
                int fm = axis == 0 ? XM : YM, fp = axis == 0 ? XP : YP;
                for (int i = 0; i < n; ++i) {
                    double wm = 0.0, wp = 0.0, extra = 0.0;
                    if (i > 0) wm = 1.0 / (dc[i] * (cc[i] - cc[i - 1]));
                    else {
                        int k = g.nbr[b][fm];
                        if (k >= 0) {
                            const std::vector<double>& Fk = axis == 0 ? L.xf[k] : L.yf[k];
                            double dk = Fk[Fk.size() - 1] - Fk[Fk.size() - 2];
                            wm = 1.0 / (dc[0] * 0.5 * (dc[0] + dk));
                        } else if (g.bc[b][fm] == MBP_DIRICHLET) {
                            extra += 2.0 / (dc[0] * dc[0]);
                        }
                    }
                    if (i < n - 1) wp = 1.0 / (dc[i] * (cc[i + 1] - cc[i]));
                    else {
                        int k = g.nbr[b][fp];
                        if (k >= 0) {
                            const std::vector<double>& Fk = axis == 0 ? L.xf[k] : L.yf[k];
                            double dk = Fk[1] - Fk[0];
                            wp = 1.0 / (dc[n - 1] * 0.5 * (dc[n - 1] + dk));
                        } else if (g.bc[b][fp] == MBP_DIRICHLET) {
                            extra += 2.0 / (dc[n - 1] * dc[n - 1]);
                        }
                    }
                    co[i] = wm;
                    co[n + i] = wp;
                    co[2 * n + i] = -(wm + wp) - extra;
                }
                if (axis == 0) d.cx = push_d(co);
                else d.cy = push_d(co);
            }
            // transfer tables to the next level
            d.rsx = d.rsy = d.rwx = d.rwy = d.pcx = d.pcy = d.pwx = d.pwy = -1;
            if (l + 1 < P->nlev) {
                const Level& C = P->levels[l + 1];
                for (int axis = 0; axis < 2; ++axis) {
                    const std::vector<double>& F = axis == 0 ? L.xf[b] : L.yf[b];
                    const std::vector<double>& G = axis == 0 ? C.xf[b] : C.yf[b];
                    int n = int(F.size()) - 1, nc = int(G.size()) - 1;
                    // a direction the next level keeps (semicoarsening) maps cell
                    // i to itself: one child, weight 1; the prolongation
                    // tables below then give weight 1 to the coincident centre
                    const int ratio = nc == n ? 1 : 2;
                    std::vector<int> rs(nc + 1);
                    for (int I = 0; I < nc; ++I) rs[I] = ratio * I;
                    rs[nc] = n;
                    std::vector<double> rw(n);
                    for (int i = 0; i < n; ++i) {
                        int I = std::min(i / ratio, nc - 1);
                        rw[i] = (F[i + 1] - F[i]) / (G[I + 1] - G[I]);
                    }
                    // prolongation: coarse centres with a ghost centre beyond each face
                    std::vector<double> ext(nc + 2);
                    for (int I = 0; I < nc; ++I) ext[I + 1] = 0.5 * (G[I] + G[I + 1]);
                    int fm = axis == 0 ? XM : YM, fp = axis == 0 ? XP : YP;
                    int k = g.nbr[b][fm];
                    if (k >= 0) {
                        const std::vector<double>& Gk = axis == 0 ? C.xf[k] : C.yf[k];
                        ext[0] = G[0] - 0.5 * (Gk[Gk.size() - 1] - Gk[Gk.size() - 2]);
                    } else {
                        ext[0] = 2.0 * G[0] - ext[1];
                    }
                    k = g.nbr[b][fp];
                    if (k >= 0) {
                        const std::vector<double>& Gk = axis == 0 ? C.xf[k] : C.yf[k];
                        ext[nc + 1] = G[nc] + 0.5 * (Gk[1] - Gk[0]);
                    } else {
                        ext[nc + 1] = 2.0 * G[nc] - ext[nc];
                    }
                    std::vector<int> pc(n);
                    std::vector<double> pw(n);
                    for (int i = 0; i < n; ++i) {
                        double x = 0.5 * (F[i] + F[i + 1]);
                        int t = 0;
                        while (t < nc && ext[t + 1] <= x) ++t;
                        pc[i] = t - 1;
                        pw[i] = (ext[t + 1] - x) / (ext[t + 1] - ext[t]);
                    }
                    if (axis == 0) {
                        d.rsx = push_i(rs); d.rwx = push_d(rw); d.pcx = push_i(pc); d.pwx = push_d(pw);
                    } else {
                        d.rsy = push_i(rs); d.rwy = push_d(rw); d.pcy = push_i(pc); d.pwy = push_d(pw);
                    }
                }
            }
            P->hblk.push_back(d);
        }
        // tiles of the global-memory kernels
        L.tile_off = int(P->htiles.size());
        for (int b = 0; b < nb; ++b)
            for (int y0 = 0; y0 < L.ny[b]; y0 += kTileY)
                for (int x0 = 0; x0 < L.nx[b]; x0 += kTileX) P->htiles.push_back(make_int4(b, x0, y0, 0));
        L.ntiles = int(P->htiles.size()) - L.tile_off;
    }

    P->dp_levels_end = int(P->hdbl.size());
    P->ip_levels_end = int(P->hint.size());

    // ---- finest-plane areas (compatibility projection, gauge) ----
    {
        const Level& L = P->levels[0];
        P->areas0.resize(L.plane);
        double s = 0.0;
        for (int b = 0; b < nb; ++b)
            for (int j = 0; j < L.ny[b]; ++j)
                for (int i = 0; i < L.nx[b]; ++i) {
                    double a = (L.xf[b][i + 1] - L.xf[b][i]) * (L.yf[b][j + 1] - L.yf[b][j]);
                    P->areas0[L.off[b] + j * L.nx[b] + i] = a;
                    s += a;
                }
        P->area_sum = s;
    }

    // ---- coarsest plane: eigen-decomposition of the symmetrised operator ----
    {
        const Level& L = P->levels.back();
        const int nc = int(L.plane);
        std::vector<double> A(size_t(nc) * nc, 0.0), area(nc);
        for (int b = 0; b < nb; ++b) {
            const DBlock& d = P->hblk[L.blk_off + b];
            const double* cx = &P->hdbl[d.cx];
            const double* cy = &P->hdbl[d.cy];
            for (int j = 0; j < d.ny; ++j)
                for (int i = 0; i < d.nx; ++i) {
                    int c = d.off + j * d.nx + i;
                    area[c] = (L.xf[b][i + 1] - L.xf[b][i]) * (L.yf[b][j + 1] - L.yf[b][j]);
                    A[size_t(c) * nc + c] += cx[2 * d.nx + i] + cy[2 * d.ny + j];
                    auto addnb = [&](int f, double w, int ii, int jj) {
                        if (w == 0.0) return;
                        int bb = b;
                        if (ii < 0 || ii >= d.nx || jj < 0 || jj >= d.ny) {
                            // the partner's last / first column or row; the
                            // tests read the original index (the partner may
                            // be longer along the crossed direction)
                            bb = g.nbr[b][f];
                            const DBlock& e = P->hblk[L.blk_off + bb];
                            if (ii < 0) ii = e.nx - 1;
                            else if (ii >= d.nx) ii = 0;
                            if (jj < 0) jj = e.ny - 1;
                            else if (jj >= d.ny) jj = 0;
                        }
                        const DBlock& e = P->hblk[L.blk_off + bb];
                        A[size_t(c) * nc + (e.off + jj * e.nx + ii)] += w;
                    };
                    addnb(XM, cx[i], i - 1, j);
                    addnb(XP, cx[d.nx + i], i + 1, j);
                    addnb(YM, cy[j], i, j - 1);
                    addnb(YP, cy[d.ny + j], i, j + 1);
                }
        }
        // S = diag(a)^(1/2) A diag(a)^(-1/2) is symmetric (the fluxes of the
        // finite-volume operator); check it, so that a wrong coupling cannot
        // hide behind the symmetrisation below
        std::vector<double> S(size_t(nc) * nc);
        double smax = 0.0;
        for (int r = 0; r < nc; ++r)
            for (int c = 0; c < nc; ++c) {
                S[size_t(r) * nc + c] = std::sqrt(area[r]) * A[size_t(r) * nc + c] / std::sqrt(area[c]);
                smax = std::max(smax, std::fabs(S[size_t(r) * nc + c]));
            }
        for (int r = 0; r < nc; ++r)
            for (int c = r + 1; c < nc; ++c)
                if (std::fabs(S[size_t(r) * nc + c] - S[size_t(c) * nc + r]) > 1e-10 * smax) {
                    if (err) *err = "internal: coarsest-plane operator is not symmetric";
                    return MBP_ERR_INVALID;
                }
        for (int r = 0; r < nc; ++r)
            for (int c = r + 1; c < nc; ++c) {
                double m = 0.5 * (S[size_t(r) * nc + c] + S[size_t(c) * nc + r]);
                S[size_t(r) * nc + c] = S[size_t(c) * nc + r] = m;
            }
        std::vector<double> V, mu;
        jacobi_eig(S, nc, V, mu);
        P->coarse_mu = mu;
        // smallest non-zero eigenvalue magnitude (the null mode of a singular
        // plane is excluded: the gauge removes it from the error)
        double mmax = 0.0;
        for (double v : mu) mmax = std::max(mmax, std::fabs(v));
        double m0 = mmax;
        for (double v : mu)
            if (std::fabs(v) > 1e-9 * mmax) m0 = std::min(m0, std::fabs(v));
        P->mu0 = m0;
        P->coarse_wl.resize(size_t(nc) * nc);
        P->coarse_wr.resize(size_t(nc) * nc);
        for (int r = 0; r < nc; ++r)
            for (int k = 0; k < nc; ++k) {
                P->coarse_wl[size_t(r) * nc + k] = V[size_t(r) * nc + k] / std::sqrt(area[r]);
                P->coarse_wr[size_t(k) * nc + r] = V[size_t(r) * nc + k] * std::sqrt(area[r]);
            }
    }

    // ---- LDS-resident levels: the smallest index whose remaining hierarchy
    //      (p and rhs of every level) fits the LDS budget.  The FP64 V-cycle
    //      may take a workgroup's whole budget.  The FP32 one (mixed
    //      precision, run for many modes and problems at once) is kept to a
    //      quarter of it: most of its phases keep few lanes busy, so its
    //      throughput comes from four workgroups sharing a CU, not from
    //      one more LDS-resident level ----
    {
        const int64_t budget = P->lds_limit;
        const int64_t budget32 = std::max<int64_t>(budget / 4, 16 * 1024);
        // p and f of every level from L0, the coarse temporary and reduction
        // scratch, and a copy of those levels' coefficient / transfer tables
        auto need = [&](int L0, int64_t elem) {
            int64_t e = 0;
            for (int l = L0; l < P->nlev; ++l) e += 2 * P->levels[l].plane;
            const int64_t tables = int64_t(P->dp_levels_end - P->levels[L0].dp_begin) * 8 +
                                   int64_t(P->ip_levels_end - P->levels[L0].ip_begin) * 4 +
                                   int64_t(P->nlev - L0) * nb * int64_t(sizeof(DBlock));
            return e * elem + int64_t(P->coarse_n) * 8 + 1024 + tables;
        };
        P->lds_level = P->nlev - 1;
        for (int l = P->nlev - 1; l >= 0; --l)
            if (need(l, 8) <= budget) P->lds_level = l;
        P->lds_level32 = P->nlev - 1;
        for (int l = P->nlev - 1; l >= 0; --l)
            if (need(l, 4) <= budget32) P->lds_level32 = l;
        P->lds_bytes64 = need(P->lds_level, 8);
        P->lds_bytes32 = need(P->lds_level32, 4);
        // two FP64 workgroups share a CU when the image fits half the budget;
        // if it only fits once the top level's rhs stays in device memory
        // (read by two sweeps and the restriction per cycle), keep it there.
        // Not when the whole solve runs in LDS (level 0) or the top level is
        // the coarsest (its rhs feeds the eigen solve from LDS).
        P->lds_fglob64 = 0;
        {
            const int64_t fbytes = P->levels[P->lds_level].plane * 8;
            if (P->lds_level > 0 && P->lds_level < P->nlev - 1 && P->lds_bytes64 > budget / 2 &&
                P->lds_bytes64 - fbytes <= budget / 2) {
                P->lds_fglob64 = 1;
                P->lds_bytes64 -= fbytes;
            }
        }
        if (P->lds_bytes64 > budget) {
            if (err) *err = "coarsest plane does not fit the LDS budget";
            return MBP_ERR_INVALID;
        }
        int64_t o = 0;
        for (int l = 0; l < P->nlev; ++l) {
            P->levels[l].lds_off = l >= P->lds_level ? o : -1;
            if (l >= P->lds_level) o += 2 * P->levels[l].plane;
        }
    }

    plan_set_shifts(P);

    // ---- level summary for the kernels ----
    {
        std::vector<int> li;
        for (const Level& L : P->levels) {
            li.push_back(int(L.plane));
            li.push_back(L.blk_off);
            li.push_back(L.tile_off);
            li.push_back(L.ntiles);
        }
        P->lvinfo = push_i(li);
    }

    // ---- projection tables of the finest level (staggered velocities on the
    //      faces): per block {dcx, dcy, gx, gy offsets, rows and columns of
    //      the blocks before it}; gx / gy hold 1 / (centre distance) per face
    //      (walls: 0 for Neumann, 1 / dc for Dirichlet with the mirrored
    //      ghost -p, joined faces 2 / (dc + dc_partner)) ----
    {
        std::vector<int> pt;
        int cny = 0, cnx = 0;
        const Level& L = P->levels[0];
        for (int b = 0; b < nb; ++b) {
            int offs[4];
            for (int axis = 0; axis < 2; ++axis) {
                const std::vector<double>& F = axis == 0 ? L.xf[b] : L.yf[b];
                const int n = int(F.size()) - 1;
                std::vector<double> dc(n), gf(n + 1, 0.0);
                for (int i = 0; i < n; ++i) dc[i] = F[i + 1] - F[i];
                for (int i = 1; i < n; ++i) gf[i] = 1.0 / (0.5 * (F[i + 1] + F[i]) - 0.5 * (F[i] + F[i - 1]));
                const int fm = axis == 0 ? XM : YM, fp = axis == 0 ? XP : YP;
                for (int side = 0; side < 2; ++side) {
                    const int f = side == 0 ? fm : fp;
                    const int at = side == 0 ? 0 : n;
                    const double dc0 = side == 0 ? dc[0] : dc[n - 1];
                    const int k = g.nbr[b][f];
                    if (k >= 0) {
                        const std::vector<double>& Fk = axis == 0 ? L.xf[k] : L.yf[k];
                        const double dk = side == 0 ? Fk[Fk.size() - 1] - Fk[Fk.size() - 2] : Fk[1] - Fk[0];
                        gf[at] = 1.0 / (0.5 * (dc0 + dk));
                    } else {
                        gf[at] = g.bc[b][f] == MBP_DIRICHLET ? 1.0 / dc0 : 0.0;
                    }
                }
                offs[axis] = push_d(dc);
                offs[2 + axis] = push_d(gf);
            }
            pt.insert(pt.end(), {offs[0], offs[1], offs[2], offs[3], cny, cnx});
            cny += L.ny[b];
            cnx += L.nx[b];
        }
        P->proj_tab = push_i(pt);
    }

    // ---- z transform tables (twiddles in extended precision) ----
    P->fft.n = nz;
    P->fft.m = nz / 2;
    P->fft.radices = fft_radices(P->fft.m);

    {
        const long double PI = 3.14159265358979323846264338327950288L;
        const int n = nz, m = nz / 2;
        auto cexp_table = [&](int count, auto angle) {
            std::vector<double> t(2 * size_t(count));
            for (int k = 0; k < count; ++k) {
                long double a = angle(k);
                t[2 * k] = double(std::cos(a));
                t[2 * k + 1] = double(std::sin(a));
            }
            return t;
        };
        P->fft_tw = push_d(cexp_table(m, [&](int t) { return -2.0L * PI * t / m; }));
        P->fft_twn = push_d(cexp_table(m + 1, [&](int k) { return -2.0L * PI * k / n; }));
        P->fft_post = push_d(cexp_table(n + 1, [&](int k) { return -PI * k / (2.0L * n); }));
        P->fft_pre4 = push_d(cexp_table(m, [&](int k) { return -PI * (4.0L * k + 1.0L) / (4.0L * n); }));
        P->fft_post4 = push_d(cexp_table(m, [&](int k) { return -PI * k / (long double)n; }));
    }
    return MBP_OK;
}

}  // namespace mbp
