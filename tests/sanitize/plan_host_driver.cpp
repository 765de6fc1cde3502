// Host-side checks of the plan builder under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_host.py with the sanitizers
// on the host pass only).  It runs no HIP call: validation, connectivity,
// congruence, the multigrid hierarchy, modal shifts (Eq. (9), with the
// Helmholtz term), transform tables (Table 1), the Jacobi eigen-solver of the
// coarsest plane and the tanh face mapping, over valid layouts (hand-built and
// seeded random ones) and a set of invalid descriptors that must be refused
// with a message.
#include <cmath>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "internal.h"

namespace {

int failures = 0;
#define CHECK(c, ...)                                   \
    do {                                                \
        if (!(c)) {                                     \
            std::fprintf(stderr, "FAIL %s:%d ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);          \
            std::fprintf(stderr, "\n");                 \
            ++failures;                                 \
        }                                               \
    } while (0)

std::vector<double> faces(int n, double a, double b, int type = 0, double factor = 0.0) {
    std::vector<double> f(n + 1);
    const int st = mbp::grid_tanh(n, a, b, type, factor, f.data());
    CHECK(st == MBP_OK, "grid_tanh n=%d", n);
    return f;
}

struct Layout {
    std::vector<std::vector<double>> xf, yf;
    std::vector<mbp_block_desc> b;
    void add(int x0, int y0, int nx, int ny, double ax, double bx, double ay, double by, int bxm, int bxp, int bym,
             int byp, double fy = 0.0) {
        xf.push_back(faces(nx, ax, bx));
        yf.push_back(faces(ny, ay, by, 0, fy));
        mbp_block_desc d{};
        d.lo[0] = x0;
        d.lo[1] = y0;
        d.hi[0] = x0 + nx - 1;
        d.hi[1] = y0 + ny - 1;
        d.bc[0] = bxm;
        d.bc[1] = bxp;
        d.bc[2] = bym;
        d.bc[3] = byp;
        b.push_back(d);
    }
    std::vector<mbp_block_desc> descs() {
        std::vector<mbp_block_desc> out = b;
        for (size_t i = 0; i < out.size(); ++i) {
            out[i].xf = xf[i].data();
            out[i].yf = yf[i].data();
        }
        return out;
    }
};

int build(Layout& L, int nz, int zlo, int zhi, double alpha, std::string* err, int* nlev = nullptr) {
    std::vector<mbp_block_desc> d = L.descs();
    mbp_synth_desc z{nz, 1.0, zlo, zhi};
    mbp_options o;
    mbp::options_default(&o);
    o.helmholtz = alpha;
    mbp_plan P;
    const int st = mbp::build_plan_host_limits(d.data(), int(d.size()), &z, &o, 160 * 1024, &P, err);
    if (st == MBP_OK) {
        CHECK(P.nlev >= 1, "levels");
        CHECK(int(P.shift.size()) == nz, "shifts");
        for (int q = 0; q < nz; ++q) CHECK(std::isfinite(P.shift[q]) && P.sabs[q] >= 0.0, "shift %d", q);
        if (nlev) *nlev = P.nlev;
    }
    return st;
}

const int D = MBP_DIRICHLET, N = MBP_NEUMANN, C = MBP_CONNECT, P = MBP_PERIODIC;

void valid_layouts() {
    std::string err;
    const int pairs[5][2] = {{P, P}, {N, N}, {D, D}, {N, D}, {D, N}};
    for (auto& pr : pairs) {
        for (int nz : {2, 6, 74, 512, 1018}) {
            Layout box;
            box.add(1, 1, 40, 36, 0.0, 1.0, 0.0, 0.9, D, D, N, N, 1.2);
            CHECK(build(box, nz, pr[0], pr[1], 0.0, &err) == MBP_OK, "box nz=%d: %s", nz, err.c_str());
            CHECK(build(box, nz, pr[0], pr[1], 3.5, &err) == MBP_OK, "box helmholtz nz=%d: %s", nz, err.c_str());
        }
    }
    // L-shape: A, B to its right, C above it
    Layout l;
    l.add(1, 1, 32, 32, 0.0, 1.0, 0.0, 1.0, N, C, N, C, 1.5);
    l.add(33, 1, 32, 32, 1.0, 2.0, 0.0, 1.0, C, N, N, N, 1.5);
    l.add(1, 33, 32, 32, 0.0, 1.0, 1.0, 2.0, N, N, C, N, 1.5);
    int nlev = 0;
    CHECK(build(l, 16, P, P, 0.0, &err, &nlev) == MBP_OK, "lshape: %s", err.c_str());
    CHECK(nlev >= 3, "lshape levels %d", nlev);
    // four blocks meeting at a point
    Layout f;
    f.add(1, 1, 20, 16, 0.0, 1.0, 0.0, 1.0, D, C, N, C);
    f.add(21, 1, 12, 16, 1.0, 1.6, 0.0, 1.0, C, D, N, C);
    f.add(1, 17, 20, 10, 0.0, 1.0, 1.0, 1.5, D, C, C, N);
    f.add(21, 17, 12, 10, 1.0, 1.6, 1.0, 1.5, C, D, C, N);
    CHECK(build(f, 8, N, D, 0.0, &err) == MBP_OK, "four blocks: %s", err.c_str());
    // eight blocks around a square obstacle
    Layout o;
    const int w[3] = {2, 1, 2}, x0[4] = {0, 2, 3, 5}, y0[4] = {0, 1, 2, 3};
    const int n = 8;
    for (int row = 0; row < 3; ++row)
        for (int col = 0; col < 3; ++col) {
            if (row == 1 && col == 1) continue;
            const int bxm = col == 0 ? N : (row == 1 && col == 2) ? N : C;
            const int bxp = col == 2 ? D : (row == 1 && col == 0) ? N : C;
            const int bym = row == 0 ? D : (col == 1 && row == 2) ? N : C;
            const int byp = row == 2 ? D : (col == 1 && row == 0) ? N : C;
            o.add(x0[col] * n + 1, y0[row] * n + 1, w[col] * n, n, x0[col], x0[col + 1], y0[row], y0[row + 1], bxm,
                  bxp, bym, byp);
        }
    CHECK(build(o, 12, P, P, 0.0, &err) == MBP_OK, "obstacle: %s", err.c_str());
    // periodic x with an odd ring on the finest grid
    Layout r;
    r.add(1, 1, 15, 12, 0.0, 1.0, 0.0, 1.0, P, P, D, N);
    CHECK(build(r, 4, N, N, 0.0, &err) == MBP_OK, "odd ring: %s", err.c_str());
}

// Seeded random layouts: rows and columns of 2-4 joined blocks (some closed
// into periodic rings), L shapes and 2 x 2 grids, with blocks from one cell
// wide to 160 cells, stretched faces across the joins and random walls.  Every
// one must plan, with its coarsest plane within the dense-solve limit.
void random_layouts() {
    std::mt19937 rng(2106);
    auto uni = [&](int a, int b) { return std::uniform_int_distribution<int>(a, b)(rng); };
    auto wall = [&]() { return uni(0, 1) ? D : N; };
    const int zp[5][2] = {{P, P}, {N, N}, {D, D}, {N, D}, {D, N}};
    const double h = 1.0 / 32;
    std::string err;
    for (int s = 0; s < 240; ++s) {
        const int scale = (s % 3 == 2) ? 4 : 1;
        auto width = [&]() { return uni(0, 9) < 3 ? uni(1, 5) : uni(6, 40) * scale; };
        const int shape = s % 4;
        const double fy = 0.2 * uni(0, 4);
        Layout L;
        if (shape < 2) {  // a row (joined in x) or a column (joined in y)
            const int nb = uni(2, 4), cross = width();
            const bool ring = uni(0, 3) == 0;
            int at = 1;
            double a0 = 0.0;
            for (int b = 0; b < nb; ++b) {
                const int len = width();
                const double a1 = a0 + len * h;
                const int lo = b == 0 ? (ring ? P : wall()) : C, hi = b == nb - 1 ? (ring ? P : wall()) : C;
                if (shape == 0)
                    L.add(at, 1, len, cross, a0, a1, 0.0, cross * h, lo, hi, wall(), wall(), fy);
                else
                    L.add(1, at, cross, len, 0.0, cross * h, a0, a1, wall(), wall(), lo, hi, fy);
                at += len;
                a0 = a1;
            }
        } else {  // an L (three blocks) or a 2 x 2 grid
            const int w0 = width(), w1 = width(), h0 = width(), h1 = width();
            const double x1 = w0 * h, x2 = (w0 + w1) * h, y1 = h0 * h, y2 = (h0 + h1) * h;
            const bool grid = shape == 3;
            L.add(1, 1, w0, h0, 0.0, x1, 0.0, y1, wall(), C, wall(), C, fy);
            L.add(1 + w0, 1, w1, h0, x1, x2, 0.0, y1, C, wall(), wall(), grid ? C : wall(), fy);
            L.add(1, 1 + h0, w0, h1, 0.0, x1, y1, y2, wall(), grid ? C : wall(), C, wall(), fy);
            if (grid) L.add(1 + w0, 1 + h0, w1, h1, x1, x2, y1, y2, C, wall(), C, wall(), fy);
        }
        const int* z = zp[s % 5];
        const int nz = 2 * uni(1, 8);
        int nlev = 0;
        const int st = build(L, nz, z[0], z[1], s % 7 == 0 ? 2.5 : 0.0, &err, &nlev);
        CHECK(st == MBP_OK, "random layout %d (shape %d, %zu blocks): %s", s, shape, L.b.size(), err.c_str());
    }
}

void invalid_layouts() {
    std::string err;
    Layout box;
    box.add(1, 1, 16, 16, 0.0, 1.0, 0.0, 1.0, D, D, N, N);
    err.clear();
    CHECK(build(box, 7, N, N, 0.0, &err) == MBP_ERR_INVALID && !err.empty(), "odd nz");
    err.clear();
    CHECK(build(box, 0, N, N, 0.0, &err) == MBP_ERR_INVALID, "nz 0");
    err.clear();
    CHECK(build(box, 8, P, N, 0.0, &err) == MBP_ERR_INVALID && !err.empty(), "bad z pair");
    err.clear();
    CHECK(build(box, 8, N, N, -1.0, &err) == MBP_ERR_INVALID, "negative alpha");
    // a joined face with no partner
    Layout a;
    a.add(1, 1, 16, 16, 0.0, 1.0, 0.0, 1.0, C, D, N, N);
    err.clear();
    CHECK(build(a, 8, N, N, 0.0, &err) == MBP_ERR_INVALID && !err.empty(), "lonely connect");
    // partner faces that do not coincide (congruence)
    Layout b;
    b.add(1, 1, 16, 16, 0.0, 1.0, 0.0, 1.0, D, C, N, N);
    b.add(17, 1, 16, 16, 1.0, 2.0, 0.0, 1.0, C, D, N, N, 1.3);
    err.clear();
    CHECK(build(b, 8, N, N, 0.0, &err) == MBP_ERR_INVALID && !err.empty(), "non-congruent faces");
    // overlapping blocks
    Layout c;
    c.add(1, 1, 16, 16, 0.0, 1.0, 0.0, 1.0, D, D, N, N);
    c.add(9, 1, 16, 16, 0.5, 1.5, 0.0, 1.0, D, D, N, N);
    err.clear();
    CHECK(build(c, 8, N, N, 0.0, &err) == MBP_ERR_INVALID && !err.empty(), "overlap");
    // faces that do not increase
    Layout d;
    d.add(1, 1, 16, 16, 0.0, 1.0, 0.0, 1.0, D, D, N, N);
    d.xf[0][5] = d.xf[0][4];
    err.clear();
    CHECK(build(d, 8, N, N, 0.0, &err) == MBP_ERR_INVALID && !err.empty(), "flat faces");
    // an unknown condition code
    Layout e;
    e.add(1, 1, 16, 16, 0.0, 1.0, 0.0, 1.0, 9, D, N, N);
    err.clear();
    CHECK(build(e, 8, N, N, 0.0, &err) == MBP_ERR_INVALID && !err.empty(), "bad condition");
    // one periodic face without its opposite
    Layout g;
    g.add(1, 1, 16, 16, 0.0, 1.0, 0.0, 1.0, P, D, N, N);
    err.clear();
    CHECK(build(g, 8, N, N, 0.0, &err) == MBP_ERR_INVALID && !err.empty(), "half periodic");
    // zero blocks, null pointers
    mbp_synth_desc z{8, 1.0, N, N};
    mbp_options o;
    mbp::options_default(&o);
    mbp_plan Pl;
    err.clear();
    CHECK(mbp::build_plan_host_limits(nullptr, 0, &z, &o, 160 * 1024, &Pl, &err) == MBP_ERR_INVALID, "no blocks");
}

void eigen() {
    std::mt19937_64 rng(7);
    std::normal_distribution<double> nd;
    for (int n : {1, 2, 5, 17, 64}) {
        std::vector<double> A(size_t(n) * n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j <= i; ++j) A[size_t(i) * n + j] = A[size_t(j) * n + i] = nd(rng);
        const std::vector<double> A0 = A;
        std::vector<double> V, w;
        mbp::jacobi_eig(A, n, V, w);
        CHECK(int(w.size()) == n && V.size() == size_t(n) * n, "sizes n=%d", n);
        double scale = 0.0;
        for (double x : A0) scale = std::max(scale, std::fabs(x));
        // A v_k = w_k v_k and V^T V = I, with v_k = column k (V row-major n x n)
        for (int k = 0; k < n; ++k) {
            for (int i = 0; i < n; ++i) {
                double s = 0.0;
                for (int j = 0; j < n; ++j) s += A0[size_t(i) * n + j] * V[size_t(j) * n + k];
                CHECK(std::fabs(s - w[k] * V[size_t(i) * n + k]) <= 1e-10 * scale * n, "eigpair n=%d k=%d", n, k);
            }
            for (int l = 0; l < n; ++l) {
                double s = 0.0;
                for (int j = 0; j < n; ++j) s += V[size_t(j) * n + k] * V[size_t(j) * n + l];
                CHECK(std::fabs(s - (k == l ? 1.0 : 0.0)) <= 1e-10 * n, "orthonormal n=%d", n);
            }
        }
    }
}

void tanh_faces() {
    for (int type : {-1, 0, 1})
        for (double fac : {0.0, 0.5, 1.5, 3.0}) {
            std::vector<double> f(65);
            CHECK(mbp::grid_tanh(64, -1.0, 2.0, type, fac, f.data()) == MBP_OK, "tanh");
            CHECK(std::fabs(f[0] + 1.0) < 1e-14 && std::fabs(f[64] - 2.0) < 1e-14, "tanh ends");
            for (int i = 0; i < 64; ++i) CHECK(f[i + 1] > f[i], "tanh increasing");
        }
    std::vector<double> f(8);
    CHECK(mbp::grid_tanh(0, 0.0, 1.0, 0, 0.0, f.data()) == MBP_ERR_INVALID, "tanh n=0");
    CHECK(mbp::grid_tanh(4, 1.0, 1.0, 0, 0.0, f.data()) == MBP_ERR_INVALID, "tanh empty range");
    CHECK(mbp::grid_tanh(4, 0.0, 1.0, 5, 0.0, f.data()) == MBP_ERR_INVALID, "tanh type");
    CHECK(mbp::grid_tanh(4, 0.0, 1.0, 0, -1.0, f.data()) == MBP_ERR_INVALID, "tanh factor");
}

}  // namespace

int main() {
    valid_layouts();
    random_layouts();
    invalid_layouts();
    eigen();
    tanh_faces();
    std::printf("%s (%d failures)\n", failures ? "FAILED" : "OK", failures);
    return failures ? 1 : 0;
}
