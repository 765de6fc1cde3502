// Real-to-real transforms along the homogeneous z direction (Algorithm 1,
// first and last loops; Table 1 kinds).  Every kind is reduced to one
// complex FFT of length m = n/2 per z column:
//   periodic  -> discrete Hartley transform from the half-length real DFT;
//   N-N       -> DCT-II by Makhoul's even/odd reordering (inverse DCT-III);
//   D-D       -> DST-II as the DCT-II of (-1)^j x read backwards (DST-III);
//   N-D       -> DCT-IV with the quarter-wave pre/post twiddles (self-inverse);
//   D-N       -> DST-IV as (-1)^q DCT-IV of x reversed (self-inverse).
// All transforms are orthonormal.  The complex FFT is a mixed-radix Stockham
// autosort held in LDS; a workgroup transforms W neighbouring columns, whose
// z rows are read and written as contiguous W-element segments.
#include <algorithm>

#include "internal.h"

namespace mbp {

struct FFTArgs {
    int n, m, kind, W, cs;
    int nstage;
    int radix[16];
    const double* tw;     // e^{-2 pi i t / m}, t < m
    const double* twn;    // e^{-2 pi i k / n}, k <= m
    const double* post;   // e^{-i pi k / (2n)}, k <= n
    const double* pre4;   // e^{-i pi (4k+1) / (4n)}, k < m
    const double* post4;  // e^{-i pi k / n}, k < m
};

struct FTile {
    long long in_base, out_base;  // element offsets of column 0 of the tile
    int in_stride, out_stride;    // distance between consecutive z rows
    int ncol;                     // valid columns (<= W)
    int pad;
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
// The transform tables are never written while a kernel runs: reading them
// through the constant address space marks the loads invariant, so they may
// move ahead of the stores of earlier results and stay in flight together.
typedef __attribute__((address_space(4))) const double ctab_t;
__device__ __forceinline__ double2 ld2(const double* t, int k) {
    const ctab_t* c = (const ctab_t*)t;
    return make_double2(c[2 * k], c[2 * k + 1]);
}

// Where a transform reads its tables: straight from device memory (through
// the constant address space), or from a copy in LDS.
struct GlobalTab {
    const double* t;
    __device__ __forceinline__ double2 operator()(int k) const { return ld2(t, k); }
};
struct LdsTab {
    const double2* t;
    __device__ __forceinline__ double2 operator()(int k) const { return t[k]; }
};

// a / b for 0 <= a < 2^22 and 1 <= b < 2^12, from the float reciprocal rb of
// b: the float quotient is within one of the true one, and the remainder
// test corrects it.
__device__ __forceinline__ int div_small(int a, int b, float rb) {
    int q = int(float(a) * rb);
    const int r = a - q * b;
    if (r < 0) --q;
    else if (r >= b) ++q;
    return q;
}

// cos and sin of 2 pi t / R for the odd radices with closed-form butterflies
template <int R>
struct Roots;
template <>
struct Roots<3> {
    static constexpr double c[3] = {1.0, -0.5, -0.5};
    static constexpr double s[3] = {0.0, 0.86602540378443864676, -0.86602540378443864676};
};
template <>
struct Roots<5> {
    static constexpr double c[5] = {1.0, 0.30901699437494742410, -0.80901699437494742410,
                                    -0.80901699437494742410, 0.30901699437494742410};
    static constexpr double s[5] = {0.0, 0.95105651629515357212, 0.58778525229247312917,
                                    -0.58778525229247312917, -0.95105651629515357212};
};
template <>
struct Roots<7> {
    static constexpr double c[7] = {1.0, 0.62348980185873353053, -0.22252093395631440429,
                                    -0.90096886790241912624, -0.90096886790241912624,
                                    -0.22252093395631440429, 0.62348980185873353053};
    static constexpr double s[7] = {0.0, 0.78183148246802980871, 0.97492791218182360702,
                                    0.43388373911755812048, -0.43388373911755812048,
                                    -0.97492791218182360702, -0.78183148246802980871};
};

// XCD-aware mapping: workgroups are dispatched round-robin over the 8 XCDs;
// give each XCD one contiguous range of tiles so neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_remap(int g, int n) {
    int x = g & 7, l = g >> 3;
    int per = n >> 3, rem = n & 7;
    return x * per + min(x, rem) + l;
}

// DFT of length R of v[0..R-1] in place, forward sign e^{-2 pi i rs/R}.
// Radices 2, 4 and 8 use their closed-form roots; odd radices read the roots
// tw[(r s mod R) m / R] from the twiddle table.
template <int R, typename TW>
__device__ __forceinline__ void dft(double2* v, const TW& tw, int m) {
    if constexpr (R == 2) {
        const double2 a = v[0], b = v[1];
        v[0] = make_double2(a.x + b.x, a.y + b.y);
        v[1] = make_double2(a.x - b.x, a.y - b.y);
    } else if constexpr (R == 4) {
        const double2 s02 = make_double2(v[0].x + v[2].x, v[0].y + v[2].y);
        const double2 d02 = make_double2(v[0].x - v[2].x, v[0].y - v[2].y);
        const double2 s13 = make_double2(v[1].x + v[3].x, v[1].y + v[3].y);
        const double2 d13 = make_double2(v[1].x - v[3].x, v[1].y - v[3].y);
        v[0] = make_double2(s02.x + s13.x, s02.y + s13.y);
        v[2] = make_double2(s02.x - s13.x, s02.y - s13.y);
        v[1] = make_double2(d02.x + d13.y, d02.y - d13.x);  // d02 - i d13
        v[3] = make_double2(d02.x - d13.y, d02.y + d13.x);  // d02 + i d13
    } else if constexpr (R == 8) {
        // two length-4 DFTs of the even / odd samples, then the radix-2 step
        // with the eighth roots e^{-i pi s / 4}
        double2 e[4] = {v[0], v[2], v[4], v[6]};
        double2 o[4] = {v[1], v[3], v[5], v[7]};
        dft<4>(e, tw, m);
        dft<4>(o, tw, m);
        const double h = 0.70710678118654752440;
        const double2 w1 = make_double2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));   // e^{-i pi/4} o1
        const double2 w2 = make_double2(o[2].y, -o[2].x);                                // -i o2
        const double2 w3 = make_double2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));  // e^{-3i pi/4} o3
        v[0] = make_double2(e[0].x + o[0].x, e[0].y + o[0].y);
        v[4] = make_double2(e[0].x - o[0].x, e[0].y - o[0].y);
        v[1] = make_double2(e[1].x + w1.x, e[1].y + w1.y);
        v[5] = make_double2(e[1].x - w1.x, e[1].y - w1.y);
        v[2] = make_double2(e[2].x + w2.x, e[2].y + w2.y);
        v[6] = make_double2(e[2].x - w2.x, e[2].y - w2.y);
        v[3] = make_double2(e[3].x + w3.x, e[3].y + w3.y);
        v[7] = make_double2(e[3].x - w3.x, e[3].y - w3.y);
    } else if constexpr (R == 3 || R == 5 || R == 7) {
        // pairs r, R - r: v_r w^{rs} + v_{R-r} w^{-rs} = a_r cos - i b_r sin
        // with a_r = v_r + v_{R-r}, b_r = v_r - v_{R-r}, w = e^{-2 pi i / R}
        constexpr int H = (R - 1) / 2;
        double2 a[H], b[H];
        double2 y0 = v[0];
#pragma unroll
        for (int r = 1; r <= H; ++r) {
            a[r - 1] = make_double2(v[r].x + v[R - r].x, v[r].y + v[R - r].y);
            b[r - 1] = make_double2(v[r].x - v[R - r].x, v[r].y - v[R - r].y);
            y0.x += a[r - 1].x;
            y0.y += a[r - 1].y;
        }
        double2 y[R];
        y[0] = y0;
#pragma unroll
        for (int s = 1; s <= H; ++s) {
            double2 re = v[0], im = make_double2(0.0, 0.0);
#pragma unroll
            for (int r = 1; r <= H; ++r) {
                const double c = Roots<R>::c[(r * s) % R], sn = Roots<R>::s[(r * s) % R];
                re.x += c * a[r - 1].x;
                re.y += c * a[r - 1].y;
                im.x += sn * b[r - 1].x;
                im.y += sn * b[r - 1].y;
            }
            y[s] = make_double2(re.x + im.y, re.y - im.x);      // re - i im
            y[R - s] = make_double2(re.x - im.y, re.y + im.x);  // re + i im
        }
#pragma unroll
        for (int s = 0; s < R; ++s) v[s] = y[s];
    } else {
        double2 y[R];
#pragma unroll
        for (int s = 0; s < R; ++s) {
            double2 acc = v[0];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const double2 rt = tw(((r * s) % R) * (m / R));
                const double2 pr = cmul(v[r], rt);
                acc.x += pr.x;
                acc.y += pr.y;
            }
            y[s] = acc;
        }
#pragma unroll
        for (int s = 0; s < R; ++s) v[s] = y[s];
    }
}

// One Stockham stage of radix R over W columns held column-major in LDS
// (column stride cs complex values).  Reads all inputs into registers before
// a barrier, then writes the outputs, so the stage runs in place.
template <int R, int BPT, typename TW>
__device__ void stage(double2* z, int cs, int m, int W, int Ns, const TW& tw, int tid, int nthr) {
    const int nbf = m / R;
    const int total = W * nbf;
    const int step = m / (Ns * R);  // twiddle index stride
    const float r_nbf = 1.0f / float(nbf), r_ns = 1.0f / float(Ns);
    double2 v[BPT][R];
    int dst[BPT];
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
        const int b = tid + t * nthr;
        dst[t] = -1;
        if (b < total) {
            const int w = div_small(b, nbf, r_nbf), j = b - w * nbf;
            const int jn = div_small(j, Ns, r_ns), k = j - jn * Ns;
            const double2* col = z + w * cs;
            // every twiddle is read unconditionally (k = 0 reads the exact
            // root 1), so all of the loads are in flight together;
            // k r step < Ns R step = m: the index needs no wrap
            double2 rt[R];
#pragma unroll
            for (int r = 1; r < R; ++r) rt[r] = tw(k * r * step);
            v[t][0] = col[j];
#pragma unroll
            for (int r = 1; r < R; ++r) v[t][r] = cmul(col[j + r * nbf], rt[r]);
            dft<R>(v[t], tw, m);
            dst[t] = w * cs + jn * Ns * R + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
        if (dst[t] < 0) continue;
#pragma unroll
        for (int r = 0; r < R; ++r) z[dst[t] + r * Ns] = v[t][r];
    }
    __syncthreads();
}

// One Stockham stage of any radix R (a prime above 31, for which no
// unrolled butterfly exists): each output of butterfly (j = jn Ns + k) is
// y_s = sum_r z[j + r m/R] w^{r (k + s Ns) m / (Ns R)}, w = e^{-2 pi i / m},
// computed straight from LDS (R complex products per output).  The host
// keeps W m <= MAXOUT * blockDim.x.
template <int MAXOUT, typename TW>
__device__ void stage_generic(double2* z, int cs, int m, int W, int Ns, int R, const TW& tw) {
    const int nbf = m / R;
    const int step = m / (Ns * R);
    const int total = W * m;
    double2 y[MAXOUT];
    int dst[MAXOUT];
#pragma unroll
    for (int t = 0; t < MAXOUT; ++t) {
        const int o = threadIdx.x + t * blockDim.x;
        dst[t] = -1;
        if (o >= total) continue;
        const int w = o / m, rest = o - w * m;
        const int s = rest / nbf, j = rest - s * nbf;
        const int jn = j / Ns, k = j - jn * Ns;
        const double2* col = z + w * cs;
        const int inc = int(((long long)(k + s * Ns) * step) % m);
        int ti = 0;
        double2 acc = make_double2(0.0, 0.0);
        for (int r = 0; r < R; ++r) {
            const double2 pr = cmul(col[j + r * nbf], tw(ti));
            acc.x += pr.x;
            acc.y += pr.y;
            ti += inc;
            if (ti >= m) ti -= m;
        }
        y[t] = acc;
        dst[t] = w * cs + jn * Ns * R + k + s * Ns;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < MAXOUT; ++t)
        if (dst[t] >= 0) z[dst[t]] = y[t];
    __syncthreads();
}

constexpr int kGenericOut = 16;  // outputs per thread of the any-radix stage

template <int R, typename TW>
__device__ void stage_dispatch(double2* z, int cs, int m, int W, int Ns, const TW& tw) {
    const int total = W * (m / R);
    const int bpt = (total + blockDim.x - 1) / blockDim.x;
    if constexpr (R > 8) {
        stage<R, 1>(z, cs, m, W, Ns, tw, threadIdx.x, blockDim.x);  // the host keeps W * m / R <= 256 here
    } else {
        // the host keeps bpt <= 16 / R for R = 2 and 4, bpt <= 2 otherwise
        if (bpt <= 1) stage<R, 1>(z, cs, m, W, Ns, tw, threadIdx.x, blockDim.x);
        else if (bpt <= 2) stage<R, 2>(z, cs, m, W, Ns, tw, threadIdx.x, blockDim.x);
        else if constexpr (R == 2 || R == 4) {
            if (bpt <= 4) stage<R, 4>(z, cs, m, W, Ns, tw, threadIdx.x, blockDim.x);
            else if constexpr (R == 2) stage<R, 8>(z, cs, m, W, Ns, tw, threadIdx.x, blockDim.x);
        }
    }
}

// Radix classes: 0 = powers of two only, 1 = with 3 / 5 / 7, 2 = any prime
// up to 31, 3 = also primes above 31 (the any-radix stage).  Each class is
// its own kernel so the power-of-two transforms do not carry the register
// footprint of the long odd butterflies.
template <int CLASS, typename TW>
__device__ void fft_columns(double2* z, int cs, const FFTArgs& a, const TW& tw) {
    int Ns = 1;
    for (int s = 0; s < a.nstage; ++s) {
        const int R = a.radix[s];
        switch (R) {
            case 2: stage_dispatch<2>(z, cs, a.m, a.W, Ns, tw); break;
            case 4: stage_dispatch<4>(z, cs, a.m, a.W, Ns, tw); break;
            case 8: stage_dispatch<8>(z, cs, a.m, a.W, Ns, tw); break;
            default:
                if constexpr (CLASS >= 1) {
                    switch (R) {
                        case 3: stage_dispatch<3>(z, cs, a.m, a.W, Ns, tw); break;
                        case 5: stage_dispatch<5>(z, cs, a.m, a.W, Ns, tw); break;
                        case 7: stage_dispatch<7>(z, cs, a.m, a.W, Ns, tw); break;
                        default:
                            if constexpr (CLASS >= 2) {
                                switch (R) {
                                    case 11: stage_dispatch<11>(z, cs, a.m, a.W, Ns, tw); break;
                                    case 13: stage_dispatch<13>(z, cs, a.m, a.W, Ns, tw); break;
                                    case 17: stage_dispatch<17>(z, cs, a.m, a.W, Ns, tw); break;
                                    case 19: stage_dispatch<19>(z, cs, a.m, a.W, Ns, tw); break;
                                    case 23: stage_dispatch<23>(z, cs, a.m, a.W, Ns, tw); break;
                                    case 29: stage_dispatch<29>(z, cs, a.m, a.W, Ns, tw); break;
                                    case 31: stage_dispatch<31>(z, cs, a.m, a.W, Ns, tw); break;
                                    default:
                                        if constexpr (CLASS >= 3)
                                            stage_generic<kGenericOut>(z, cs, a.m, a.W, Ns, R, tw);
                                        break;
                                }
                            }
                            break;
                    }
                }
                break;
        }
        Ns *= R;
    }
}

constexpr int kLoadBatch = 8;   // input elements per thread in flight together
constexpr int kStoreBatch = 4;  // output elements per thread whose table reads go together
constexpr int kInvBatch = 2;    // inverse cosine kinds: elements per thread read together

// Forward (dir = 0) or inverse (dir = 1) transform of W columns per workgroup.
template <int CLASS>
__global__ void __launch_bounds__(256) k_r2r(FFTArgs a, const FTile* __restrict__ tiles, int ntiles,
                                             int dir, const double* __restrict__ in,
                                             double* __restrict__ out, int* nonfinite) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    double2* z = reinterpret_cast<double2*>(lds_raw);
    const int tix = xcd_remap(blockIdx.x, ntiles);
    const FTile T = tiles[tix];
    const int n = a.n, m = a.m, W = a.W, cs = a.cs;
    const int lw = __ffs(W) - 1;  // W is a power of two
    const int kind = a.kind;
    const double sc2 = sqrt(2.0 / n), sc1 = sqrt(1.0 / n);
    // which algorithm runs: forward kinds, and the inverse of N-N / D-D
    const bool inv_cos = dir == 1 && (kind == Z_NN || kind == Z_DD);

    // ---------------- load + pre-processing ----------------
    if (!inv_cos) {
        bool bad = false;
        // kLoadBatch elements per thread are loaded before any is used, so
        // their loads are in flight together.  Every load is unconditional:
        // elements past the end repeat the last one, columns past the tile's
        // last read that one and are zeroed.
        for (int base = 0; base < n * W; base += kLoadBatch * blockDim.x) {
            double xs[kLoadBatch];
#pragma unroll
            for (int b = 0; b < kLoadBatch; ++b) {
                const int idx = min(base + b * int(blockDim.x) + int(threadIdx.x), n * W - 1);
                const int k = idx >> lw, w = idx & (W - 1);
                xs[b] = in[T.in_base + (long long)k * T.in_stride + min(w, T.ncol - 1)];
            }
#pragma unroll
            for (int b = 0; b < kLoadBatch; ++b) {
            const int idx = min(base + b * int(blockDim.x) + int(threadIdx.x), n * W - 1);
            const int k = idx >> lw, w = idx & (W - 1);
            double x = w >= T.ncol ? 0.0 : xs[b];
            if (!isfinite(x)) bad = true;
            double* zc = reinterpret_cast<double*>(z + w * cs);
            // position u in the length-n real sequence fed to the FFT, chosen
            // without branches: PP keeps k; NN / DD take Makhoul's even / odd
            // reordering (DD with alternating signs); ND packs for the DCT-IV,
            // DN packs the reversed input j = n - 1 - k the same way
            const int uc = (k & 1) ? n - 1 - (k >> 1) : (k >> 1);
            const int kk = kind == Z_DN ? n - 1 - k : k;
            const int u4 = (kk & 1) ? ((n - 1 - kk) >> 1) * 2 + 1 : (kk >> 1) * 2;
            const int u = kind == Z_PP ? k : (kind == Z_NN || kind == Z_DD) ? uc : u4;
            x = (kind == Z_DD && (k & 1)) ? -x : x;
            zc[u] = x;  // real part at even u, imaginary part at odd u
            }
        }
        if (bad && nonfinite) atomicOr(nonfinite, 1);
        __syncthreads();
        if (kind == Z_ND || kind == Z_DN) {
            const float rm = 1.0f / float(m);
            for (int idx = threadIdx.x; idx < m * W; idx += blockDim.x) {
                int w = div_small(idx, m, rm), k = idx - w * m;
                z[w * cs + k] = cmul(z[w * cs + k], ld2(a.pre4, k));
            }
            __syncthreads();
        }
    } else {
        // inverse of the cosine kinds: V_q = e^{i pi q/(2n)} (y'_q - i y'_{n-q}),
        // Z_k = (V_k + conj V_{m-k}) + i (V_k - conj V_{m-k}) e^{2 pi i k/n};
        // the FFT below then computes conj(IFFT) of conj(Z).
        const int half = m / 2;
        for (int base = 0; base < (half + 1) * W; base += kInvBatch * blockDim.x) {
            // y'_q = y_q / c_q at q = k, n-k, m-k, m+k (y'_n = 0), and the
            // table values, read for kInvBatch elements before any is used
            double yv[kInvBatch][4];
            double2 pk[kInvBatch], pmk[kInvBatch], tk[kInvBatch], tmk[kInvBatch];
#pragma unroll
            for (int b = 0; b < kInvBatch; ++b) {
                const int idx = min(base + b * int(blockDim.x) + int(threadIdx.x), (half + 1) * W - 1);
                const int k = idx >> lw, w = idx & (W - 1);
                const int qs[4] = {k, n - k, m - k, m + k};
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int qc = min(qs[v], n - 1);
                    const int row = kind == Z_DD ? n - 1 - qc : qc;
                    yv[b][v] = in[T.in_base + (long long)row * T.in_stride + min(w, T.ncol - 1)];
                }
                pk[b] = ld2(a.post, k);
                pmk[b] = ld2(a.post, m - k);
                tk[b] = ld2(a.twn, k);
                tmk[b] = ld2(a.twn, m - k);
            }
#pragma unroll
            for (int b = 0; b < kInvBatch; ++b) {
                const int idx = min(base + b * int(blockDim.x) + int(threadIdx.x), (half + 1) * W - 1);
                const int k = idx >> lw, w = idx & (W - 1);
                const bool colok = w < T.ncol;
                const int qs[4] = {k, n - k, m - k, m + k};
                double y[4];
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    y[v] = (qs[v] < n && colok) ? yv[b][v] / (qs[v] == 0 ? sc1 : sc2) : 0.0;
                // V_q = e^{i pi q/(2n)} (y'_q - i y'_{n-q}) for q = k and m - k
                const double2 Vk = cmul(cconj(pk[b]), make_double2(y[0], -y[1]));
                const double2 Vmk = cmul(cconj(pmk[b]), make_double2(y[2], -y[3]));
                // Z_kk = (A + conj B) + i (A - conj B) e^{2 pi i kk / n}
                {
                    const double2 Bc = cconj(Vmk);
                    const double2 s = make_double2(Vk.x + Bc.x, Vk.y + Bc.y);
                    const double2 d = make_double2(Vk.x - Bc.x, Vk.y - Bc.y);
                    const double2 id = cmul(make_double2(-d.y, d.x), cconj(tk[b]));
                    if (k < m) z[w * cs + k] = cconj(make_double2(s.x + id.x, s.y + id.y));
                }
                if (k > 0 && m - k != k && m - k < m) {
                    const double2 Bc = cconj(Vk);
                    const double2 s = make_double2(Vmk.x + Bc.x, Vmk.y + Bc.y);
                    const double2 d = make_double2(Vmk.x - Bc.x, Vmk.y - Bc.y);
                    const double2 id = cmul(make_double2(-d.y, d.x), cconj(tmk[b]));
                    z[w * cs + (m - k)] = cconj(make_double2(s.x + id.x, s.y + id.y));
                }
            }
        }
        __syncthreads();
    }

    // ---------------- complex FFT of length m ----------------
    fft_columns<CLASS>(z, cs, a, GlobalTab{a.tw});

    // ---------------- post-processing + store ----------------
    if (inv_cos) {
        const double inv_n = 1.0 / n;
#pragma unroll 8
        for (int base = 0; base < n * W; base += blockDim.x) {
            const int idx = min(base + int(threadIdx.x), n * W - 1);
            // lanes past the tile's last column redo that column and store
            // the same value to the same place: no branch around the store
            int j = idx >> lw, w = min(idx & (W - 1), T.ncol - 1);
            int u = (j & 1) ? n - 1 - (j >> 1) : (j >> 1);
            double2 Fz = z[w * cs + (u >> 1)];
            double v = (u & 1) ? -Fz.y * inv_n : Fz.x * inv_n;
            if (kind == Z_DD && (j & 1)) v = -v;
            out[T.out_base + (long long)j * T.out_stride + w] = v;
        }
        return;
    }
    if (kind == Z_ND || kind == Z_DN) {
        for (int base = 0; base < m * W; base += kStoreBatch * blockDim.x) {
            double2 zv[kStoreBatch], tv[kStoreBatch];
#pragma unroll
            for (int b = 0; b < kStoreBatch; ++b) {
                const int idx = min(base + b * int(blockDim.x) + int(threadIdx.x), m * W - 1);
                const int k = idx >> lw, w = min(idx & (W - 1), T.ncol - 1);
                zv[b] = z[w * cs + k];
                tv[b] = ld2(a.post4, k);
            }
#pragma unroll
            for (int b = 0; b < kStoreBatch; ++b) {
            const int idx = min(base + b * int(blockDim.x) + int(threadIdx.x), m * W - 1);
            const int k = idx >> lw, w = min(idx & (W - 1), T.ncol - 1);
            double2 u = cmul(zv[b], tv[b]);
            int q0 = 2 * k, q1 = n - 1 - 2 * k;
            double y0 = sc2 * u.x, y1 = -sc2 * u.y;
            if (kind == Z_DN) {
                if (q0 & 1) y0 = -y0;
                if (q1 & 1) y1 = -y1;
            }
            out[T.out_base + (long long)q0 * T.out_stride + w] = y0;
            out[T.out_base + (long long)q1 * T.out_stride + w] = y1;
            }
        }
        return;
    }
    // PP / NN / DD: real DFT X_k (k = 0..m) from the half-length FFT
    for (int base = 0; base < (m + 1) * W; base += kStoreBatch * blockDim.x) {
        double2 tks[kStoreBatch], pks[kStoreBatch], pns[kStoreBatch];
#pragma unroll
        for (int b = 0; b < kStoreBatch; ++b) {
            const int k = min(base + b * int(blockDim.x) + int(threadIdx.x), (m + 1) * W - 1) >> lw;
            tks[b] = ld2(a.twn, k);
            pks[b] = ld2(a.post, k);
            pns[b] = ld2(a.post, n - k);
        }
#pragma unroll
        for (int b = 0; b < kStoreBatch; ++b) {
        const int idx = min(base + b * int(blockDim.x) + int(threadIdx.x), (m + 1) * W - 1);
        int k = idx >> lw, w = min(idx & (W - 1), T.ncol - 1);
        const double2 tk = tks[b], pk = pks[b], pn = pns[b];
        double2 Zk = z[w * cs + (k == m ? 0 : k)];
        double2 Zc = cconj(z[w * cs + (k == 0 ? 0 : m - k)]);
        double2 s = make_double2(0.5 * (Zk.x + Zc.x), 0.5 * (Zk.y + Zc.y));
        double2 d = make_double2(0.5 * (Zk.x - Zc.x), 0.5 * (Zk.y - Zc.y));
        double2 t = cmul(tk, d);  // e^{-2 pi i k/n} (Zk - Zc) / 2
        double2 X = make_double2(s.x + t.y, s.y - t.x);  // s - i t
        // PP: Hartley values at k and n - k; NN / DD: DCT-II
        // y_q = c_q Re(e^{-i pi q/(2n)} X_q) at q = k and n - k (X_{n-k} = conj X_k),
        // DD written in reversed order.  k = 0 and k = m have no partner: the
        // second store repeats the first.  Selects, not branches, so that the
        // loop body is one block.
        const bool pp = kind == Z_PP, dd = kind == Z_DD, pair = k > 0 && k < m;
        const double yk = pp ? sc1 * (X.x - X.y) : (k == 0 ? sc1 : sc2) * (pk.x * X.x - pk.y * X.y);
        const double yn = pp ? sc1 * (X.x + X.y) : sc2 * (pn.x * X.x + pn.y * X.y);
        const int rk = dd ? n - 1 - k : k;
        const int rn = pp ? n - k : dd ? k - 1 : n - k;
        double* o = out + T.out_base + w;
        const long long st = T.out_stride;
        o[rk * st] = yk;
        o[(pair ? rn : rk) * st] = pair ? yn : yk;
        }
    }
}

// ---------------------------------------------------------------------------
// Streaming form of the same transforms, for long power-of-two half lengths
// (m >= 128).  A workgroup loops over tiles of W >= 16 columns (z rows read
// and written as segments of 128 B or more), and the next tile's input is
// loaded into registers, kStreamPer values per thread, while the current
// tile is transformed and stored: the loads stay in flight through the LDS
// phases.  Every table the loop reads is copied to LDS once per workgroup,
// because a load from device memory issued after the prefetch would have to
// wait for it.  The host sets NT = n W / kStreamPer, so every loop below has
// a fixed trip count.
constexpr int kStreamPer = 16;

// v, hidden from the optimiser: index arithmetic built on it is redone in
// each phase of the tile loop instead of being hoisted out of the loop or
// shared between phases, which would hold it in registers throughout.
__device__ __forceinline__ int fresh(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Raw row of real position p of the sequence the forward FFT takes (the
// inverse of the placement in k_r2r): PP keeps p; N-N / D-D undo Makhoul's
// even / odd reordering; N-D undoes the quarter-wave packing, D-N that of the
// reversed input.
__device__ __forceinline__ int fwd_row(int kind, int n, int p) {
    if (kind == Z_PP) return p;
    if (kind == Z_NN || kind == Z_DD) return p < n / 2 ? 2 * p : 2 * (n - 1 - p) + 1;
    const int kk = (p & 1) ? n - p : p;
    return kind == Z_DN ? n - 1 - kk : kk;
}

// The thread's 16 inputs of a tile, gathered so that the first FFT stage
// runs in registers.  Lanes run over the W columns first (tid mod W), so
// every load of a wave reads whole row segments.
//   Forward PP, N-D, D-N: the thread owns first-stage butterfly j = tid / W
//   of its column, whose inputs are the complex values u = j + r m / 8,
//   r < 8, each two real positions 2u, 2u + 1 (element 2r + parity).
//   Forward N-N, D-D: element e is row e NT / W + tid / W.
//   Inverse cosine kinds: for each of the thread's four groups (k, w) (group
//   index g NT + tid, k < m / 2), the rows that Z_k and Z_{m-k} need, y at k,
//   n - k, m - k, m + k (group 0: 0, m, m / 2, 3 m / 2, for Z_0 and Z_{m/2});
//   rows count in the stored order, reversed for D-D.
template <int NT>
__device__ __forceinline__ void stream_load(double (&r)[kStreamPer], const double* __restrict__ in, const FTile& T,
                                            int lw, int W, int n, int kind, bool inv_cos) {
    const int tid = fresh(threadIdx.x);
    // columns past the tile's last read that one (discarded later)
    const int col = min(tid & (W - 1), T.ncol - 1);
    const int m = n / 2;
    const double* base = in + T.in_base + col;
    if (!inv_cos && (kind == Z_NN || kind == Z_DD)) {
        // N-N / D-D forward: plain rows e NT / W + tid / W (consecutive rows
        // in a wave; the gathered order reads rows four apart, which measured
        // slower), placed in the FFT's input order through LDS
        const int lane = (tid >> lw) * T.in_stride + col;
        const long long step = (long long)(NT >> lw) * T.in_stride;
#pragma unroll
        for (int e = 0; e < kStreamPer; ++e) r[e] = (in + T.in_base + e * step)[lane];
        return;
    }
    if (!inv_cos) {
        const int j = tid >> lw, nbf = m / 8;
#pragma unroll
        for (int e = 0; e < kStreamPer; ++e) {
            const int p = 2 * (j + (e >> 1) * nbf) + (e & 1);
            r[e] = base[(long long)fwd_row(kind, n, p) * T.in_stride];
        }
        return;
    }
    const bool rev = kind == Z_DD;
#pragma unroll
    for (int g = 0; g < kStreamPer / 4; ++g) {
        const int k = (g * NT + tid) >> lw;
        const int q[4] = {k, k == 0 ? m : n - k, k == 0 ? m / 2 : m - k, k == 0 ? m + m / 2 : m + k};
#pragma unroll
        for (int v = 0; v < 4; ++v) r[4 * g + v] = base[(long long)(rev ? n - 1 - q[v] : q[v]) * T.in_stride];
    }
}

// One Stockham stage of the streaming form (the same arithmetic as stage):
// BPT = 8 / R butterflies per thread, consecutive lanes on consecutive
// columns, so that the column stride (an odd number of complex values) spreads
// every access of a wave over the LDS banks whatever the stage's output
// stride.  The roots w^r of a butterfly are powers of one table value
// (w^2 = w w, w^3 = w^2 w, ...; a few units in the last place), and the first
// stage (Ns = 1) needs none.
template <int R, int BPT, int NT>
__device__ void stream_stage(double2* z, int cs, int m, int lw, int Ns, const double2* __restrict__ tw) {
    const int nbf = m / R;
    const int step = m / (Ns * R);
    const int tid = fresh(threadIdx.x);
    double2 v[BPT][R];
    int dst[BPT];
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
        const int b = tid + t * NT;
        const int w = b & ((1 << lw) - 1), j = b >> lw;
        const int jn = j >> (__ffs(Ns) - 1), k = j & (Ns - 1);  // Ns is a power of two
        const double2* col = z + w * cs;
#pragma unroll
        for (int r = 0; r < R; ++r) v[t][r] = col[j + r * nbf];
        if (Ns > 1) {
            const double2 w1 = tw[k * step];
            double2 wr = w1;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                v[t][r] = cmul(v[t][r], wr);
                if (r + 1 < R) wr = cmul(wr, w1);
            }
        }
        dft<R>(v[t], GlobalTab{nullptr}, m);
        dst[t] = w * cs + jn * Ns * R + k;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
#pragma unroll
        for (int r = 0; r < R; ++r) z[dst[t] + r * Ns] = v[t][r];
    }
    __syncthreads();
}

// The Stockham stages of the streaming form: n W = kStreamPer NT gives every
// thread 8 / R butterflies of each radix R.
template <int NT>
__device__ void fft_stream_columns(double2* z, int cs, const FFTArgs& a, const double2* tw, int first) {
    const int lw = __ffs(a.W) - 1;
    int Ns = 1;
    for (int s = 0; s < first; ++s) Ns *= a.radix[s];
    for (int s = first; s < a.nstage; ++s) {
        const int R = a.radix[s];
        if (R == 8) stream_stage<8, 1, NT>(z, cs, a.m, lw, Ns, tw);
        else if (R == 4) stream_stage<4, 2, NT>(z, cs, a.m, lw, Ns, tw);
        else stream_stage<2, 4, NT>(z, cs, a.m, lw, Ns, tw);
        Ns *= R;
    }
}

template <int NT>
__global__ void __launch_bounds__(NT) k_r2r_stream(FFTArgs a, const FTile* __restrict__ tiles, int ntiles, int dir,
                                                   const double* __restrict__ in, double* __restrict__ out,
                                                   int* nonfinite) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    double2* z = reinterpret_cast<double2*>(lds_raw);
    const int n = a.n, m = a.m, W = a.W, cs = a.cs;
    const int lw = __ffs(W) - 1;
    const int kind = a.kind;
    const double sc2 = sqrt(2.0 / n), sc1 = sqrt(1.0 / n);
    const double isc2 = sqrt(0.5 * n), isc1 = sqrt(double(n));
    const bool inv_cos = dir == 1 && (kind == Z_NN || kind == Z_DD);
    const bool quarter = kind == Z_ND || kind == Z_DN;
    const bool cosine = !inv_cos && (kind == Z_NN || kind == Z_DD);  // forward N-N / D-D
    // tables behind the W-column image: tw (m values), then twn (m + 1) and
    // post (m + 1; the bins above m use post[n - k] = -i conj(post[k])), or
    // for the quarter-wave kinds pre4 (m) and post4 (m)
    double2* twl = z + W * cs;
    double2* t1 = twl + m;
    double2* t2 = t1 + m + 1;
    for (int i = threadIdx.x; i < m; i += NT) twl[i] = ld2(a.tw, i);
    if (quarter) {
        for (int i = threadIdx.x; i < m; i += NT) {
            t1[i] = ld2(a.pre4, i);
            t2[i] = ld2(a.post4, i);
        }
    } else {
        for (int i = threadIdx.x; i <= m; i += NT) {
            t1[i] = ld2(a.twn, i);
            t2[i] = ld2(a.post, i);
        }
    }
    __syncthreads();  // the first tile's placement already reads the tables

    const int G = gridDim.x;
    int v = blockIdx.x;
    FTile T = tiles[xcd_remap(v, ntiles)];
    double r[kStreamPer];
    stream_load<NT>(r, in, T, lw, W, n, kind, inv_cos);
    bool bad = false;
    for (;;) {
        // ---- this tile's input, registers -> LDS: the inverse cosine kinds
        //      as Z_k (as in k_r2r) made from the gathered values; forward N-N
        //      and D-D in the order the FFT takes (as in k_r2r); the other
        //      forward kinds through the first FFT stage
        int tid = fresh(threadIdx.x);
        if (inv_cos) {
            const int w = tid & (W - 1);
            const bool colok = w < T.ncol;
            const int half = m / 2;
#pragma unroll
            for (int g = 0; g < kStreamPer / 4; ++g) {
                const int k = (g * NT + tid) >> lw;
                // y'_q = y_q / c_q of the four gathered rows
                const double y0 = colok ? r[4 * g] * (k == 0 ? isc1 : isc2) : 0.0;
                const double y1 = colok ? r[4 * g + 1] * isc2 : 0.0;
                const double y2 = colok ? r[4 * g + 2] * isc2 : 0.0;
                const double y3 = colok ? r[4 * g + 3] * isc2 : 0.0;
                // V_q = e^{i pi q/(2n)} (y'_q - i y'_{n-q});
                // Z_q = conj((A + conj B) + i (A - conj B) e^{2 pi i q/n}), A = V_q, B = V_{m-q}
                auto Z = [&](double2 A, double2 B, int q) -> double2 {
                    const double2 Bc = cconj(B);
                    const double2 sm = make_double2(A.x + Bc.x, A.y + Bc.y);
                    const double2 d = make_double2(A.x - Bc.x, A.y - Bc.y);
                    const double2 id = cmul(make_double2(-d.y, d.x), cconj(t1[q]));
                    return cconj(make_double2(sm.x + id.x, sm.y + id.y));
                };
                double2* zc = z + w * cs;
                if (k > 0) {
                    const double2 A = cmul(cconj(t2[k]), make_double2(y0, -y1));       // V_k
                    const double2 B = cmul(cconj(t2[m - k]), make_double2(y2, -y3));   // V_{m-k}
                    zc[k] = Z(A, B, k);
                    zc[m - k] = Z(B, A, m - k);
                } else {
                    const double2 A = cmul(cconj(t2[0]), make_double2(y0, 0.0));      // V_0
                    const double2 B = cmul(cconj(t2[m]), make_double2(y1, -y1));      // V_m
                    const double2 H = cmul(cconj(t2[half]), make_double2(y2, -y3));   // V_{m/2}
                    zc[0] = Z(A, B, 0);
                    zc[half] = Z(H, H, half);
                }
            }
        } else if (cosine) {
#pragma unroll
            for (int e = 0; e < kStreamPer; ++e) {
                const int idx = e * NT + tid;
                const int k = idx >> lw, w = idx & (W - 1);
                const double x = w >= T.ncol ? 0.0 : r[e];
                if (!isfinite(x)) bad = true;
                const int u = (k & 1) ? n - 1 - (k >> 1) : (k >> 1);
                reinterpret_cast<double*>(z + w * cs)[u] = (kind == Z_DD && (k & 1)) ? -x : x;
            }
        } else {
            // the first radix-8 stage (Ns = 1: no twiddles) on the gathered
            // values, written to its Stockham output positions 8 j + r
            const int w = tid & (W - 1), j = tid >> lw, nbf = m / 8;
            const bool colok = w < T.ncol;
            double2 zin[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int u = j + q * nbf;
                double re = colok ? r[2 * q] : 0.0, im = colok ? r[2 * q + 1] : 0.0;
                if (!isfinite(re) || !isfinite(im)) bad = true;
                zin[q] = make_double2(re, im);
                if (quarter) zin[q] = cmul(zin[q], t1[u]);
            }
            dft<8>(zin, GlobalTab{nullptr}, m);
            double2* zc = z + w * cs + 8 * j;
#pragma unroll
            for (int q = 0; q < 8; ++q) zc[q] = zin[q];
        }
        // ---- the next tile's loads, in flight while this one is transformed
        const int vn = v + G;
        FTile Tn = T;
        if (vn < ntiles) {
            Tn = tiles[xcd_remap(vn, ntiles)];
            stream_load<NT>(r, in, Tn, lw, W, n, kind, inv_cos);
        }
        __syncthreads();

        fft_stream_columns<NT>(z, cs, a, twl, (inv_cos || cosine) ? 0 : 1);
        tid = fresh(threadIdx.x);

        if (inv_cos) {
            const double inv_n = 1.0 / n;
#pragma unroll
            for (int e = 0; e < kStreamPer; ++e) {
                const int idx = e * NT + tid;
                const int j = idx >> lw, w = idx & (W - 1);
                const int u = (j & 1) ? n - 1 - (j >> 1) : (j >> 1);
                const double2 F = z[w * cs + (u >> 1)];
                double y = (u & 1) ? -F.y * inv_n : F.x * inv_n;
                if (kind == Z_DD && (j & 1)) y = -y;
                if (w < T.ncol) out[T.out_base + (long long)j * T.out_stride + w] = y;
            }
        } else if (quarter) {
#pragma unroll
            for (int e = 0; e < kStreamPer / 2; ++e) {
                const int idx = e * NT + tid;
                const int k = idx >> lw, w = idx & (W - 1);
                const double2 u = cmul(z[w * cs + k], t2[k]);
                const int q0 = 2 * k, q1 = n - 1 - 2 * k;
                double y0 = sc2 * u.x, y1 = -sc2 * u.y;
                if (kind == Z_DN) {
                    if (q0 & 1) y0 = -y0;
                    if (q1 & 1) y1 = -y1;
                }
                if (w < T.ncol) {
                    out[T.out_base + (long long)q0 * T.out_stride + w] = y0;
                    out[T.out_base + (long long)q1 * T.out_stride + w] = y1;
                }
            }
        } else {
            // PP / NN / DD: bins k < m give the outputs at k and n - k (as in
            // k_r2r); bin 0's group also gives bin m.  m W = 8 NT groups.
            const bool pp = kind == Z_PP, dd = kind == Z_DD;
#pragma unroll
            for (int e = 0; e < kStreamPer / 2; ++e) {
                const int idx = e * NT + tid;
                const int k = idx >> lw, w = idx & (W - 1);
                // bin q's real DFT value X_q from the half-length FFT
                auto Xq = [&](int q) -> double2 {
                    const double2 Zk = z[w * cs + (q == m ? 0 : q)];
                    const double2 Zc = cconj(z[w * cs + (q == 0 ? 0 : m - q)]);
                    const double2 sm = make_double2(0.5 * (Zk.x + Zc.x), 0.5 * (Zk.y + Zc.y));
                    const double2 d = make_double2(0.5 * (Zk.x - Zc.x), 0.5 * (Zk.y - Zc.y));
                    const double2 t = cmul(t1[q], d);
                    return make_double2(sm.x + t.y, sm.y - t.x);
                };
                // output at row rk of bin q (the only one for q = 0 and q = m)
                auto first = [&](int q, const double2& X) -> double {
                    const double2 pk = t2[q];
                    return pp ? sc1 * (X.x - X.y) : (q == 0 ? sc1 : sc2) * (pk.x * X.x - pk.y * X.y);
                };
                const double2 X = Xq(k);
                const double ya = first(k, X);
                const int ra = dd ? n - 1 - k : k;
                double yb;
                int rb;
                if (k == 0) {
                    yb = first(m, Xq(m));
                    rb = dd ? n - 1 - m : m;
                } else {
                    const double2 pk = t2[k];
                    const double2 pn = make_double2(-pk.y, -pk.x);  // post[n - k]
                    yb = pp ? sc1 * (X.x + X.y) : sc2 * (pn.x * X.x + pn.y * X.y);
                    rb = pp ? n - k : dd ? k - 1 : n - k;
                }
                if (w < T.ncol) {
                    double* o = out + T.out_base + w;
                    o[(long long)ra * T.out_stride] = ya;
                    o[(long long)rb * T.out_stride] = yb;
                }
            }
        }
        if (vn >= ntiles) break;
        __syncthreads();  // the next tile overwrites the image
        T = Tn;
        v = vn;
    }
    if (bad && nonfinite) atomicOr(nonfinite, 1);
}

int fft_col_stride(const mbp_plan* P);

// Columns per workgroup, a power of two up to 64: wide tiles read long row
// segments and amortise the stage barriers.  Each stage gives a thread at
// most 16 complex values (4 butterflies of radix 4, 8 of radix 2, 2 of the
// radices 3 to 8, 1 of the larger ones).  The LDS image W * cs complex
// values is held to 40 KB (four workgroups per CU) unless that leaves fewer
// than 8 columns, then to 80 KB (two per CU).
constexpr int64_t kFFTLdsSmall = 40 * 1024;
constexpr int64_t kFFTLds = 80 * 1024;

static int fft_width_for(const mbp_plan* P, int64_t lds) {
    const int m = P->fft.m;
    int W = 64;
    while (W > 1 && int64_t(W) * fft_col_stride(P) * 16 > std::min<int64_t>(lds, P->lds_limit)) W >>= 1;
    for (int R : P->fft.radices) {
        const int per = R > 8 ? 1 : (R == 2 ? 8 : R == 4 ? 4 : 2);  // butterflies per thread
        while (W > 1 && W * (m / R) > per * 256) W >>= 1;
        if (R > 31)  // the any-radix stage holds W m / 256 outputs per thread
            while (W > 1 && W * m > kGenericOut * 256) W >>= 1;
    }
    return W;
}

static int radix_class(const mbp_plan* P);

// Streaming form: power-of-two half lengths m >= 128, W the widest power of
// two in [16, 64] with NT = n W / kStreamPer <= MBP_FFT_STREAM_MAXNT threads
// and the image plus the tables (3 m + 2 values) in the LDS limit; 0 when the
// form does not apply (the per-tile kernel runs).
#ifndef MBP_FFT_STREAM_MAXNT
#define MBP_FFT_STREAM_MAXNT 1024
#endif
static int stream_width(const mbp_plan* P) {
    const int n = P->fft.n, m = P->fft.m;
    if (radix_class(P) != 0 || m < 128 || P->fft.radices[0] != 8) return 0;
    const int cs = fft_col_stride(P);
    for (int W = 64; W >= 16; W >>= 1) {
        const int nt = n * W / kStreamPer;
        if (nt > MBP_FFT_STREAM_MAXNT || nt < 256) continue;
        if ((int64_t(W) * cs + 3 * m + 2) * 16 <= P->lds_limit) return W;
    }
    return 0;
}

int fft_columns_per_wg(const mbp_plan* P) {
    const int Ws = stream_width(P);
    if (Ws) return Ws;
    const int W = fft_width_for(P, kFFTLdsSmall);
    return W >= 8 ? W : fft_width_for(P, kFFTLds);
}

// Column stride in complex values: one padding slot breaks the power-of-two
// bank pattern when the padded image still fits.
int fft_col_stride(const mbp_plan* P) {
    const int m = P->fft.m;
    return (int64_t(8) * (m + 1) * 16 <= std::min<int64_t>(kFFTLds, P->lds_limit)) ? m + 1 : m;
}

void fft_build_tiles(const mbp_plan* P, std::vector<unsigned char>& fwd, std::vector<unsigned char>& inv,
                     int* ntiles) {
    const int W = fft_columns_per_wg(P);
    std::vector<FTile> f, iv;
    for (int b = 0; b < P->g.nb; ++b) {
        long long cols = (long long)P->g.nx[b] * P->g.ny[b];
        long long off2 = P->levels[0].off[b];
        for (long long c0 = 0; c0 < cols; c0 += W) {
            FTile t{};
            t.ncol = int(std::min<long long>(W, cols - c0));
            t.in_base = P->block_off[b] + c0;
            t.in_stride = int(cols);
            t.out_base = off2 + c0;
            t.out_stride = int(P->plane0);
            f.push_back(t);
            FTile u{};
            u.ncol = t.ncol;
            u.in_base = off2 + c0;
            u.in_stride = int(P->plane0);
            u.out_base = P->block_off[b] + c0;
            u.out_stride = int(cols);
            iv.push_back(u);
        }
    }
    *ntiles = int(f.size());
    fwd.assign(reinterpret_cast<unsigned char*>(f.data()),
               reinterpret_cast<unsigned char*>(f.data()) + f.size() * sizeof(FTile));
    inv.assign(reinterpret_cast<unsigned char*>(iv.data()),
               reinterpret_cast<unsigned char*>(iv.data()) + iv.size() * sizeof(FTile));
}

static FFTArgs make_args(const mbp_plan* P) {
    FFTArgs a{};
    a.n = P->fft.n;
    a.m = P->fft.m;
    a.kind = P->g.zkind;
    a.W = fft_columns_per_wg(P);
    a.cs = fft_col_stride(P);
    a.nstage = int(P->fft.radices.size());
    for (int s = 0; s < a.nstage && s < 16; ++s) a.radix[s] = P->fft.radices[s];
    a.tw = P->d_dbl + P->fft_tw;
    a.twn = P->d_dbl + P->fft_twn;
    a.post = P->d_dbl + P->fft_post;
    a.pre4 = P->d_dbl + P->fft_pre4;
    a.post4 = P->d_dbl + P->fft_post4;
    return a;
}

static size_t lds_bytes(const mbp_plan* P) {
    const size_t img = size_t(fft_columns_per_wg(P)) * fft_col_stride(P);
    return (stream_width(P) ? img + 3 * size_t(P->fft.m) + 2 : img) * sizeof(double2);
}

static int radix_class(const mbp_plan* P) {
    int c = 0;
    for (int R : P->fft.radices) {
        if (R == 3 || R == 5 || R == 7) c = std::max(c, 1);
        else if (R > 31) c = 3;
        else if (R > 8) c = std::max(c, 2);
    }
    return c;
}

template <int CLASS>
static void launch_r2r(const mbp_plan* P, const FFTArgs& a, const void* tiles, int dir, const double* in,
                       double* out, int* nonfinite, hipStream_t s) {
    const size_t bytes = lds_bytes(P);
    if (bytes > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_r2r<CLASS>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
    hipLaunchKernelGGL(k_r2r<CLASS>, dim3(P->fft_ntiles), dim3(256), bytes, s, a,
                       reinterpret_cast<const FTile*>(tiles), P->fft_ntiles, dir, in, out, nonfinite);
}

template <int NT>
static void launch_stream(const mbp_plan* P, const FFTArgs& a, const void* tiles, int dir, const double* in,
                          double* out, int* nonfinite, hipStream_t s) {
    const size_t bytes = lds_bytes(P);
    if (bytes > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_r2r_stream<NT>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
    hipLaunchKernelGGL(k_r2r_stream<NT>, dim3(P->fft_grid), dim3(NT), bytes, s, a,
                       reinterpret_cast<const FTile*>(tiles), P->fft_ntiles, dir, in, out, nonfinite);
}

// Launch shape of the streaming form on the current device: the thread count
// and a grid of as many workgroups as fit on the chip at once (a multiple of
// 8, so each keeps its XCD's share of tiles), at most one per tile.
int fft_stream_setup(mbp_plan* P) {
    P->fft_stream_nt = 0;
    P->fft_grid = 0;
    const int W = stream_width(P);
    if (!W) return MBP_OK;
    const int nt = P->fft.n * W / kStreamPer;
    const size_t bytes = lds_bytes(P);
    const void* fn = nt == 256    ? reinterpret_cast<const void*>(k_r2r_stream<256>)
                     : nt == 512 ? reinterpret_cast<const void*>(k_r2r_stream<512>)
                                 : reinterpret_cast<const void*>(k_r2r_stream<1024>);
    if (bytes > 64 * 1024 &&
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)) != hipSuccess)
        return MBP_ERR_HIP;
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, nt, bytes) != hipSuccess)
        return MBP_ERR_HIP;
    int g = std::min<int64_t>(P->fft_ntiles, int64_t(std::max(per, 1)) * std::max(ncu, 1));
    if (g >= 8) g -= g % 8;
    P->fft_stream_nt = nt;
    P->fft_grid = std::max(g, 1);
    return MBP_OK;
}

static void run_r2r(const mbp_plan* P, const void* tiles, int dir, const double* in, double* out,
                    int* nonfinite, hipStream_t s) {
    const FFTArgs a = make_args(P);
    if (P->fft_stream_nt) {
        switch (P->fft_stream_nt) {
            case 256: launch_stream<256>(P, a, tiles, dir, in, out, nonfinite, s); break;
            case 512: launch_stream<512>(P, a, tiles, dir, in, out, nonfinite, s); break;
            default: launch_stream<1024>(P, a, tiles, dir, in, out, nonfinite, s); break;
        }
        return;
    }
    switch (radix_class(P)) {
        case 0: launch_r2r<0>(P, a, tiles, dir, in, out, nonfinite, s); break;
        case 1: launch_r2r<1>(P, a, tiles, dir, in, out, nonfinite, s); break;
        case 2: launch_r2r<2>(P, a, tiles, dir, in, out, nonfinite, s); break;
        default: launch_r2r<3>(P, a, tiles, dir, in, out, nonfinite, s); break;
    }
}

void launch_forward(const mbp_plan* P, const double* f, double* fhat, int* nonfinite, hipStream_t s) {
    run_r2r(P, P->d_ftiles_fwd, 0, f, fhat, nonfinite, s);
}

void launch_inverse(const mbp_plan* P, const double* phat, double* p, hipStream_t s) {
    run_r2r(P, P->d_ftiles_inv, 1, phat, p, nullptr, s);
}

}  // namespace mbp
