// Moment indexing of the P_N system and the sparsity of its flux operators (host + device).
//
// Moments are the real spherical harmonics m_l^k of degree l <= N, index j = l^2 + l + k
// (Sec. 3.1).  Three reflections act on them diagonally:
//   z -> -z (mu -> -mu):        (-1)^(l+|k|)
//   x -> -x (phi -> -phi):      +1 for k >= 0 (cosine and zonal harmonics), -1 for k < 0 (sine)
//   y -> -y (phi -> pi - phi):  (-1)^|k| for k >= 0, (-1)^(|k|+1) for k < 0
// (the directions are Omega = (sqrt(1-mu^2) sin phi, sqrt(1-mu^2) cos phi, mu)).  The three
// parities form a class of 8 values.  Omega_x is odd under the x reflection and even under
// the other two, and multiplying by it moves the degree and the order |k| by exactly one:
// A_x = int m m^T Omega_x couples j and i only when both change by one and the classes
// differ in the x parity alone.  Likewise A_y with the y parity.  |A_x| and |A_y| are
// functions of A_x and A_y that commute with all three reflections, so they couple only
// moments of the same class.  The library checks these patterns against the matrices it
// builds; the kernels only touch the entries inside them.
#pragma once

#include <array>
#include <cstdint>

namespace snrt {
namespace pn {

constexpr int kMaxDegree = 30;        // largest P_N degree the library accepts
constexpr int kMaxFusedDegree = 9;    // degrees 0..9 have a fully unrolled FP32 step kernel
constexpr int kFusedHighDegree = 13;  // and degree 13 (the CSD degree of Sec. 7) as well
constexpr int kMaxFusedDegree64 = 2;  // the same for FP64 (its accumulators take twice the
                                      // registers; larger degrees use the chunked kernel)
template <typename T>
constexpr int max_fused_degree() { return sizeof(T) == 4 ? kMaxFusedDegree : kMaxFusedDegree64; }
template <typename T>
constexpr bool has_fused_kernel(int N) {
    return N <= max_fused_degree<T>() || (sizeof(T) == 4 && N == kFusedHighDegree);
}

constexpr int nmom(int N) { return (N + 1) * (N + 1); }

struct Mom {
    int l = 0, k = 0, cls = 0;
};

constexpr Mom mom(int j) {
    int l = 0;
    while ((l + 1) * (l + 1) <= j) ++l;
    const int k = j - l * l - l;
    const int a = k < 0 ? -k : k;
    const int pz = (l + a) & 1, px = k < 0 ? 1 : 0, py = (a + px) & 1;
    return Mom{l, k, pz * 4 + px * 2 + py};
}

constexpr bool step_by_one(int a, int b) { return a - b == 1 || b - a == 1; }
constexpr int absi(int a) { return a < 0 ? -a : a; }

constexpr bool ax_nz(const Mom& a, const Mom& b) {
    return step_by_one(a.l, b.l) && step_by_one(absi(a.k), absi(b.k)) && (a.cls ^ b.cls) == 2;
}
constexpr bool ay_nz(const Mom& a, const Mom& b) {
    return step_by_one(a.l, b.l) && step_by_one(absi(a.k), absi(b.k)) && (a.cls ^ b.cls) == 1;
}
constexpr bool abs_nz(const Mom& a, const Mom& b) { return a.cls == b.cls; }

// Operand of a flux coefficient: the per-cell aggregates the step forms for every moment m,
//   X_m = sum_f n_x,f (u_i + u_f)_m,    Y_m = sum_f n_y,f (u_i + u_f)_m,
//   P_m = sum_f |n_x,f| (u_i - u_f)_m,  Q_m = sum_f |n_y,f| (u_i - u_f)_m   (u = moments/rho),
// so that sum_f F_up = (A_x X + A_y Y + |A_x| P + |A_y| Q) / 2.
enum : int8_t { kOpX = 0, kOpY = 1, kOpP = 2, kOpQ = 3 };

struct Op {
    int16_t k = 0;    // output moment
    int8_t kind = 0;  // kOp*
};

// Calls f(m, k, kind) for every structurally non-zero coefficient, grouped by the input
// moment m, in the order of the packed coefficient table.
template <class F>
constexpr void visit_ops(int N, F&& f) {
    std::array<Mom, nmom(kMaxDegree)> ms{};
    const int nm = nmom(N);
    for (int j = 0; j < nm; ++j) ms[j] = mom(j);
    for (int m = 0; m < nm; ++m)
        for (int k = 0; k < nm; ++k) {
            if (ax_nz(ms[m], ms[k])) f(m, k, (int)kOpX);
            if (ay_nz(ms[m], ms[k])) f(m, k, (int)kOpY);
            if (abs_nz(ms[m], ms[k])) {
                f(m, k, (int)kOpP);
                f(m, k, (int)kOpQ);
            }
        }
}

// Omega_x and Omega_y are both even under the z reflection, so A_x, A_y, |A_x| and |A_y|
// all keep the z parity: the moment system of a 2-D problem splits into two independent
// subsystems, the z-even and the z-odd moments (the diagonal scattering keeps them apart
// too).
constexpr int zpar(int j) { return mom(j).cls >> 2; }

template <int N, int PZ>
struct SubMoments {
    static constexpr int count = [] {
        int c = 0;
        for (int j = 0; j < nmom(N); ++j) c += zpar(j) == PZ;
        return c;
    }();
    static constexpr std::array<int, count> list = [] {
        std::array<int, count> a{};
        int c = 0;
        for (int j = 0; j < nmom(N); ++j)
            if (zpar(j) == PZ) a[c++] = j;
        return a;
    }();
};

// The z-parity-PZ moments ordered by reflection class for the matrix-core step: the four
// classes of that parity (local class lc = x parity * 2 + y parity) one after the other,
// largest first (equal sizes in class order), each in increasing moment order.  Inside a
// class, |A_x| and |A_y| are dense: with the class's moments as both inputs and outputs in
// this order, the class block is a product of the class's coefficient matrix with the
// stacked P and Q aggregates of its inputs.
template <int N, int PZ>
struct ClassOrder {
    static constexpr int NM = nmom(N);
    static constexpr std::array<int, 4> size = [] {
        std::array<int, 4> c{};
        for (int j = 0; j < NM; ++j)
            if (zpar(j) == PZ) ++c[mom(j).cls & 3];
        return c;
    }();
    // classes by decreasing size (stable)
    static constexpr std::array<int, 4> order = [] {
        std::array<int, 4> o{0, 1, 2, 3};
        for (int a = 0; a < 4; ++a)
            for (int b = a + 1; b < 4; ++b)
                if (size[o[b]] > size[o[a]] || (size[o[b]] == size[o[a]] && o[b] < o[a])) {
                    const int t = o[a];
                    o[a] = o[b];
                    o[b] = t;
                }
        return o;
    }();
    static constexpr int count = size[0] + size[1] + size[2] + size[3];
    static constexpr std::array<int, count> list = [] {
        std::array<int, count> l{};
        int c = 0;
        for (int q = 0; q < 4; ++q)
            for (int j = 0; j < NM; ++j)
                if (zpar(j) == PZ && (mom(j).cls & 3) == order[q]) l[c++] = j;
        return l;
    }();
    // position of moment j inside its class (its row and column in the class block)
    static constexpr std::array<int, NM> local = [] {
        std::array<int, NM> t{};
        std::array<int, 4> used{};
        for (int j = 0; j < NM; ++j) {
            t[j] = -1;
            if (zpar(j) == PZ) t[j] = used[mom(j).cls & 3]++;
        }
        return t;
    }();
    // moment at position t of local class lc (-1 past the class)
    static constexpr int at(int lc, int t) {
        int c = 0;
        for (int j = 0; j < NM; ++j)
            if (zpar(j) == PZ && (mom(j).cls & 3) == lc) {
                if (c == t) return j;
                ++c;
            }
        return -1;
    }
};

template <int N>
struct OpTable {
    static constexpr int NM = nmom(N);
    static constexpr int count = [] {
        int c = 0;
        visit_ops(N, [&](int, int, int) { ++c; });
        return c;
    }();
    static constexpr std::array<Op, count> ops = [] {
        std::array<Op, count> a{};
        int c = 0;
        visit_ops(N, [&](int, int k, int kind) {
            a[c].k = (int16_t)k;
            a[c].kind = (int8_t)kind;
            ++c;
        });
        return a;
    }();
    // ops of input moment m: [start[m], start[m+1])
    static constexpr std::array<int, NM + 1> start = [] {
        std::array<int, NM + 1> s{};
        int c = 0;
        visit_ops(N, [&](int m, int, int) {
            ++c;
            s[m + 1] = c;
        });
        for (int m = 1; m <= NM; ++m)
            if (s[m] < s[m - 1]) s[m] = s[m - 1];
        return s;
    }();
};

// The A_x and A_y coefficients (kinds X, Y) of OpTable<N> as a table of their own, in
// OpTable order: sidx[i] is the position of op i (-1 for the |A_x|, |A_y| kinds).
template <int N>
struct SparseOps {
    static constexpr int nops = OpTable<N>::count;
    static constexpr std::array<int, nops> sidx = [] {
        std::array<int, nops> a{};
        int c = 0;
        for (int i = 0; i < nops; ++i) {
            const int kind = OpTable<N>::ops[i].kind;
            a[i] = (kind == kOpX || kind == kOpY) ? c++ : -1;
        }
        return a;
    }();
    static constexpr int count = [] {
        int c = 0;
        for (int i = 0; i < nops; ++i)
            c += OpTable<N>::ops[i].kind == kOpX || OpTable<N>::ops[i].kind == kOpY;
        return c;
    }();
};

}  // namespace pn
}  // namespace snrt
