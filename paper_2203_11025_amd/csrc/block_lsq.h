// Host-side least squares of block flexible GMRES (section 4: block
// restarted FGMRES of Calandra, Gratton, Langou, Pinel and Vasseur), used by
// block_fgmres.hip.  Plain C++ with no HIP dependency, so that the CPU tests
// can build it on its own.
#pragma once

#include <cmath>
#include <complex>
#include <vector>

namespace helm {

typedef std::complex<double> cd;

// Least squares of a block FGMRES cycle, min || E - H Y || with H the block
// Hessenberg matrix ((m + 1) s x m s) and E the first block column scaled by
// the Cholesky factor of the residual block, by Householder reflections
// computed one block column at a time as the Arnoldi process adds it: step j
// applies the reflections of the earlier columns to the new block column,
// then finds its own s reflections over rows j s .. (j + 2) s - 1 (the
// Hessenberg structure leaves nothing below) and applies them to E.  The
// reduced block column stays in H (upper triangular part R), so a step costs
// O(j s^3) instead of refactoring O((j s)^3).  Each reflection is I - 2 u u^H
// / (u^H u) with u = x + phase(x_0) ||x|| e_0 on its column's sub-diagonal
// part.
struct BlockLsq {
    int s = 0, M1 = 0, MS = 0;
    std::vector<cd> H, E;           // [M1][MS], [M1][s], reduced in place
    std::vector<std::vector<cd>> u;  // reflection of column c, rows c .. c + u[c].size() - 1
    std::vector<double> un;          // u^H u (0: no reflection)

    void reset(int s_, int m, const std::vector<cd> &beta)
    {
        s = s_;
        M1 = (m + 1) * s;
        MS = m * s;
        H.assign((size_t)M1 * MS, cd(0.0));
        E.assign((size_t)M1 * s, cd(0.0));
        for (int i = 0; i < s; ++i)
            for (int k = 0; k < s; ++k) E[(size_t)i * s + k] = beta[(size_t)i * s + k];
        u.assign(MS, {});
        un.assign(MS, 0.0);
    }
    cd &h(int r, int c) { return H[(size_t)r * MS + c]; }
    // applies reflection c to column j of H (ncols = 1) or to E (all s columns)
    void reflect_h(int c, int j)
    {
        if (un[c] == 0.0) return;
        const std::vector<cd> &v = u[c];
        cd t = 0.0;
        for (size_t i = 0; i < v.size(); ++i) t += std::conj(v[i]) * h(c + (int)i, j);
        t *= 2.0 / un[c];
        for (size_t i = 0; i < v.size(); ++i) h(c + (int)i, j) -= v[i] * t;
    }
    void reflect_e(int c)
    {
        if (un[c] == 0.0) return;
        const std::vector<cd> &v = u[c];
        for (int q = 0; q < s; ++q) {
            cd t = 0.0;
            for (size_t i = 0; i < v.size(); ++i) t += std::conj(v[i]) * E[(size_t)(c + i) * s + q];
            t *= 2.0 / un[c];
            for (size_t i = 0; i < v.size(); ++i) E[(size_t)(c + i) * s + q] -= v[i] * t;
        }
    }
    // block column j of H (rows 0 .. (j + 2) s - 1) has been filled: reduce
    // it; res[q] = the least-squares residual norm of right-hand side q
    void add_column(int j, std::vector<double> &res)
    {
        const int c0 = j * s, rows = (j + 2) * s;
        for (int k = 0; k < s; ++k)
            for (int c = 0; c < c0; ++c) reflect_h(c, c0 + k);
        for (int k = 0; k < s; ++k) {
            const int c = c0 + k;
            double nrm = 0.0;
            for (int i = c; i < rows; ++i) nrm += std::norm(h(i, c));
            nrm = std::sqrt(nrm);
            if (nrm == 0.0) continue;
            const cd a0 = h(c, c);
            const cd ph = std::abs(a0) > 0.0 ? a0 / std::abs(a0) : cd(1.0);
            std::vector<cd> v(rows - c);
            for (int i = c; i < rows; ++i) v[i - c] = h(i, c);
            v[0] += ph * nrm;
            double n2 = 0.0;
            for (const cd &z : v) n2 += std::norm(z);
            u[c] = std::move(v);
            un[c] = n2;
            for (int kk = k; kk < s; ++kk) reflect_h(c, c0 + kk);
            reflect_e(c);
        }
        // ||E - R Y||: the rows below the reduced columns, plus, where a
        // column had nothing left to reduce (a zero pivot, which solve()
        // answers with a zero component), the misfit of its own row
        const int cols = (j + 1) * s;
        std::vector<double> r2(s, 0.0);
        for (int q = 0; q < s; ++q)
            for (int i = cols; i < rows; ++i) r2[q] += std::norm(E[(size_t)i * s + q]);
        bool zero_pivot = false;
        for (int c = 0; c < cols; ++c) zero_pivot = zero_pivot || h(c, c) == cd(0.0);
        if (zero_pivot) {
            std::vector<cd> Y;
            solve(j + 1, Y);
            for (int c = 0; c < cols; ++c) {
                if (h(c, c) != cd(0.0)) continue;
                for (int q = 0; q < s; ++q) {
                    cd t = E[(size_t)c * s + q];
                    for (int k = c + 1; k < cols; ++k) t -= h(c, k) * Y[(size_t)k * s + q];
                    r2[q] += std::norm(t);
                }
            }
        }
        res.assign(s, 0.0);
        for (int q = 0; q < s; ++q) res[q] = std::sqrt(r2[q]);
    }
    // Y ((kk s) x s) from the reduced system of the first kk block columns
    void solve(int kk, std::vector<cd> &Y)
    {
        const int cols = kk * s;
        Y.assign((size_t)cols * s, cd(0.0));
        for (int q = 0; q < s; ++q)
            for (int i = cols - 1; i >= 0; --i) {
                cd t = E[(size_t)i * s + q];
                for (int k = i + 1; k < cols; ++k) t -= h(i, k) * Y[(size_t)k * s + q];
                Y[(size_t)i * s + q] = h(i, i) != cd(0.0) ? t / h(i, i) : cd(0.0);
            }
    }
};

}  // namespace helm
