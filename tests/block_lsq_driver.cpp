// Feeds a block Hessenberg matrix to the library's block least-squares
// reduction (paper_2203_11025_amd/csrc/block_lsq.h) one block column at a
// time, as block FGMRES does, and writes after every column the residual
// norms it reports and the solution of the reduced system.  Built with gcc's
// sanitizers by tests/test_block_lsq_host.py, which compares the output with
// numpy's least squares; nothing else uses it.
//
// Input file (binary): int32 s, int32 m, beta (s x s complex128, row-major),
// Hbar ((m + 1) s x m s complex128, row-major).
// Output file (binary): for j = 0 .. m - 1: res (s float64), then
// Y ((j + 1) s x s complex128, row-major).
#include <cstdio>
#include <vector>

#include "block_lsq.h"

using helm::cd;

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int s = 0, m = 0;
    if (std::fread(&s, sizeof(int), 1, f) != 1 || std::fread(&m, sizeof(int), 1, f) != 1 || s < 1 || m < 1)
        return 2;
    const size_t M1 = (size_t)(m + 1) * s, MS = (size_t)m * s;
    std::vector<cd> beta((size_t)s * s), H(M1 * MS);
    if (std::fread(beta.data(), sizeof(cd), beta.size(), f) != beta.size() ||
        std::fread(H.data(), sizeof(cd), H.size(), f) != H.size())
        return 2;
    std::fclose(f);

    helm::BlockLsq L;
    L.reset(s, m, beta);
    FILE *o = std::fopen(argv[2], "wb");
    if (!o) return 2;
    std::vector<double> res;
    std::vector<cd> Y;
    for (int j = 0; j < m; ++j) {
        // block column j has rows 0 .. (j + 2) s - 1 (block Hessenberg)
        for (int r = 0; r < (j + 2) * s; ++r)
            for (int k = 0; k < s; ++k) L.h(r, j * s + k) = H[(size_t)r * MS + (size_t)j * s + k];
        L.add_column(j, res);
        L.solve(j + 1, Y);
        std::fwrite(res.data(), sizeof(double), res.size(), o);
        std::fwrite(Y.data(), sizeof(cd), Y.size(), o);
    }
    std::fclose(o);
    return 0;
}
