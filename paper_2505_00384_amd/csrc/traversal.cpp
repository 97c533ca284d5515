// Cell traversal order of the operator kernel.
//
// A cell reads its six neighbours' values and the face data it shares with
// them, so the order in which workgroups visit cells decides how often those
// reads hit in the L2 of the XCD that runs them.  For meshes numbered as a
// structured nx*ny*nz block (x fastest; any direction periodic or bounded),
// cells are visited by tiles of TX x TY columns, each tile swept layer by
// layer: the +-x and +-y neighbours are a few cells away in the sequence and
// the +-z neighbour one tile layer away, well inside one L2.  The kernel
// splits the sequence into one contiguous range per XCD.  Other meshes keep
// their own numbering.
#include <vector>

#include "common.hpp"

namespace hx {

namespace {

bool is_structured(const int32_t *nb, int64_t n, int64_t nx, int64_t ny, int64_t nz)
{
    if (nx * ny * nz != n) return false;
    for (int64_t c = 0; c < n; ++c) {
        const int64_t ix = c % nx, iy = (c / nx) % ny, iz = c / (nx * ny);
        const int64_t dims[3] = {nx, ny, nz}, idx[3] = {ix, iy, iz};
        const int64_t stride[3] = {1, nx, nx * ny};
        for (int d = 0; d < 3; ++d)
            for (int s = 0; s < 2; ++s) {
                const int32_t v = nb[6 * c + 2 * d + s];
                if (v < 0) continue;
                int64_t k = idx[d] + (s ? 1 : -1);
                k = (k + dims[d]) % dims[d];
                if (v != c + (k - idx[d]) * stride[d]) return false;
            }
    }
    return true;
}

// extent of the first run of cells linked through face f (+x: 1, +y: 3)
int64_t run_length(const int32_t *nb, int64_t n, int f, int64_t step)
{
    int64_t len = 1, c = 0;
    while (len <= n) {
        const int32_t v = nb[6 * c + f];
        if (v != c + step) break;
        c = v;
        ++len;
    }
    return len;
}

}  // namespace

void build_traversal(const int32_t *nb, int64_t n, int32_t *order)
{
    const int64_t nx = run_length(nb, n, 1, 1);
    const int64_t ny = (nx > 0 && n % nx == 0) ? run_length(nb, n, 3, nx) : 0;
    const int64_t nz = (nx * ny > 0 && n % (nx * ny) == 0) ? n / (nx * ny) : 0;
    if (nz == 0 || !is_structured(nb, n, nx, ny, nz)) {
        for (int64_t c = 0; c < n; ++c) order[c] = (int32_t)c;
        return;
    }
    const int64_t TX = nx < 32 ? nx : 32, TY = ny < 8 ? ny : 8;
    int64_t o = 0;
    for (int64_t ty = 0; ty < ny; ty += TY)
        for (int64_t tx = 0; tx < nx; tx += TX)
            for (int64_t z = 0; z < nz; ++z)
                for (int64_t y = ty; y < ty + TY && y < ny; ++y)
                    for (int64_t x = tx; x < tx + TX && x < nx; ++x)
                        order[o++] = (int32_t)(x + nx * (y + ny * z));
}

}  // namespace hx
