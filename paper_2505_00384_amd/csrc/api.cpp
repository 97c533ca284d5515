// C-ABI entry points of libhelmdg: context, argument validation, mesh and
// coefficient set-up, operator / preconditioner application.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace hx {

hx_status fail(hx_ctx *c, hx_status s, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

hx_status dalloc(hx_ctx *c, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(c, HX_ERR_OOM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    return HX_OK;
}

void dfree(void **p)
{
    if (*p) (void)hipFree(*p);
    *p = nullptr;
}

static void free_mesh(hx_ctx *c)
{
    void **bufs[] = {(void **)&c->nodes, (void **)&c->nbr, (void **)&c->visit, (void **)&c->visitp, (void **)&c->ref, (void **)&c->vol,
                     (void **)&c->ell, (void **)&c->mindet, (void **)&c->sigma,
                     (void **)&c->cell64, (void **)&c->cell32, (void **)&c->face64,
                     (void **)&c->face32, (void **)&c->cellgeo, (void **)&c->facegeo, (void **)&c->dg64, (void **)&c->dg32, (void **)&c->cgpart, (void **)&c->pqpart,
                     (void **)&c->bjS64, (void **)&c->bjS32,
                     (void **)&c->bjL64, (void **)&c->bjL32, (void **)&c->bjC64,
                     (void **)&c->bjC32, (void **)&c->coef_feat, (void **)&c->work64,
                     (void **)&c->work32, (void **)&c->psW, (void **)&c->psWC, (void **)&c->psMr,
                     (void **)&c->psMd, (void **)&c->psFn, (void **)&c->psFh, (void **)&c->psWork,
                     (void **)&c->refq, (void **)&c->qcell, (void **)&c->qface, (void **)&c->chebw,
                     (void **)&c->mg_cptr, (void **)&c->mg_clist, (void **)&c->mg_child8, (void **)&c->mgw,
                     (void **)&c->mgw32, (void **)&c->chebw32, (void **)&c->ctype,
                     (void **)&c->acell64, (void **)&c->acell32, (void **)&c->kk64,
                     (void **)&c->kk32, (void **)&c->aface64, (void **)&c->aface32,
                     (void **)&c->fc64, (void **)&c->fc32, (void **)&c->hang, (void **)&c->hgeo,
                     (void **)&c->hsig, (void **)&c->harea, (void **)&c->hdata64,
                     (void **)&c->hdata32, (void **)&c->hcontrib64, (void **)&c->hcontrib32,
                     (void **)&c->hcells, (void **)&c->hptr, (void **)&c->hlist,
                     (void **)&c->endsig};
    for (void **b : bufs) dfree(b);
    delete c->order_h;
    delete c->nbr_h;
    delete c->ctype_h;
    c->order_h = nullptr;
    c->nbr_h = nullptr;
    c->ctype_h = nullptr;
    c->n_vis_op = 0;
    c->vis_mode = 0;
    c->n_hang = c->n_hcell = 0;
    c->n_affine = c->n_iface = c->n_cface = 0;
    c->work64_len = c->work32_len = 0;
    c->has_mesh = c->has_coef = c->has_press = c->has_q = false;
    c->cheb_deg = 0;
    c->mg_coarse = nullptr;
    c->mg_nc = 0;
}

// Traversal records {cell, neighbours -x, +x, -y, +y, -z, +z, mask}.
// visitp: every cell once in the traversal order, mask 0 (kernels that read
// no compressed data).  visit (the operator): with the compression on and
// both kinds of cells present, the general cells and the affine cells form
// two groups, each in the traversal order and padded with records of cell -1
// to whole waves; the waves of the two groups are interleaved in proportion
// (so both groups advance together and every CU runs both kinds), and every
// wave's records are of one kind.  Mask bit 0: affine cell (also set on the
// padding of the affine group); bit 1 + f: face f (-x, +x, -y, +y, -z, +z)
// lies between two affine cells and is read compressed.
static hx_status update_visit_masks(hx_ctx *c)
{
    const std::vector<int32_t> &order = *c->order_h, &nb = *c->nbr_h;
    const std::vector<uint8_t> &ct = *c->ctype_h;
    const size_t nc = (size_t)c->n_cells;
    const int cpw = op_cells_per_wave(c->n);
    auto record = [&](int32_t *r, int32_t cell, int aff) {
        int32_t mask = aff;
        for (int f = 0; f < 6; ++f) {
            const int32_t n2 = cell >= 0 ? nb[6 * (size_t)cell + f] : -1;
            r[1 + f] = n2;
            if (aff && cell >= 0 && n2 >= 0 && ct[n2]) mask |= 2 << f;
        }
        r[0] = cell;
        r[7] = mask;
    };
    std::vector<int32_t> plain(nc * 8);
    for (size_t i = 0; i < nc; ++i) record(&plain[8 * i], order[i], 0);
    // the two groups, padded to whole waves
    std::vector<int32_t> grp[2];
    for (size_t i = 0; i < nc; ++i) grp[c->compress && ct[order[i]] ? 1 : 0].push_back(order[i]);
    for (auto &g : grp)
        while (g.size() % cpw) g.push_back(-1);
    const size_t w0 = grp[0].size() / cpw, w1 = grp[1].size() / cpw;
    c->vis_mode = (w0 && w1) ? 2 : (w1 ? 1 : 0);
    std::vector<int32_t> v((w0 + w1) * cpw * 8);
    size_t t0 = 0, t1 = 0, o = 0;
    while (t0 < w0 || t1 < w1) {
        // next wave from the group that is behind in proportion
        const int g = (t1 < w1 && (t0 >= w0 || t1 * w0 <= t0 * w1)) ? 1 : 0;
        size_t &t = g ? t1 : t0;
        for (int k = 0; k < cpw; ++k, ++o) record(&v[8 * o], grp[g][t * cpw + k], g);
        ++t;
    }
    c->n_vis_op = (int64_t)o;
    HX_HIP(c, hipMemcpyAsync(c->visit, v.data(), sizeof(int32_t) * v.size(), hipMemcpyHostToDevice,
                             c->stream));
    HX_HIP(c, hipMemcpyAsync(c->visitp, plain.data(), sizeof(int32_t) * nc * 8, hipMemcpyHostToDevice,
                             c->stream));
    HX_HIP(c, hipStreamSynchronize(c->stream));
    return HX_OK;
}

// Block-Jacobi penalty of each non-conforming cell end: the fine cell's
// quarter penalty, or the area-weighted mean over the four quarters of a
// coarse face (the end term of the separable block stands for the whole face).
static hx_status update_hang_sigma(hx_ctx *c)
{
    if (c->n_hang == 0) return HX_OK;
    HX_HIP(c, launch_hang_geometry(c));
    std::vector<double> sig((size_t)c->n_hang), area((size_t)c->n_hang);
    std::vector<int32_t> rec((size_t)c->n_hang * 4);
    HX_HIP(c, hipMemcpyAsync(sig.data(), c->hsig, sizeof(double) * sig.size(), hipMemcpyDeviceToHost, c->stream));
    HX_HIP(c, hipMemcpyAsync(area.data(), c->harea, sizeof(double) * area.size(), hipMemcpyDeviceToHost,
                             c->stream));
    HX_HIP(c, hipMemcpyAsync(rec.data(), c->hang, sizeof(int32_t) * rec.size(), hipMemcpyDeviceToHost,
                             c->stream));
    HX_HIP(c, hipStreamSynchronize(c->stream));
    const size_t nc = (size_t)c->n_cells;
    std::vector<double> num(nc * 6, 0.0), den(nc * 6, 0.0), es(nc * 6, -1.0);
    for (size_t h = 0; h < sig.size(); ++h) {
        const int32_t C = rec[4 * h], fc = rec[4 * h + 1], F = rec[4 * h + 2];
        num[6 * (size_t)C + fc] += area[h] * sig[h];
        den[6 * (size_t)C + fc] += area[h];
        num[6 * (size_t)F + (fc ^ 1)] += area[h] * sig[h];
        den[6 * (size_t)F + (fc ^ 1)] += area[h];
    }
    for (size_t i = 0; i < nc * 6; ++i)
        if (den[i] > 0.0) es[i] = num[i] / den[i];
    HX_HIP(c, hipMemcpyAsync(c->endsig, es.data(), sizeof(double) * es.size(), hipMemcpyHostToDevice,
                             c->stream));
    HX_HIP(c, hipStreamSynchronize(c->stream));
    return HX_OK;
}

// Check the quarter-face records against the neighbour table (host arrays):
// every face marked -2 is a coarse face listed with its four quarters once
// each, or a fine face listed once; records name cells, faces and quarters
// in range.
static hx_status check_hanging(hx_ctx *c, int64_t n_cells, const int64_t *nbr, int64_t n_hang,
                               const int64_t *hang)
{
    std::vector<int> cover((size_t)n_cells * 6, 0), qmask((size_t)n_cells * 6, 0);
    for (int64_t h = 0; h < n_hang; ++h) {
        const int64_t C = hang[4 * h], fc = hang[4 * h + 1], F = hang[4 * h + 2], s = hang[4 * h + 3];
        if (C < 0 || C >= n_cells || F < 0 || F >= n_cells || C == F || fc < 0 || fc > 5 || s < 0 || s > 3)
            return fail(c, HX_ERR_MESH, "hanging record %lld out of range", (long long)h);
        if (nbr[6 * C + fc] != -2 || nbr[6 * F + (fc ^ 1)] != -2)
            return fail(c, HX_ERR_MESH, "hanging record %lld: its faces are not marked -2", (long long)h);
        int &q = qmask[6 * (size_t)C + fc];
        if (q & (1 << s)) return fail(c, HX_ERR_MESH, "hanging record %lld: quarter %lld twice", (long long)h, (long long)s);
        q |= 1 << s;
        cover[6 * (size_t)C + fc] += 1;
        if (cover[6 * (size_t)F + (fc ^ 1)]++ != 0)
            return fail(c, HX_ERR_MESH, "hanging record %lld: fine face listed twice", (long long)h);
    }
    for (int64_t i = 0; i < n_cells; ++i)
        for (int f = 0; f < 6; ++f) {
            if (nbr[6 * i + f] != -2) continue;
            const int k = cover[6 * (size_t)i + f];
            if (k != 1 && !(k == 4 && qmask[6 * (size_t)i + f] == 15))
                return fail(c, HX_ERR_MESH, "cell %lld face %d marked -2 without its quarter records",
                            (long long)i, f);
        }
    return HX_OK;
}

}  // namespace hx

using namespace hx;

extern "C" {

int hx_max_degree(void) { return MAXK; }

hx_status hx_create(hx_ctx **out, int device, void *hip_stream)
{
    if (!out) return HX_ERR_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return HX_ERR_DEVICE;
    }
    if (device < 0 || device >= ndev) return HX_ERR_ARG;
    if (hipSetDevice(device) != hipSuccess) return HX_ERR_DEVICE;
    hx_ctx *c = new hx_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    hx_status s = dalloc(c, (void **)&c->red, sizeof(double) * (size_t)1024 * 72);
    if (s == HX_OK) s = dalloc(c, (void **)&c->dpart, sizeof(double) * (size_t)1024 * 128);
    if (s == HX_OK && hipHostMalloc((void **)&c->red_host, sizeof(double) * 1024) != hipSuccess)
        s = HX_ERR_DEVICE;
    if (s == HX_OK && (hipHostMalloc((void **)&c->pin_host, sizeof(double) * 2 * FG_SLOT,
                                     hipHostMallocMapped) != hipSuccess ||
                       hipHostGetDevicePointer((void **)&c->pin_dev, c->pin_host, 0) != hipSuccess))
        s = HX_ERR_DEVICE;
    if (s == HX_OK) s = noalloc_init(c);
    if (s != HX_OK) {
        hx_destroy(c);
        return s;
    }
    *out = c;
    return HX_OK;
}

hx_status hx_destroy(hx_ctx *c)
{
    if (!c) return HX_OK;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    mlp_destroy(c);
    free_mesh(c);
    dfree((void **)&c->red);
    dfree((void **)&c->dpart);
    if (c->red_host) (void)hipHostFree(c->red_host);
    if (c->pin_host) (void)hipHostFree(c->pin_host);
    delete c;
    return HX_OK;
}

const char *hx_last_error(const hx_ctx *c) { return c ? c->err.c_str() : "null context"; }

int64_t hx_num_dofs(const hx_ctx *c) { return (c && c->has_mesh) ? c->n_dofs : -1; }

hx_status hx_setup_mesh(hx_ctx *c, int degree, int64_t n_cells, int geo_degree,
                        const double *geo_nodes, const int64_t *neighbours)
{
    return hx_setup_mesh_hanging(c, degree, n_cells, geo_degree, geo_nodes, neighbours, 0, nullptr);
}

hx_status hx_setup_mesh_hanging(hx_ctx *c, int degree, int64_t n_cells, int geo_degree,
                                const double *geo_nodes, const int64_t *neighbours, int64_t n_hang,
                                const int64_t *hang)
{
    if (!c) return HX_ERR_ARG;
    c->err.clear();
    if (degree < 1 || degree > MAXK)
        return fail(c, HX_ERR_ARG, "degree %d outside 1..%d", degree, MAXK);
    if (geo_degree < 1 || geo_degree > MAXG)
        return fail(c, HX_ERR_ARG, "geometry degree %d outside 1..%d", geo_degree, MAXG);
    if (n_cells < 1 || n_cells >= (int64_t(1) << 31))
        return fail(c, HX_ERR_ARG, "n_cells %lld out of range", (long long)n_cells);
    if (!geo_nodes || !neighbours) return fail(c, HX_ERR_ARG, "null mesh array");
    // neighbour table: range and conformity
    std::vector<int32_t> nb32((size_t)n_cells * 6);
    for (int64_t i = 0; i < n_cells; ++i)
        for (int f = 0; f < 6; ++f) {
            const int64_t v = neighbours[6 * i + f];
            if (v < (n_hang > 0 ? -2 : -1) || v >= n_cells)
                return fail(c, HX_ERR_MESH, "neighbour %lld of cell %lld face %d out of range",
                            (long long)v, (long long)i, f);
            if (v >= 0 && neighbours[6 * v + (f ^ 1)] != i)
                return fail(c, HX_ERR_MESH, "cell %lld face %d: neighbour %lld does not point back",
                            (long long)i, f, (long long)v);
            nb32[6 * i + f] = (int32_t)v;
        }
    if (n_hang < 0 || (n_hang > 0 && !hang)) return fail(c, HX_ERR_ARG, "bad hanging-face table");
    if (n_hang > 0) {
        hx_status sh = check_hanging(c, n_cells, neighbours, n_hang, hang);
        if (sh != HX_OK) return sh;
    }
    HX_HIP(c, hipSetDevice(c->device));
    free_mesh(c);
    c->k = degree;
    c->n = degree + 1;
    c->nf = c->n * c->n;
    c->nd = c->nf * c->n;
    c->g = geo_degree;
    c->n_cells = n_cells;
    c->n_dofs = n_cells * c->nd;
    const size_t ng3 = (size_t)(geo_degree + 1) * (geo_degree + 1) * (geo_degree + 1);
    const size_t nc = (size_t)n_cells;
    build_ref_tables(c->n, c->ref_host);
    hx_status s = HX_OK;
#define ALLOC(ptr, bytes)                                  \
    if (s == HX_OK) s = dalloc(c, (void **)&(ptr), (bytes));
    ALLOC(c->nodes, sizeof(double) * nc * ng3 * 3);
    ALLOC(c->nbr, sizeof(int32_t) * nc * 6);
    ALLOC(c->visit, sizeof(int32_t) * (nc + 2 * 64) * 8);
    ALLOC(c->visitp, sizeof(int32_t) * nc * 8);
    ALLOC(c->ref, sizeof(RefTab64));
    ALLOC(c->vol, sizeof(double) * nc);
    ALLOC(c->ell, sizeof(double) * nc * 3);
    ALLOC(c->mindet, sizeof(double) * nc);
    ALLOC(c->sigma, sizeof(double) * nc * 3);
    ALLOC(c->cell64, sizeof(double) * nc * 7 * c->nd);
    ALLOC(c->cell32, sizeof(float) * nc * 7 * c->nd);
    ALLOC(c->face64, sizeof(double) * nc * 3 * 7 * c->nf);
    ALLOC(c->face32, sizeof(float) * nc * 3 * 7 * c->nf);
    ALLOC(c->cellgeo, sizeof(double) * nc * 7 * c->nd);
    ALLOC(c->facegeo, sizeof(double) * nc * 3 * 7 * c->nf);
    ALLOC(c->dg64, sizeof(double) * 2 * nc * c->nd);
    ALLOC(c->dg32, sizeof(float) * 2 * nc * c->nd);
    ALLOC(c->cgpart, sizeof(double) * 2 * (nc + 1));
    ALLOC(c->pqpart, sizeof(double) * 2 * (nc + 1));
    ALLOC(c->bjS64, sizeof(double) * nc * 3 * c->nf);
    ALLOC(c->bjS32, sizeof(float) * nc * 3 * c->nf);
    ALLOC(c->bjL64, sizeof(double) * nc * 3 * c->n);
    ALLOC(c->bjL32, sizeof(float) * nc * 3 * c->n);
    ALLOC(c->bjC64, sizeof(double) * nc * 4);
    ALLOC(c->bjC32, sizeof(float) * nc * 4);
    ALLOC(c->coef_feat, sizeof(double) * nc);
    ALLOC(c->ctype, nc);
    ALLOC(c->acell64, sizeof(double) * nc * 2 * c->nd);
    ALLOC(c->acell32, sizeof(float) * nc * 2 * c->nd);
    ALLOC(c->kk64, sizeof(double) * nc * 8);
    ALLOC(c->kk32, sizeof(float) * nc * 8);
    ALLOC(c->aface64, sizeof(double) * nc * 3 * 2 * c->nf);
    ALLOC(c->aface32, sizeof(float) * nc * 3 * 2 * c->nf);
    ALLOC(c->fc64, sizeof(double) * nc * 3 * 8);
    ALLOC(c->fc32, sizeof(float) * nc * 3 * 8);
    c->n_hang = n_hang;
    std::vector<int32_t> hcells, hptr, hlist;
    if (n_hang > 0) {
        const size_t nh = (size_t)n_hang;
        ALLOC(c->hang, sizeof(int32_t) * nh * 4);
        ALLOC(c->hgeo, sizeof(double) * nh * 7 * c->nf);
        ALLOC(c->hsig, sizeof(double) * nh);
        ALLOC(c->harea, sizeof(double) * nh);
        ALLOC(c->hdata64, sizeof(double) * nh * 7 * c->nf);
        ALLOC(c->hdata32, sizeof(float) * nh * 7 * c->nf);
        ALLOC(c->hcontrib64, sizeof(double) * nh * 2 * c->nd);
        ALLOC(c->hcontrib32, sizeof(float) * nh * 2 * c->nd);
        ALLOC(c->endsig, sizeof(double) * nc * 6);
        // the quarter contributions of each cell, in record order
        std::vector<std::vector<int32_t>> by((size_t)n_cells);
        for (size_t h = 0; h < nh; ++h) {
            by[(size_t)hang[4 * h]].push_back((int32_t)(2 * h));
            by[(size_t)hang[4 * h + 2]].push_back((int32_t)(2 * h + 1));
        }
        hptr.push_back(0);
        for (size_t i = 0; i < nc; ++i) {
            if (by[i].empty()) continue;
            hcells.push_back((int32_t)i);
            hlist.insert(hlist.end(), by[i].begin(), by[i].end());
            hptr.push_back((int32_t)hlist.size());
        }
        c->n_hcell = (int64_t)hcells.size();
        ALLOC(c->hcells, sizeof(int32_t) * hcells.size());
        ALLOC(c->hptr, sizeof(int32_t) * hptr.size());
        ALLOC(c->hlist, sizeof(int32_t) * hlist.size());
    }
#undef ALLOC
    if (s != HX_OK) {
        free_mesh(c);
        return s;
    }
    HX_HIP(c, hipMemcpyAsync(c->nodes, geo_nodes, sizeof(double) * nc * ng3 * 3,
                             hipMemcpyHostToDevice, c->stream));
    HX_HIP(c, hipMemcpyAsync(c->nbr, nb32.data(), sizeof(int32_t) * nc * 6, hipMemcpyHostToDevice,
                             c->stream));
    if (n_hang > 0) {
        std::vector<int32_t> h32((size_t)n_hang * 4);
        for (size_t i = 0; i < h32.size(); ++i) h32[i] = (int32_t)hang[i];
        HX_HIP(c, hipMemcpyAsync(c->hang, h32.data(), sizeof(int32_t) * h32.size(), hipMemcpyHostToDevice,
                                 c->stream));
        HX_HIP(c, hipMemcpyAsync(c->hcells, hcells.data(), sizeof(int32_t) * hcells.size(),
                                 hipMemcpyHostToDevice, c->stream));
        HX_HIP(c, hipMemcpyAsync(c->hptr, hptr.data(), sizeof(int32_t) * hptr.size(), hipMemcpyHostToDevice,
                                 c->stream));
        HX_HIP(c, hipMemcpyAsync(c->hlist, hlist.data(), sizeof(int32_t) * hlist.size(),
                                 hipMemcpyHostToDevice, c->stream));
        HX_HIP(c, hipStreamSynchronize(c->stream));
    }
    c->order_h = new std::vector<int32_t>(nc);
    build_traversal(nb32.data(), n_cells, c->order_h->data());
    c->nbr_h = new std::vector<int32_t>(nb32);
    HX_HIP(c, hipMemcpyAsync(c->ref, &c->ref_host, sizeof(RefTab64), hipMemcpyHostToDevice,
                             c->stream));
    HX_HIP(c, launch_cell_geometry(c));
    std::vector<double> md(nc);
    HX_HIP(c, hipMemcpyAsync(md.data(), c->mindet, sizeof(double) * nc, hipMemcpyDeviceToHost,
                             c->stream));
    HX_HIP(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < nc; ++i)
        if (!(md[i] > 0.0)) {
            free_mesh(c);
            return fail(c, HX_ERR_MESH, "cell %zu: detJ = %g <= 0 at a quadrature point", i, md[i]);
        }
    HX_HIP(c, launch_face_sigma(c));
    {
        hx_status sh = update_hang_sigma(c);
        if (sh != HX_OK) return sh;
    }
    HX_HIP(c, launch_bj_eigen(c));
    HX_HIP(c, launch_geofac(c));
    HX_HIP(c, launch_affine_detect(c));
    c->ctype_h = new std::vector<uint8_t>(nc);
    HX_HIP(c, hipMemcpyAsync(c->ctype_h->data(), c->ctype, nc, hipMemcpyDeviceToHost, c->stream));
    HX_HIP(c, hipStreamSynchronize(c->stream));
    {
        const std::vector<uint8_t> &ct = *c->ctype_h;
        for (size_t i = 0; i < nc; ++i) {
            c->n_affine += ct[i];
            for (int d = 0; d < 3; ++d) {
                const int32_t nb = nb32[6 * i + 2 * d + 1];
                if (nb < 0) continue;
                ++c->n_iface;
                if (ct[i] && ct[nb]) ++c->n_cface;
            }
        }
    }
    hx_status sm = update_visit_masks(c);
    if (sm != HX_OK) return sm;
    c->has_mesh = true;
    return HX_OK;
}

hx_status hx_set_cell_compression(hx_ctx *c, int on)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_mesh) return fail(c, HX_ERR_STATE, "set_cell_compression before setup_mesh");
    c->compress = on ? 1 : 0;
    return update_visit_masks(c);
}

hx_status hx_operator_info(const hx_ctx *cc, int prec, int64_t *counts, double *bytes)
{
    if (!cc) return HX_ERR_ARG;
    hx_ctx *c = const_cast<hx_ctx *>(cc);
    if (!c->has_mesh) return fail(c, HX_ERR_STATE, "no mesh");
    if (prec != HX_F64 && prec != HX_F32) return fail(c, HX_ERR_ARG, "bad precision %d", prec);
    if (counts) {
        counts[0] = c->n_cells;
        counts[1] = c->n_affine;
        counts[2] = c->n_iface;
        counts[3] = c->n_cface;
    }
    if (bytes) {
        const double T = prec == HX_F64 ? 8.0 : 4.0;
        const double na = c->compress ? (double)c->n_affine : 0.0;
        const double nfc = c->compress ? (double)c->n_cface : 0.0;
        const double nd = c->nd, nf = c->nf;
        *bytes = T * (2.0 * (double)c->n_dofs + ((double)c->n_cells - na) * 7.0 * nd +
                      na * (2.0 * nd + 6.0) + ((double)c->n_iface - nfc) * 7.0 * nf +
                      nfc * (2.0 * nf + 7.0) + (double)c->n_hang * 7.0 * nf);
    }
    return HX_OK;
}

hx_status hx_dof_coordinates(hx_ctx *c, double *xyz)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_mesh) return fail(c, HX_ERR_STATE, "no mesh");
    if (!xyz) return fail(c, HX_ERR_ARG, "null output");
    HX_HIP(c, launch_dof_coords(c, xyz));
    return HX_OK;
}

hx_status hx_set_coefficients(hx_ctx *c, const double *alpha, const double *beta,
                              double penalty_factor, int on_device)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_mesh) return fail(c, HX_ERR_STATE, "set_coefficients before setup_mesh");
    if (!alpha || !beta) return fail(c, HX_ERR_ARG, "null coefficient array");
    if (!(penalty_factor > 0.0) || !std::isfinite(penalty_factor))
        return fail(c, HX_ERR_ARG, "penalty factor must be positive");
    HX_HIP(c, hipSetDevice(c->device));
    const size_t bytes = sizeof(double) * (size_t)c->n_dofs;
    double *da = (double *)alpha, *db = (double *)beta;
    double *tmp = nullptr;
    if (!on_device) {
        hx_status s = dalloc(c, (void **)&tmp, 2 * bytes);
        if (s != HX_OK) return s;
        da = tmp;
        db = tmp + c->n_dofs;
        HX_HIP(c, hipMemcpyAsync(da, alpha, bytes, hipMemcpyHostToDevice, c->stream));
        HX_HIP(c, hipMemcpyAsync(db, beta, bytes, hipMemcpyHostToDevice, c->stream));
    }
    if (penalty_factor != c->P) {
        c->P = penalty_factor;
        HX_HIP(c, launch_face_sigma(c));
        hx_status sh = update_hang_sigma(c);
        if (sh != HX_OK) return sh;
        HX_HIP(c, launch_bj_eigen(c));
    }
    hipError_t e = launch_set_coefficients(c, da, db);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (tmp) dfree((void **)&tmp);
    if (e != hipSuccess) return fail(c, HX_ERR_DEVICE, "set_coefficients: %s", hipGetErrorString(e));
    c->has_coef = true;
    return HX_OK;
}

hx_status hx_set_pressure_system(hx_ctx *c, const double *rho, const double *h, double gamma,
                                 double tau, double penalty_factor, int on_device)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_mesh) return fail(c, HX_ERR_STATE, "set_pressure_system before setup_mesh");
    if (c->n_hang) return fail(c, HX_ERR_STATE, "the pressure system is not built on meshes with hanging faces");
    if (!rho || !h) return fail(c, HX_ERR_ARG, "null field");
    if (!(gamma > 1.0) || !std::isfinite(gamma)) return fail(c, HX_ERR_ARG, "gamma must exceed 1");
    if (!(tau > 0.0) || !std::isfinite(tau)) return fail(c, HX_ERR_ARG, "tau must be positive");
    if (!(penalty_factor > 0.0) || !std::isfinite(penalty_factor))
        return fail(c, HX_ERR_ARG, "penalty factor must be positive");
    HX_HIP(c, hipSetDevice(c->device));
    const int64_t n = c->n_dofs, nc = c->n_cells;
    hx_status s = HX_OK;
    if (!c->psW) {
        auto al = [&](double **p, size_t count) {
            if (s == HX_OK) s = dalloc(c, (void **)p, sizeof(double) * count);
        };
        al(&c->psW, (size_t)nc * 9 * c->nd);
        al(&c->psWC, (size_t)nc * 9 * c->nd);
        al(&c->psMr, (size_t)n);
        al(&c->psMd, (size_t)n);
        al(&c->psFn, (size_t)nc * 18 * c->nf);
        al(&c->psFh, (size_t)nc * 6 * c->nf);
        al(&c->psWork, (size_t)7 * n);
        if (s != HX_OK) return s;
    }
    // fields on the device: [rho, h, alpha, beta]
    double *tmp = nullptr;
    if ((s = dalloc(c, (void **)&tmp, sizeof(double) * 4 * n)) != HX_OK) return s;
    double *dr = tmp, *dh = tmp + n, *al = tmp + 2 * n, *be = tmp + 3 * n;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    hipError_t e = hipMemcpyAsync(dr, rho, sizeof(double) * n, kind, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dh, h, sizeof(double) * n, kind, c->stream);
    if (e == hipSuccess) e = launch_press_setup(c, dr, dh, gamma);
    if (e == hipSuccess) e = blas_fill(c, n, 1.0 / (gamma - 1.0), al);
    if (e == hipSuccess) e = blas_axpby(c, n, tau * tau, dh, 0.0, be);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        dfree((void **)&tmp);
        return fail(c, HX_ERR_DEVICE, "set_pressure_system: %s", hipGetErrorString(e));
    }
    s = hx_set_coefficients(c, al, be, penalty_factor, 1);
    dfree((void **)&tmp);
    if (s != HX_OK) return s;
    c->ps_tau = tau;
    c->has_press = true;
    return HX_OK;
}

hx_status hx_set_consistent(hx_ctx *c, const double *alpha, const double *beta, int on_device)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_coef) return fail(c, HX_ERR_STATE, "set_consistent before set_coefficients");
    if (c->n_hang) return fail(c, HX_ERR_STATE, "consistent integration is not built on meshes with hanging faces");
    if (!alpha || !beta) return fail(c, HX_ERR_ARG, "null coefficient array");
    HX_HIP(c, hipSetDevice(c->device));
    const int64_t n = c->n_dofs, nc = c->n_cells;
    const int nq = 2 * c->n - 1;
    hx_status s = HX_OK;
    if (!c->qcell) {
        if ((s = dalloc(c, (void **)&c->refq, sizeof(RefTabQ))) != HX_OK) return s;
        if ((s = dalloc(c, (void **)&c->qcell, sizeof(double) * nc * 7 * nq * nq * nq)) != HX_OK) return s;
        if ((s = dalloc(c, (void **)&c->qface, sizeof(double) * nc * 3 * 7 * nq * nq)) != HX_OK) return s;
    }
    c->nq = nq;
    RefTabQ tq;
    build_q_tables(c->n, nq, tq);
    double *tmp = nullptr;
    if ((s = dalloc(c, (void **)&tmp, sizeof(double) * 2 * n)) != HX_OK) return s;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    hipError_t e = hipMemcpyAsync(c->refq, &tq, sizeof(RefTabQ), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(tmp, alpha, sizeof(double) * n, kind, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(tmp + n, beta, sizeof(double) * n, kind, c->stream);
    if (e == hipSuccess) e = launch_q_setup(c, tmp, tmp + n);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dfree((void **)&tmp);
    if (e != hipSuccess) return fail(c, HX_ERR_DEVICE, "set_consistent: %s", hipGetErrorString(e));
    c->has_q = true;
    return HX_OK;
}

hx_status hx_apply_consistent(hx_ctx *c, const double *x, double *y)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_q) return fail(c, HX_ERR_STATE, "consistent integration not set up");
    if (!x || !y || x == y) return fail(c, HX_ERR_ARG, "null or aliasing vectors");
    HX_HIP(c, hipSetDevice(c->device));
    HX_HIP(c, launch_apply_q(c, x, y));
    return HX_OK;
}

hx_status hx_apply_pressure_part(hx_ctx *c, int part, const double *in, double *out)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_press) return fail(c, HX_ERR_STATE, "pressure system not set");
    if (!in || !out || in == out) return fail(c, HX_ERR_ARG, "null or aliasing vectors");
    HX_HIP(c, hipSetDevice(c->device));
    const int64_t n = c->n_dofs;
    switch (part) {
    case HX_PS_GRAD: HX_HIP(c, launch_grad(c, in, out)); return HX_OK;
    case HX_PS_DIV: HX_HIP(c, launch_div(c, in, out)); return HX_OK;
    case HX_PS_VMASS_INV:
        for (int e = 0; e < 3; ++e) HX_HIP(c, launch_mass64(c, c->psMr, c->nd, 1, in + e * n, out + e * n));
        return HX_OK;
    case HX_PS_DMASS: HX_HIP(c, launch_mass64(c, c->psMd, c->nd, 0, in, out)); return HX_OK;
    case HX_PS_SYSTEM: HX_HIP(c, press_apply64(c, in, out, nullptr)); return HX_OK;
    default: return fail(c, HX_ERR_ARG, "unknown pressure-system part %d", part);
    }
}

hx_status hx_pressure_rhs(hx_ctx *c, const double *F, const double *G, double *rhs)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_press) return fail(c, HX_ERR_STATE, "pressure system not set");
    if (!F || !G || !rhs || rhs == G) return fail(c, HX_ERR_ARG, "null or aliasing vectors");
    HX_HIP(c, hipSetDevice(c->device));
    const int64_t n = c->n_dofs;
    double *v3 = c->psWork + 3 * n;
    for (int e = 0; e < 3; ++e) HX_HIP(c, launch_mass64(c, c->psMr, c->nd, 1, F + e * n, v3 + e * n));
    HX_HIP(c, launch_div(c, v3, rhs));
    HX_HIP(c, blas_axpby(c, n, 1.0, G, -1.0, rhs));
    return HX_OK;
}

hx_status hx_pressure_velocity(hx_ctx *c, const double *F, const double *P, double *U)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_press) return fail(c, HX_ERR_STATE, "pressure system not set");
    if (!F || !P || !U || U == F) return fail(c, HX_ERR_ARG, "null or aliasing vectors");
    HX_HIP(c, hipSetDevice(c->device));
    const int64_t n = c->n_dofs;
    double *u3 = c->psWork;
    HX_HIP(c, launch_grad(c, P, u3));
    HX_HIP(c, blas_axpby(c, 3 * n, 1.0, F, -1.0, u3));
    for (int e = 0; e < 3; ++e) HX_HIP(c, launch_mass64(c, c->psMr, c->nd, 1, u3 + e * n, U + e * n));
    return HX_OK;
}

hx_status hx_apply_operator(hx_ctx *c, hx_prec prec, const void *x, void *y)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_coef) return fail(c, HX_ERR_STATE, "apply before setup_mesh/set_coefficients");
    if (!x || !y) return fail(c, HX_ERR_ARG, "null vector");
    if (x == y) return fail(c, HX_ERR_ARG, "x and y alias");
    if (prec == HX_F64) HX_HIP(c, launch_apply64(c, (const double *)x, (double *)y, nullptr));
    else if (prec == HX_F32) HX_HIP(c, launch_apply32(c, (const float *)x, (float *)y, nullptr));
    else return fail(c, HX_ERR_ARG, "unknown precision %d", (int)prec);
    return HX_OK;
}

hx_status hx_residual(hx_ctx *c, const double *b, const double *x, double *r)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_coef) return fail(c, HX_ERR_STATE, "residual before setup_mesh/set_coefficients");
    if (!b || !x || !r) return fail(c, HX_ERR_ARG, "null vector");
    if (x == r || b == r) return fail(c, HX_ERR_ARG, "r aliases x or b");
    HX_HIP(c, launch_apply64(c, x, r, b));
    return HX_OK;
}

hx_status hx_apply_operator_part(hx_ctx *c, hx_prec prec, int part, const void *x, void *y)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_coef) return fail(c, HX_ERR_STATE, "apply before set_coefficients");
    if (!x || !y) return fail(c, HX_ERR_ARG, "null vector");
    if (part != HX_PART_CELL && part != HX_PART_FACE) return fail(c, HX_ERR_ARG, "bad part %d", part);
    if (prec == HX_F64)
        HX_HIP(c, launch_apply_part64(c, part, (const double *)x, (double *)y));
    else if (prec == HX_F32)
        HX_HIP(c, launch_apply_part32(c, part, (const float *)x, (float *)y));
    else
        return fail(c, HX_ERR_ARG, "bad precision %d", (int)prec);
    return HX_OK;
}

hx_status hx_apply_preconditioner(hx_ctx *c, hx_pc kind, hx_prec prec, const void *r, void *z)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_coef) return fail(c, HX_ERR_STATE, "preconditioner before set_coefficients");
    if (!r || !z) return fail(c, HX_ERR_ARG, "null vector");
    if (r == z) return fail(c, HX_ERR_ARG, "r and z alias");
    if (prec != HX_F64 && prec != HX_F32) return fail(c, HX_ERR_ARG, "unknown precision");
    const size_t es = prec == HX_F64 ? 8 : 4;
    switch (kind) {
    case HX_PC_NONE:
        HX_HIP(c, hipMemcpyAsync(z, r, es * c->n_dofs, hipMemcpyDeviceToDevice, c->stream));
        return HX_OK;
    case HX_PC_BLOCK_JACOBI:
        if (prec == HX_F64) HX_HIP(c, launch_bj64(c, (const double *)r, (double *)z));
        else HX_HIP(c, launch_bj32(c, (const float *)r, (float *)z));
        return HX_OK;
    case HX_PC_HELMHOLTZ_DIAG:
    case HX_PC_MASS_DIAG: {
        const int which = kind == HX_PC_HELMHOLTZ_DIAG ? 0 : 1;
        if (prec == HX_F64) HX_HIP(c, launch_diag64(c, which, (const double *)r, (double *)z));
        else HX_HIP(c, launch_diag32(c, which, (const float *)r, (float *)z));
        return HX_OK;
    }
    case HX_PC_CHEBYSHEV:
        if (prec != HX_F64) return fail(c, HX_ERR_ARG, "the Chebyshev preconditioner is FP64");
        if (c->cheb_deg < 1) return fail(c, HX_ERR_STATE, "Chebyshev preconditioner not set");
        HX_HIP(c, cheb_apply64(c, (const double *)r, (double *)z));
        return HX_OK;
    case HX_PC_MULTIGRID:
    case HX_PC_MULTIGRID_MIXED: {
        if (prec != HX_F64)
            return fail(c, HX_ERR_ARG, "the multigrid preconditioner takes FP64 vectors");
        const hx_status s = mg_check(c);
        if (s != HX_OK) return s;
        if (kind == HX_PC_MULTIGRID) HX_HIP(c, mg_vcycle64(c, (const double *)r, (double *)z));
        else HX_HIP(c, mg_vcycle_mixed(c, (const double *)r, (double *)z));
        return HX_OK;
    }
    case HX_PC_MASS_BLOCK:
        if (prec == HX_F64) HX_HIP(c, launch_massinv64(c, (const double *)r, (double *)z));
        else HX_HIP(c, launch_massinv32(c, (const float *)r, (float *)z));
        return HX_OK;
    case HX_PC_LEARNED: {
        if (prec != HX_F64) return fail(c, HX_ERR_ARG, "learned preconditioner is FP64-in/out");
        return mlp_precondition(c, (const double *)r, (double *)z);
    }
    default:
        return fail(c, HX_ERR_ARG, "unknown preconditioner %d", (int)kind);
    }
}

hx_status hx_dot(hx_ctx *c, int64_t n, const double *x, const double *y, double *out)
{
    if (!c || !x || !y || !out || n < 0) return c ? fail(c, HX_ERR_ARG, "bad dot arguments") : HX_ERR_ARG;
    HX_HIP(c, blas_dot(c, n, x, y, c->red + 1024 * 70));
    HX_HIP(c, hipMemcpyAsync(out, c->red + 1024 * 70, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HX_HIP(c, hipStreamSynchronize(c->stream));
    return HX_OK;
}

int64_t hx_network_size(const hx_ctx *c) { return c && c->has_mesh ? mlp_param_count(c) : -1; }

hx_status hx_set_network(hx_ctx *c, const float *w, int64_t n)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_mesh) return fail(c, HX_ERR_STATE, "set_network before setup_mesh");
    if (!w) return fail(c, HX_ERR_ARG, "null weights");
    return mlp_set(c, w, n);
}

hx_status hx_get_network(const hx_ctx *c, float *w, int64_t n)
{
    if (!c || !w) return HX_ERR_ARG;
    return mlp_get(c, w, n);
}

hx_status hx_gather_features(hx_ctx *c, const double *r, float *feats, float *scale)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_coef) return fail(c, HX_ERR_STATE, "features before set_coefficients");
    if (!r || !feats || !scale) return fail(c, HX_ERR_ARG, "null pointer");
    return mlp_features(c, r, feats, scale);
}

hx_status hx_training_pair(hx_ctx *c, const double *b, const double *x_star, const double *x_j,
                           float clip, float *feats, float *targets)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_coef) return fail(c, HX_ERR_STATE, "training pair before set_coefficients");
    if (!b || !x_star || !x_j || !feats || !targets) return fail(c, HX_ERR_ARG, "null pointer");
    if (x_j == b) return fail(c, HX_ERR_ARG, "x_j and b alias");
    if (!(clip >= 0.0f)) return fail(c, HX_ERR_ARG, "clip must be >= 0");
    return mlp_training_pair(c, b, x_star, x_j, clip, feats, targets);
}

hx_status hx_network_forward(hx_ctx *c, const float *feats, int64_t batch, float *out)
{
    if (!c) return HX_ERR_ARG;
    if (!feats || !out || batch < 0) return fail(c, HX_ERR_ARG, "bad forward arguments");
    return mlp_forward(c, feats, batch, out);
}

hx_status hx_network_forward_noalloc(hx_ctx *c, const float *feats, int64_t batch, float *out)
{
    if (!c) return HX_ERR_ARG;
    if (!feats || !out || batch < 0) return fail(c, HX_ERR_ARG, "bad forward arguments");
    if (!c->has_mesh) return fail(c, HX_ERR_STATE, "network_forward_noalloc before setup_mesh");
    return mlp_forward_noalloc(c, feats, batch, out);
}

int64_t hx_network_noalloc_max_batch(const hx_ctx *c)
{
    return c && c->has_mesh ? mlp_noalloc_max_batch(c) : -1;
}

hx_status hx_train_step(hx_ctx *c, const float *feats, const float *targets, int64_t batch,
                        float lr, float *loss_out, float *grad_out)
{
    if (!c) return HX_ERR_ARG;
    if (!feats || !targets || batch <= 0) return fail(c, HX_ERR_ARG, "bad training arguments");
    return mlp_train(c, feats, targets, batch, lr, loss_out, grad_out);
}

hx_status hx_network_trace(hx_ctx *c, int what, float *host_buf, int64_t count)
{
    if (!c) return HX_ERR_ARG;
    if (!host_buf || count < 0) return fail(c, HX_ERR_ARG, "null buffer or negative count");
    return mlp_trace(c, what, host_buf, count);
}

hx_status hx_debug_export(hx_ctx *c, int what, void *host_buf, int64_t bytes)
{
    if (!c || !host_buf) return HX_ERR_ARG;
    if (!c->has_mesh) return fail(c, HX_ERR_STATE, "no mesh");
    const void *src = nullptr;
    size_t need = 0;
    const size_t nc = (size_t)c->n_cells;
    switch (what) {
    case HX_EXPORT_CELL_DATA: src = c->cell64; need = sizeof(double) * nc * 7 * c->nd; break;
    case HX_EXPORT_FACE_DATA: src = c->face64; need = sizeof(double) * nc * 3 * 7 * c->nf; break;
    case HX_EXPORT_SIGMA: src = c->sigma; need = sizeof(double) * nc * 3; break;
    case HX_EXPORT_VOLUME: src = c->vol; need = sizeof(double) * nc; break;
    case HX_EXPORT_BJ_SCALARS: src = c->bjC64; need = sizeof(double) * nc * 4; break;
    case HX_EXPORT_INV_DIAG: src = c->dg64; need = sizeof(double) * 2 * nc * c->nd; break;
    default: return fail(c, HX_ERR_ARG, "unknown export %d", what);
    }
    if ((what == HX_EXPORT_CELL_DATA || what == HX_EXPORT_FACE_DATA || what == HX_EXPORT_BJ_SCALARS ||
         what == HX_EXPORT_INV_DIAG) &&
        !c->has_coef)
        return fail(c, HX_ERR_STATE, "no coefficients");
    if (bytes < (int64_t)need) return fail(c, HX_ERR_ARG, "buffer too small (%zu needed)", need);
    HX_HIP(c, hipMemcpyAsync(host_buf, src, need, hipMemcpyDeviceToHost, c->stream));
    HX_HIP(c, hipStreamSynchronize(c->stream));
    return HX_OK;
}

}  // extern "C"
