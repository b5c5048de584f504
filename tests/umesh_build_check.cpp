// Host entry points over the library's unstructured-mesh construction
// (paper_2008_11520_amd/csrc/umesh_build.h) for the CPU test that compares it
// with the FP64 reference implementation: built as a small shared library.
#include "umesh_build.h"

#include <cstring>

using namespace dnnmg;

static std::string g_err;

extern "C" const char *ub_error() { return g_err.c_str(); }

extern "C" int ub_counts(int nc, int ne, const double *xy, const int *elems, int ndir, const int *dirs, int ncirc,
                         const double *circ, int ncurved, const int *curved, int K, int *E, int *Fn)
{
    UMeshHost m;
    g_err = build_umesh(nc, ne, xy, elems, ndir, dirs, ncirc, circ, ncurved, curved, K, m);
    if (!g_err.empty()) return 1;
    *E = m.E;
    *Fn = m.Fn;
    return 0;
}

extern "C" int ub_build(int nc, int ne, const double *xy, const int *elems, int ndir, const int *dirs, int ncirc,
                        const double *circ, int ncurved, const int *curved, int K, int *pmap, double *fxy,
                        double *rel, unsigned char *mask, int *node_ptr, int *node_occ, int *cnode_ptr,
                        int *cnode_occ, float *feat)
{
    UMeshHost m;
    g_err = build_umesh(nc, ne, xy, elems, ndir, dirs, ncirc, circ, ncurved, curved, K, m);
    if (!g_err.empty()) return 1;
    std::memcpy(pmap, m.pmap.data(), sizeof(int) * m.pmap.size());
    std::memcpy(fxy, m.fxy.data(), sizeof(double) * m.fxy.size());
    std::memcpy(rel, m.rel.data(), sizeof(double) * m.rel.size());
    std::memcpy(mask, m.mask.data(), m.mask.size());
    std::memcpy(node_ptr, m.node_ptr.data(), sizeof(int) * m.node_ptr.size());
    std::memcpy(node_occ, m.node_occ.data(), sizeof(int) * m.node_occ.size());
    std::memcpy(cnode_ptr, m.cnode_ptr.data(), sizeof(int) * m.cnode_ptr.size());
    std::memcpy(cnode_occ, m.cnode_occ.data(), sizeof(int) * m.cnode_occ.size());
    std::memcpy(feat, m.feat.data(), sizeof(float) * m.feat.size());
    return 0;
}
