// Host-side construction of the fixed superset pattern and of the maps the
// kernels use (paper Sec. 3.3: "precomputed tetrahedron-to-edge incidence";
// here the elasticity analogue, tet -> 3x3 node blocks).
//
// Blocks.  Every node that lies in some candidate tet owns a diagonal block
// (i,i); every node pair i<j that shares a candidate tet owns an off-diagonal
// block (i,j).  A block's incidence segment lists the candidate tets that
// contribute to it in ascending tet id; this order is the summation order of
// every entry, in the rebuild and in the streaming update alike.
//
// CSR, for node blocks of size bs (3 for elasticity, 1 for the scalar proxy
// operator).  Row bs*i+p has the columns bs*j+q of every neighbour j of i
// (i itself included) in ascending order, so the bs rows of node i share one
// column list of length bs*deg(i).  A block's values therefore sit at
//   up + p*rowlen(i) + q            (upper block, row node i)
//   lo + q*rowlen(j) + p            (its mirror, row node j)
// with up / lo the CSR index of entry (bs*i,bs*j) / (bs*j,bs*i).
#include <algorithm>
#include <cstring>

#include "sta_internal.h"

namespace sta {

namespace {
const int kPairA[6] = {0, 0, 0, 1, 1, 2};
const int kPairB[6] = {1, 2, 3, 2, 3, 3};
}  // namespace

std::string build_host_pattern(int64_t n, const int32_t* tets, int64_t m, HostPattern& P, int bs)
{
    // diagonal blocks: used nodes in ascending id
    std::vector<int32_t> did(n, -1);
    for (int64_t e = 0; e < m; ++e)
        for (int a = 0; a < 4; ++a)
            did[tets[4 * e + a]] = 0;
    int64_t nd = 0;
    for (int64_t i = 0; i < n; ++i)
        if (did[i] == 0)
            did[i] = (int32_t)nd++;

    // off-diagonal blocks: sorted unique (min, max) node pairs
    std::vector<uint64_t> keys((size_t)m * 6);
    for (int64_t e = 0; e < m; ++e)
        for (int p = 0; p < 6; ++p) {
            uint64_t a = (uint32_t)tets[4 * e + kPairA[p]], b = (uint32_t)tets[4 * e + kPairB[p]];
            uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
            keys[6 * e + p] = (lo << 32) | hi;
        }
    std::vector<uint64_t> okeys(keys);
    std::sort(okeys.begin(), okeys.end());
    okeys.erase(std::unique(okeys.begin(), okeys.end()), okeys.end());
    const int64_t no = (int64_t)okeys.size();
    if (nd > INT32_MAX || no > INT32_MAX || 6 * m > INT32_MAX)
        return "mesh too large for 32-bit block indices";

    // element -> block ids, and segment sizes
    P.e2b.assign((size_t)m * 10, 0);
    std::vector<int64_t> dcount(nd + 1, 0), ocount(no + 1, 0);
    for (int64_t e = 0; e < m; ++e) {
        for (int a = 0; a < 4; ++a) {
            int32_t b = did[tets[4 * e + a]];
            P.e2b[10 * e + a] = b;
            dcount[b + 1]++;
        }
        for (int p = 0; p < 6; ++p) {
            int32_t b = (int32_t)(std::lower_bound(okeys.begin(), okeys.end(), keys[6 * e + p]) - okeys.begin());
            P.e2b[10 * e + 4 + p] = b;
            ocount[b + 1]++;
        }
    }
    P.dseg.assign(nd + 1, 0);
    P.oseg.assign(no + 1, 0);
    for (int64_t b = 0; b < nd; ++b)
        P.dseg[b + 1] = (int32_t)(P.dseg[b] + dcount[b + 1]);
    for (int64_t b = 0; b < no; ++b)
        P.oseg[b + 1] = (int32_t)(P.oseg[b] + ocount[b + 1]);

    // incidences in ascending element id within each segment (counting sort)
    P.dinc.assign((size_t)m * 4, 0);
    P.oinc.assign((size_t)m * 6, 0);
    P.e2p.assign((size_t)m * 10, 0);
    std::vector<int32_t> dfill(P.dseg.begin(), P.dseg.end() - 1), ofill(P.oseg.begin(), P.oseg.end() - 1);
    for (int64_t e = 0; e < m; ++e) {
        for (int a = 0; a < 4; ++a) {
            int32_t b = P.e2b[10 * e + a];
            int32_t k = dfill[b]++;
            P.dinc[k] = (int32_t)e;
            P.e2p[10 * e + a] = k;
        }
        for (int p = 0; p < 6; ++p) {
            int32_t b = P.e2b[10 * e + 4 + p];
            int32_t k = ofill[b]++;
            P.oinc[k] = (int32_t)e;
            P.e2p[10 * e + 4 + p] = k;
        }
    }

    // node adjacency (self included), ascending
    std::vector<int64_t> deg(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        deg[i + 1] = did[i] >= 0 ? 1 : 0;
    for (uint64_t k : okeys) {
        deg[(k >> 32) + 1]++;
        deg[(k & 0xffffffffu) + 1]++;
    }
    std::vector<int64_t> aoff(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        aoff[i + 1] = aoff[i] + deg[i + 1];
    std::vector<int32_t> adj((size_t)aoff[n]);
    std::vector<int64_t> afill(aoff.begin(), aoff.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        if (did[i] >= 0)
            adj[afill[i]++] = (int32_t)i;
    for (uint64_t k : okeys) {
        int64_t i = (int64_t)(k >> 32), j = (int64_t)(k & 0xffffffffu);
        adj[afill[i]++] = (int32_t)j;
        adj[afill[j]++] = (int32_t)i;
    }
    for (int64_t i = 0; i < n; ++i)
        std::sort(adj.begin() + aoff[i], adj.begin() + aoff[i + 1]);

    // CSR
    int64_t nnz = 0;
    for (int64_t i = 0; i < n; ++i)
        nnz += (int64_t)bs * bs * (aoff[i + 1] - aoff[i]);
    if (nnz > INT32_MAX)
        return "pattern has more than 2^31-1 entries";
    P.nnz = nnz;
    P.rowptr.assign((size_t)bs * n + 1, 0);
    P.colidx.assign((size_t)nnz, 0);
    int64_t at = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t d = aoff[i + 1] - aoff[i];
        for (int p = 0; p < bs; ++p) {
            P.rowptr[bs * i + p] = (int32_t)at;
            for (int64_t s = 0; s < d; ++s)
                for (int q = 0; q < bs; ++q)
                    P.colidx[at++] = bs * adj[aoff[i] + s] + q;
        }
    }
    P.rowptr[bs * n] = (int32_t)at;

    auto pos = [&](int64_t i, int64_t j) -> int64_t {
        auto b = adj.begin() + aoff[i], e = adj.begin() + aoff[i + 1];
        return std::lower_bound(b, e, (int32_t)j) - b;
    };
    P.dmeta.assign((size_t)nd * 2, 0);
    for (int64_t i = 0; i < n; ++i) {
        if (did[i] < 0)
            continue;
        const int64_t b = did[i];
        P.dmeta[2 * b + 0] = (int32_t)(P.rowptr[bs * i] + bs * pos(i, i));
        P.dmeta[2 * b + 1] = (int32_t)(bs * (aoff[i + 1] - aoff[i]));
    }
    P.ometa.assign((size_t)no * 4, 0);
    P.opair.assign((size_t)no * 2, 0);
    for (int64_t b = 0; b < no; ++b) {
        const int64_t i = (int64_t)(okeys[b] >> 32), j = (int64_t)(okeys[b] & 0xffffffffu);
        P.opair[2 * b + 0] = (int32_t)i;
        P.opair[2 * b + 1] = (int32_t)j;
        P.ometa[4 * b + 0] = (int32_t)(P.rowptr[bs * i] + bs * pos(i, j));
        P.ometa[4 * b + 1] = (int32_t)(bs * (aoff[i + 1] - aoff[i]));
        P.ometa[4 * b + 2] = (int32_t)(P.rowptr[bs * j] + bs * pos(j, i));
        P.ometa[4 * b + 3] = (int32_t)(bs * (aoff[j + 1] - aoff[j]));
    }
    P.ndiag.assign(did.begin(), did.end());
    P.nd = nd;
    P.no = no;
    return "";
}

}  // namespace sta
