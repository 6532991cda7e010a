// Internal layout of a stafem context: host bookkeeping plus the device
// buffers the kernels read and write.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "stafem.h"

namespace sta {

// Device-detected error bits (Ctl::ferr / Ctl::err).
enum : int32_t {
    ERR_RANGE = 1,       // edit id out of range or state not in {0, 1}
    ERR_DUP = 2,         // the same tet twice in one edit list
    ERR_DEGENERATE = 4,  // det == 0 in an element
};

// Control words kept in device memory so that a frame never needs the host
// (and can be replayed from a captured graph).
struct Ctl {
    uint32_t epoch;      // frames started; stamps equal to epoch+1 belong to the frame in flight
    int32_t ferr;        // error bits of the frame in flight (edit kernel)
    int32_t frame_err;   // error bits of the last finished edit phase (read by the reduce phase)
    int32_t err;         // sticky error bits, cleared by sta_status_sync
    uint32_t done;       // edit-phase workgroups finished (last one publishes and resets)
    int32_t pad[3];
};

// Material constants, evaluated once on the host in the fixed order.
struct Material {
    double cdt;   // dt*dt
    double clam;  // nu / ((1+nu)*(1-2nu))
    double cmu;   // 0.5 / (1+nu)
    double rho;
};

// Everything the kernels need, passed by value.
struct DevView {
    int32_t n_nodes, n_tets;
    int32_t nd, no;               // diagonal / off-diagonal 3x3 blocks
    const double* xs;             // SoA node coordinates
    const double* ys;
    const double* zs;
    const int4* T;                // tets
    const double* E;
    uint8_t* mask;
    // diagonal blocks: segment offsets into dinc, element id per incidence,
    // (CSR index of entry (3i,3i), row length 3*deg(i))
    const int32_t* dseg;
    const int32_t* dinc;
    const int2* dmeta;
    // off-diagonal blocks (i<j): (CSR index of (3i,3j), row length of i,
    // CSR index of (3j,3i), row length of j)
    const int32_t* oseg;
    const int32_t* oinc;
    const int4* ometa;
    // per element: 4 diagonal then 6 off-diagonal block ids / incidence positions,
    // local pair order 00 11 22 33 | 01 02 03 12 13 23
    const int32_t* e2b;
    const int32_t* e2p;
    double* cd;                   // 6 unique values per diagonal incidence
    double* co;                   // 9 values per off-diagonal incidence (block orientation)
    uint32_t* cver;               // parameter version each element's contribution was computed at
    double* values;               // CSR values
    // streaming state
    uint32_t* estamp;             // per tet: epoch of the last edit naming it
    uint32_t* dstamp;             // per diagonal block: epoch of the last claim
    uint32_t* ostamp;             // per off-diagonal block
    int32_t* claims;              // per edit: 10 claimed block ids (or -1)
    uint8_t* undo;                // per edit: previous mask value, 0xFF = nothing to undo
    Ctl* ctl;
    Material mat;
};

struct DevBuffers {
    std::vector<void*> owned;
};

}  // namespace sta

struct sta_ctx {
    int64_t n_nodes = 0, n_tets = 0, n_rows = 0, nnz = 0, nd = 0, no = 0;
    double nu = 0, rho = 0, dt = 0;
    uint32_t ver = 1;     // parameter version
    bool stale = false;
    int64_t last_n_edits = 0;
    int device = 0;
    sta::DevView v{};
    int32_t* rowptr = nullptr;  // device
    int32_t* colidx = nullptr;  // device
    std::vector<void*> owned;   // every device allocation
    // host copies for statistics
    std::vector<int32_t> h_dseg, h_oseg;
    std::string errmsg;
};

namespace sta {

// Kernel launchers (assembly.hip).
hipError_t launch_element(const DevView& v, bool all_tets, uint32_t ver, hipStream_t s);
hipError_t launch_reduce_all(const DevView& v, hipStream_t s);
hipError_t launch_edits(const DevView& v, const int32_t* ids, const uint8_t* states, int32_t n,
                        uint32_t ver, hipStream_t s);
hipError_t launch_set_params(const DevView& v, const double* x_aos, const double* E, double* xs, double* ys,
                             double* zs, double* Eout, hipStream_t s);

// Host pattern builder (pattern.cpp).  Fills host arrays; returns "" or an error message.
struct HostPattern {
    int64_t nd = 0, no = 0, nnz = 0;
    std::vector<int32_t> rowptr, colidx;
    std::vector<int32_t> dseg, dinc, oseg, oinc;
    std::vector<int32_t> dmeta;  // 2 per block
    std::vector<int32_t> ometa;  // 4 per block
    std::vector<int32_t> e2b, e2p;  // 10 per element
};
std::string build_host_pattern(int64_t n_nodes, const int32_t* tets, int64_t n_tets, HostPattern& P);

}  // namespace sta
