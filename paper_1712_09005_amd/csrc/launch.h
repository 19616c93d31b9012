// Host-side launch entry points of the kernels (one per kernel kind).  Each
// takes the compile-time configuration as runtime values and dispatches to
// the matching template instance.
#pragma once

#include <hip/hip_runtime.h>

#include "tsne_dev.h"

namespace tsne {

struct Cfg {
    int dtype;   // 0 float, 1 double
    int s;       // 1, 2
    int p;       // 2..6
    int form;    // 0 A, 1 B, 2 V
    int lpr;     // CSR lanes per row
};

struct CallArgs {
    const void* Yin;
    void* Y;
    void* uY;
    void* gains;
    void* Frep;
    double* Zout;
    void* Fattr;
    double* KLout;
    const int64_t* row_ptr;
    const int32_t* col;
    const void* val;
    double tscale;  // fixed-point scale of the tiled attraction's row sums
    int set_ptrs;   // copy the pointer fields
    int set_P;      // copy row_ptr/col/val and tscale
    int set_iter;   // write *iter = iter
    int iter;
    int set_end;    // write iter_end
    int iter_end;
    int set_sched;  // write *sched
    Sched sched;
    int counting;   // geometry kernel advances the iteration counter
};

// Grid geometry of one launch.
struct Launch {
    int grid;
    int block;
    size_t lds;
};

hipError_t launch_set_args(Inst* inst, const CallArgs& a, hipStream_t st);
hipError_t launch_pack_cv(const int32_t* col, const float* val, void* cv, int64_t nnz, hipStream_t st);
hipError_t launch_kind(int kind, const Cfg& c, const LaunchMap& map, const Launch& l,
                       hipStream_t st);

}  // namespace tsne
