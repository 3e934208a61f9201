// Internal declarations of the thermal solve: the assembly of eq.
// wf_thermal (te_assemble.hip) and the classical AMG, CG and Newton driver
// that use it (te_camg.hip).
#pragma once

#include "te_internal.h"
#include "te_setup_gpu.h"

namespace te {

// node -> (cell, local index) incidence, entries cell * npe + local,
// ascending per node
struct Incidence {
    DBuf<int64_t> start;  // [N+1]
    DBuf<int64_t> inc;    // [C*npe]
};

// Everything the thermal assembly needs, owned by the solver: copies of the
// mesh and the boundary data, the incidences and the pattern of J.
struct ThermalAsm {
    int64_t n = 0, nc = 0;
    int degree = 1, npe = 4, npf = 3, nm = 0, np = 0;
    DBuf<double> coords;          // [N][3]
    DBuf<int32_t> cells;          // [C][npe]
    DBuf<int32_t> cell_material;  // [C]
    DBuf<double> tab;             // [3][nm][np]: T, kappa, cv
    DBuf<double> rho;             // [nm]
    int64_t n_faces = 0;
    DBuf<int32_t> faces;          // [F][npf]
    DBuf<double> h, T_bc;         // [F]
    Incidence I;                  // node -> cells
    DBuf<int64_t> fptr, fent;     // node -> (face, local) entries in face order
    DBuf<int64_t> ptr;            // pattern of J: node coupling
    DBuf<int32_t> col;
    int64_t nnz = 0;
};

// Validates and copies the inputs, builds the incidences and the pattern.
void thermal_asm_init(ThermalAsm &ta, const te_mesh *m, const te_thermal_tables *tab, const int32_t *cell_material,
                      const te_robin *robin, hipStream_t s);
// F [N] and J's values [nnz] (pattern ta.ptr / ta.col) at T; T_old == NULL
// or dt <= 0: steady (no time term).
void thermal_asm_run(const ThermalAsm &ta, const double *T, const double *T_old, double dt, double *Jval, double *F,
                     hipStream_t s);

}  // namespace te
