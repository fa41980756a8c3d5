// The tetrahedral (three-dimensional) path of the library: a context of its
// own behind the same C ABI entry points (hdgmg.h), selected by
// hdgmg_mesh.dim == 3.
#pragma once
#include <string>

#include "../../include/hdgmg.h"

namespace hdgmg {

struct Ctx3;

// Set-up of the hierarchy, topology, edge patches and transfers' averaging
// part; device memory through alloc_fn / free_fn (null: hipMalloc).
hdgmg_status d3_setup(const hdgmg_mesh* mesh, int k, double beta, const double* nu, int nu_len, double gamma,
                      const hdgmg_opts* opts, void* stream, hdgmg_alloc_fn alloc_fn, hdgmg_free_fn free_fn,
                      void* alloc_ctx, Ctx3** out, std::string& err);
void d3_destroy(Ctx3* c);
const char* d3_error(const Ctx3* c);
hdgmg_status d3_assemble(Ctx3* c);
hdgmg_status d3_solve(Ctx3* c, const double* f_qp, const double* x0, double* u_qp, double* p_qp, double* state,
                      hdgmg_info* info);
hdgmg_status d3_rhs(Ctx3* c, const double* f_qp, double* g);
hdgmg_status d3_apply(Ctx3* c, const double* x, double* y);
hdgmg_status d3_precondition(Ctx3* c, const double* r, double* z);
// sc / part: the Krylov scalars and partials (null: the context's own)
hdgmg_status d3_inner_solve(Ctx3* c, const double* b, double* x, int* its, double* rel_res, double* sc,
                            double* part);
hdgmg_status d3_recover(Ctx3* c, const double* f_qp, const double* state, double* u_qp, double* p_qp);
hdgmg_status d3_query(const Ctx3* c, int what, int level, int64_t* value);
hdgmg_status d3_export(const Ctx3* c, int what, int level, void* dst, size_t bytes);
hdgmg_status d3_kernel_timer(Ctx3* c, int cls, int enable);
hdgmg_status d3_kernel_timer_read(Ctx3* c, int cls, double* total_ms, int64_t* launches, double* bytes);

}  // namespace hdgmg
