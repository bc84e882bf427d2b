// State-averaged PNO machinery (placeholder until the grouped kernels land).
#include "context.h"

namespace pnoeom {

void build_sapno(Context&, int, double, double) {
  throw Error(PNOEOM_EINVAL, "SA-PNO build is not available in this build");
}
void pno_compress(Context&, int, const double*, const double*, double*) {
  throw Error(PNOEOM_ESTATE, "PNO compress before build_sapno");
}
void pno_expand(Context&, int, const double*, double*, double*) {
  throw Error(PNOEOM_ESTATE, "PNO expand before build_sapno");
}
void sigma_pno(Context&, int, const double*, double*, int) {
  throw Error(PNOEOM_ESTATE, "PNO sigma before build_sapno");
}
void precond_pno(Context&, double*, double) { throw Error(PNOEOM_ESTATE, "PNO preconditioner before build_sapno"); }
void project_pno(Context&, double*) { throw Error(PNOEOM_ESTATE, "PNO projector before build_sapno"); }

}  // namespace pnoeom
