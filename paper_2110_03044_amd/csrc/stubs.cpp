// Entry points not implemented yet: they fail with FL_E_UNSUPPORTED.
#include "fl_internal.h"

using namespace fl;

extern "C" {
fl_status fl_batch_create(int, fl_mesh *const *, const int *, const int *, const double *, int,
                          double *const *, const double *const *, int, int, fl_batch **) {
    return fail(FL_E_UNSUPPORTED, "not implemented");
}
fl_status fl_batch_step(fl_batch *, int, void *) { return fail(FL_E_UNSUPPORTED, "not implemented"); }
fl_status fl_batch_step_unbatched(fl_batch *, int, void *) {
    return fail(FL_E_UNSUPPORTED, "not implemented");
}
fl_status fl_batch_tile(const fl_batch *, int *) { return fail(FL_E_UNSUPPORTED, "not implemented"); }
fl_status fl_batch_destroy(fl_batch *) { return FL_OK; }
}
