// CP-ALS dense steps (Algorithm 1): Gram products, the R x R float64 solve,
// row solve with column normalisation, and the fit.
#include "fcoo_internal.h"

extern "C" {

int fcoo_gram(fcoo_tensor *t, int mode, const void *A, int dtype, int R, double *G, void *stream)
{
    (void)t; (void)mode; (void)A; (void)dtype; (void)R; (void)G; (void)stream;
    return fcoo::fail(FCOO_EUNSUPPORTED, "fcoo_gram: not available in this build");
}

int fcoo_cp_als_iter(fcoo_tensor *t, void *const *factors, int dtype, int R, double *lambda,
                     double *grams, int grams_valid, double *fit, int *used_pinv, void *stream)
{
    (void)t; (void)factors; (void)dtype; (void)R; (void)lambda; (void)grams; (void)grams_valid;
    (void)fit; (void)used_pinv; (void)stream;
    return fcoo::fail(FCOO_EUNSUPPORTED, "fcoo_cp_als_iter: not available in this build");
}

}
