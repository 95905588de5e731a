// Host export of the F quantile routine (hk_fquant.h) for tests of the critical value.
#include "hk_fquant.h"
#include "hk.h"

extern "C" double hk_f_quantile(double d1, double d2, double alpha)
{
    return hk::f_quantile(d1, d2, alpha);
}
