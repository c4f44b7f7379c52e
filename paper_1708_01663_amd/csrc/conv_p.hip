// Kernels of the FFT-convolution operator for one transform length, chosen
// at compile time by -DCISOR_P=<length> (the build compiles this file once
// per length in CISOR_FFT_SIZES, so the lengths build in parallel).
#include "conv_kernels.hpp"

#ifndef CISOR_P
#error "CISOR_P (transform length) must be defined"
#endif

namespace cisor {

#define CISOR_INST_P(Rs, Rc)                                                                        \
  template int launch_conv_p<Rs, Rc, CISOR_P, PRO_X, EPI_AX>(Ctx &, ConvArgs<Rs, Rc> &, bool);     \
  template int launch_conv_p<Rs, Rc, CISOR_P, PRO_X, EPI_TR>(Ctx &, ConvArgs<Rs, Rc> &, bool);     \
  template int launch_conv_p<Rs, Rc, CISOR_P, PRO_X, EPI_G>(Ctx &, ConvArgs<Rs, Rc> &, bool);      \
  template int launch_conv_p<Rs, Rc, CISOR_P, PRO_X, EPI_GF>(Ctx &, ConvArgs<Rs, Rc> &, bool);     \
  template int launch_conv_p<Rs, Rc, CISOR_P, PRO_X, EPI_GRAD>(Ctx &, ConvArgs<Rs, Rc> &, bool);   \
  template int launch_conv_p<Rs, Rc, CISOR_P, PRO_PUPD, EPI_V>(Ctx &, ConvArgs<Rs, Rc> &, bool);   \
  template int launch_conv_p<Rs, Rc, CISOR_P, PRO_SUPD, EPI_T>(Ctx &, ConvArgs<Rs, Rc> &, bool);   \
  template int launch_stage_p<Rs, Rc, CISOR_P>(Ctx &, ConvArgs<Rs, Rc> &, int, bool);
CISOR_INST_P(float, float)
CISOR_INST_P(double, double)
template int launch_conv_p<float, double, CISOR_P, PRO_X, EPI_TR>(Ctx &, ConvArgs<float, double> &, bool);

}  // namespace cisor
