// The served gather/scatter kernels, compiled for the CPU stand-in runtime.
// TEST INFRASTRUCTURE ONLY.
#include "../../paper_1805_00106_amd/csrc/sw_serve.hip"
