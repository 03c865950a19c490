// FP32 instantiation of the batched kernels and their launchers.
#include "sk_launch_impl.h"
template struct SkLaunch<float>;
