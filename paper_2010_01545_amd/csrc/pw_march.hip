// pw_march.hip -- x-marching kernels (placeholder: not yet available).
#include "pw_internal.h"

template <typename T>
bool march_supported(const Geom&)
{
    return false;
}

template <typename T>
void launch_fwd_march(const FwdArgs<T>&, const Geom&, hipStream_t)
{
}

template <typename T>
void launch_adj_march(const AdjArgs<T>&, const Geom&, hipStream_t)
{
}

template bool march_supported<double>(const Geom&);
template bool march_supported<float>(const Geom&);
template void launch_fwd_march<double>(const FwdArgs<double>&, const Geom&, hipStream_t);
template void launch_fwd_march<float>(const FwdArgs<float>&, const Geom&, hipStream_t);
template void launch_adj_march<double>(const AdjArgs<double>&, const Geom&, hipStream_t);
template void launch_adj_march<float>(const AdjArgs<float>&, const Geom&, hipStream_t);
