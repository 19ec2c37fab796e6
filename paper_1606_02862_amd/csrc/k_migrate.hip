// Standalone supercell migration (see pic_migrate.hpp): run once at the end
// of every pic_step call so that the frames are dense for any reader.  Within
// a call, each step's particle kernel absorbs the previous step's arrivals.
#include "pic_migrate.hpp"

namespace pic {

template <class R>
__global__ __launch_bounds__(BLOCK) void k_migrate(GridViewT<R> g, SpeciesViewT<R> s, int par)
{
    extern __shared__ int lds[];
    __shared__ int counters[3];
    const int sc = sc_of_block(blockIdx.x, g.nsc, g.ncx * g.ncy, g.xcd_remap);
    fill_supercell<BLOCK>(g, s, sc, par, lds, counters);
}

template <class R>
hipError_t launch_migrate(const GridViewT<R>& g, const SpeciesViewT<R>& s, int par, hipStream_t st)
{
    const size_t lds = (size_t)3 * s.cap_in * sizeof(int) + ((size_t)s.cap_in + 31) / 32 * sizeof(unsigned);
    hipLaunchKernelGGL(k_migrate<R>, dim3(g.nsc), dim3(BLOCK), lds, st, g, s, par);
    return hipGetLastError();
}

template hipError_t launch_migrate<float>(const GridView&, const SpeciesView&, int, hipStream_t);
template hipError_t launch_migrate<double>(const GridView64&, const SpeciesView64&, int, hipStream_t);

}  // namespace pic
