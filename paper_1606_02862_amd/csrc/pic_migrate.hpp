// Supercell migration, shared by the standalone migration kernel and the
// particle kernel (which absorbs the previous step's arrivals before pushing).
//
// Each supercell closes the holes its leavers left and takes in the particles
// that arrived from its 26 neighbours, keeping its frames dense (slots
// [0, count) occupied).  Only leavers, arrivals and at most as many tail
// particles are touched.
//
// With n particles, h holes and m arrivals the new count is n' = n - h + m.
// Vacancies are the holes below n' plus the slots [n, n') when the supercell
// grows; sources are the surviving particles at or above n' plus every
// arrival.  The two lists have equal length and the k-th source (the
// survivors, then arrival 0, 1, ...) moves into the k-th vacancy; no source
// slot is also a destination, so the moves are independent.  Each thread
// loads its first arrival while the holes are classified.
#pragma once

#include "pic_device.hpp"

namespace pic {

// Arrival list of supercell `sc` for step parity `par`.
template <class R>
__device__ inline int64_t inbox_index(const SpeciesViewT<R>& s, int nsc, int par, int sc, int k)
{
    return ((int64_t)par * nsc + sc) * s.cap_in + k;
}

// Whole-workgroup call (contains barriers).  Scratch: 3 * cap_in ints plus
// ceil(cap_in / 32) words; counters: 3 ints.  Returns the new count.
template <int NT, class R>
__device__ inline int fill_supercell(const GridViewT<R>& g, const SpeciesViewT<R>& s, int sc, int par, int* scratch,
                                     int* counters)
{
    int* s_hole = scratch;
    int* s_vac = s_hole + s.cap_in;
    int* s_src = s_vac + s.cap_in;
    unsigned* s_mark = (unsigned*)(s_src + s.cap_in);
    const int tid = threadIdx.x;
    const int n = s.count[sc];
    const int h = s.hole_count[sc];
    int m = s.in_count[par * g.nsc + sc];
    if (m > s.cap_in) m = s.cap_in;  // overflow already flagged by the particle kernel
    int np = n - h + m;
    if (np > s.cap) {                // frames full: drop the excess arrivals and report
        if (tid == 0) g.flags[FLAG_CAPACITY] = 1;
        m -= np - s.cap;
        np = s.cap;
    }
    // the first NT arrivals, loaded while the holes are classified
    R pfx = R(0), pfy = R(0), pfz = R(0), pfux = R(0), pfuy = R(0), pfuz = R(0), pfw = R(0);
    uint32_t pfid = 0;
    uint8_t pfzs = 0;
    if (tid < m) {
        const int64_t q = inbox_index(s, g.nsc, par, sc, tid);
        pfx = s.ix[q]; pfy = s.iy[q]; pfz = s.iz[q];
        pfux = s.iux[q]; pfuy = s.iuy[q]; pfuz = s.iuz[q];
        pfw = s.iw[q]; pfid = s.iid[q];
        if (s.zs) pfzs = s.izs[q];
    }
    const int lo = np < n ? np : n;  // survivors at or above n' must move down
    const int nmark = n - lo;        // <= h

    if (tid == 0) { counters[0] = 0; counters[1] = 0; }
    for (int t = tid; t < (nmark + 31) / 32; t += NT) s_mark[t] = 0u;
    for (int t = tid; t < h; t += NT) s_hole[t] = s.holes[(int64_t)sc * s.cap_in + t];
    __syncthreads();

    for (int t = tid; t < h; t += NT) {
        const int hv = s_hole[t];
        if (hv < np) s_vac[atomicAdd(&counters[0], 1)] = hv;
        else if (hv < n) atomicOr(&s_mark[(hv - lo) >> 5], 1u << ((hv - lo) & 31));
    }
    __syncthreads();
    const int nv_holes = counters[0];
    for (int t = tid; t < nmark; t += NT) {
        if (!(s_mark[t >> 5] & (1u << (t & 31)))) s_src[atomicAdd(&counters[1], 1)] = lo + t;
    }
    __syncthreads();
    const int ns_surv = counters[1];
    for (int t = n + tid; t < np; t += NT) s_vac[nv_holes + (t - n)] = t;
    const int total = ns_surv + m;
    const int nvac = nv_holes + (np > n ? np - n : 0);
    if (tid == 0 && nvac != total) g.flags[FLAG_CAPACITY] = 1;  // cannot happen with consistent inputs
    __syncthreads();

    const int64_t base = (int64_t)sc * s.cap;
    const int nmove = nvac < total ? nvac : total;
    const int nsv = ns_surv < nmove ? ns_surv : nmove;
    for (int t = tid; t < nsv; t += NT) {  // survivors
        const int64_t d = base + s_vac[t];
        const int64_t q = base + s_src[t];
        s.x[d] = s.x[q]; s.y[d] = s.y[q]; s.z[d] = s.z[q];
        s.ux[d] = s.ux[q]; s.uy[d] = s.uy[q]; s.uz[d] = s.uz[q];
        s.w[d] = s.w[q]; s.id[d] = s.id[q];
        if (s.zs) s.zs[d] = s.zs[q];
    }
    for (int a = tid; a < nmove - nsv; a += NT) {  // arrival a into vacancy nsv + a
        const int64_t d = base + s_vac[nsv + a];
        if (a == tid) {
            s.x[d] = pfx; s.y[d] = pfy; s.z[d] = pfz;
            s.ux[d] = pfux; s.uy[d] = pfuy; s.uz[d] = pfuz;
            s.w[d] = pfw; s.id[d] = pfid;
            if (s.zs) s.zs[d] = pfzs;
        } else {
            const int64_t q = inbox_index(s, g.nsc, par, sc, a);
            s.x[d] = s.ix[q]; s.y[d] = s.iy[q]; s.z[d] = s.iz[q];
            s.ux[d] = s.iux[q]; s.uy[d] = s.iuy[q]; s.uz[d] = s.iuz[q];
            s.w[d] = s.iw[q]; s.id[d] = s.iid[q];
            if (s.zs) s.zs[d] = s.izs[q];
        }
    }
    __syncthreads();  // moves visible to the whole workgroup; scratch free again
    if (tid == 0) {
        s.count[sc] = np;
        s.in_count[par * g.nsc + sc] = 0;
        s.hole_count[sc] = 0;
    }
    return np;
}

}  // namespace pic
