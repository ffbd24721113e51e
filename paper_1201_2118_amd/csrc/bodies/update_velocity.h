// update_velocity.h -- per-cell body of the generated UPDATE_VELOCITY kernel
// (the paper's velocity-update kernel): the projection u = F - dt grad p on
// the unknowns of each component.  F, G, H are the "in" level of the
// velocity, u, v, w its "out" level; p is cached with a one-cell halo on the
// + side of each axis.  The same expressions as the hand-written projection.
#pragma once

namespace ns {
namespace gen {

template <class K>
__device__ __forceinline__ void UPDATE_VELOCITY_body(const K& x) {
  const double dt = x.dt;
  const double pc = x.p();
  if (x.i <= x.g.hi[0]) x.store_u((double)x.u_in() - dt * (x.p(1, 0, 0) - pc) * x.g.idx);
  if (x.j <= x.g.hi[1]) x.store_v((double)x.v_in() - dt * (x.p(0, 1, 0) - pc) * x.g.idy);
  if (x.k <= x.g.hi[2]) x.store_w((double)x.w_in() - dt * (x.p(0, 0, 1) - pc) * x.g.idz);
}

}  // namespace gen
}  // namespace ns
