"""MD checkpoints that resume bit for bit.

A checkpoint holds the positions and velocities, the positions the
neighbour lists were last built from and the step count, in one ``.npz``
file (plain arrays, no pickled objects).  Forces need no storing: the
first step of ``d3_md_nve`` recomputes them, and because the lists are
rebuilt from the stored build positions (same bins, same sorted order,
same list order) those forces, and every step after them, carry the same
bits as in an uninterrupted run.  The rebuild schedule is the same too:
the stale test measures displacements from the same build positions.

NVE runs draw no random numbers, so there is no generator state to keep.
"""

import numpy as np

from . import d3


def save(path, ctx, pos, vel, step, stream=None):
    """Write pos, vel (device (n,3) FP64 tensors), the positions of the
    context's last build and ``step`` to ``path``."""
    import torch
    build_pos = torch.empty_like(pos)
    d3.d3_build_positions(ctx, build_pos, stream)
    torch.cuda.synchronize()
    np.savez(path, pos=pos.cpu().numpy(), vel=vel.cpu().numpy(),
             build_pos=build_pos.cpu().numpy(), step=np.int64(step))


def load(path):
    """The arrays of a checkpoint: dict with pos, vel, build_pos, step."""
    with np.load(path, allow_pickle=False) as z:
        return {"pos": z["pos"].copy(), "vel": z["vel"].copy(),
                "build_pos": z["build_pos"].copy(), "step": int(z["step"])}


def resume(ctx, state, types, cell, pbc, device="cuda", stream=None):
    """Rebuild ``ctx``'s lists from the checkpoint's build positions
    (``types``: device int32 tensor of the species) and return the
    positions and velocities as device tensors, ready for ``d3_md_nve``."""
    import torch
    bp = torch.as_tensor(state["build_pos"], dtype=torch.float64, device=device).contiguous()
    d3.d3_build_neighbors(ctx, bp, types, cell, pbc, stream)
    pos = torch.as_tensor(state["pos"], dtype=torch.float64, device=device).clone()
    vel = torch.as_tensor(state["vel"], dtype=torch.float64, device=device).clone()
    return pos, vel
