"""Matrix-free phase-field fracture linear solver for AMD MI355X (gfx950).

The compute path lives in libmfpff.so (HIP kernels behind the C ABI of
include/mfpff.h); this package is its ctypes binding and the autograd
wrapper of the residual.

A quasi-static tension test, step by step (all arrays float64 on the device,
vectors component-blocked [u_0 | ... | u_{d-1} | phi], nodes lexicographic
with axis 0 fastest)::

    from paper_2005_00331_amd import Context, make_problem
    levels = [(16, 2), (32, 2), (64, 2)]                 # (cells per direction, degree), coarse to fine
    ctx = Context(make_problem(2, levels, eps=2 / 64, split="amor", pdas_project=True))
    nn = ctx.n_nodes
    u = torch.zeros(2 * nn, dtype=torch.float64, device="cuda")
    # phi0: 1 off the initial crack, 0 on it.  A load-free step first relaxes the sharp band into
    # the phase-field profile, so that the extrapolated phi~ of the loaded steps starts from it.
    phi_prev = phi0.clone()
    ctx.load_step(u, phi_prev, phi0, None, [0.0, 0.0], raise_on_noconv=False)
    phi_prev2 = None
    for t in range(1, n_steps + 1):
        phi = phi_prev.clone()
        active, info = ctx.load_step(u, phi, phi_prev, phi_prev2, [0.0, t * du])
        # info["reaction_top"] is the load on the pulled face; u, phi hold the new state
        phi_prev2, phi_prev = phi_prev, phi

Lower-level calls: ``newton_step`` (one step of Algorithm 1), ``pdas_solve``
(Algorithm 1 to its stopping test), ``set_linearization`` + ``gmres_solve``
(one linear solve), ``apply_jacobian``, ``vcycle``, ``residual``.
"""
from .binding import (F32, F64, OP_ACCUMULATE, OP_BLOCKDIAG, OP_G, OP_GT, Context, MfpffError, Problem,  # noqa: F401
                      load_library, make_problem, problem_from)
