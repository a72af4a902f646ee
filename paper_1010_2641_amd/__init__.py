"""paper_1010_2641_amd -- direct kinematic scattering sums on MI355X (gfx950).

A(S_k) = sum_j f_j exp(2 i pi S_k . r_j) (Favre-Nicolin et al. 2010, Eq. 2) and its
adjoint with respect to the atom positions, computed by hand-written HIP kernels in
libnx.so (C ABI: include/nx.h).  The torch-facing wrappers live in ``api`` and are
loaded on first use, so that ``workloads`` (input generation) imports without the
GPU library.
"""
__all__ = ["scatter", "scatter_fwd", "scatter_bwd", "scatter_fwd_f64", "scatter_bwd_f64",
           "scatter_bwd_ex", "scatter_bwd_ex_f64", "scatter_fwd_species", "scatter_bwd_species",
           "scatter_species", "loss_grad", "fit_step", "fit_step_species", "ScatterFn",
           "ScatterSpeciesFn", "workspace_bytes"]


def __getattr__(name):
    if name in __all__:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
