"""MI355X-native MCF phase unwrapping: residues, integer likelihood-ratio edge
costs, successive-shortest-path minimum-cost flow and integration, all in HIP
kernels for gfx950 behind the C ABI of include/ww.h.

The HIP library is loaded on first use (``paper_2609_36267_amd.binding``);
``paper_2609_36267_amd.synth`` (seeded synthetic inputs) needs no GPU.
"""
__all__ = ["binding", "synth", "build"]


def __getattr__(name):
    if name in ("residues", "build_cost_lut", "edge_costs", "mcf_solve", "integrate", "unwrap",
                "default_cost_params", "default_lut_params", "WWError", "load"):
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
