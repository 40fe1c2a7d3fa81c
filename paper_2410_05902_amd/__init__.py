"""MI355X-native mini-batch kernel k-means (hot path of arXiv 2410.05902).

Heavy imports are lazy so that the seeded workload generators
(``paper_2410_05902_amd.workloads``) can be used without torch or the HIP
library being loaded.
"""


def __getattr__(name):
    if name in ("Model",):
        from .model import Model
        return Model
    if name in ("BatchObjective", "batch_objective"):
        from . import autograd as _ag
        return getattr(_ag, name)
    raise AttributeError(name)
