"""The five workloads the hot path is built and measured on.

Each entry fixes the mosaic generator, the model parameters and the targets.
Parameters the workload descriptions leave open are filled with the values
of the large workload (switch 1e-3, flip 1e-4, mu 1e-4, spacings with mean
1e-3), which is the reading recorded in the design notes.
"""

from __future__ import annotations

import os
from typing import Dict

import numpy as np

from .mosaic import (MosaicSpec, cache_dir, evenly_spaced_targets, mosaic_haplotypes,
                     rho_from_spacings, spacings)

CONFIGS: Dict[str, dict] = {
    # plain FP64 forward+backward, full oracle parity
    "c1": dict(N=200, L=2000, K=20, beta_a=0.5, switch=0.01, flip=1e-3,
               mu=1e-3, d_mean=0.01, T=10, seed=11),
    # plain vs FP32-scaled sweep, N x N distances at 100 targets
    "c2": dict(N=10_000, L=100_000, K=200, beta_a=0.5, switch=1e-3, flip=1e-4,
               mu=1e-4, d_mean=1e-3, T=100, seed=22),
    # precision study; 60% of variants rare (MAF < 1%) at founder level
    "c3": dict(N=50_000, L=20_000, K=1000, beta_a=0.2, rare_fraction=0.6,
               switch=1e-3, flip=1e-4, mu=1e-4, d_mean=1e-3, T=20, seed=33),
    # differentiation: PAC log-likelihood and its gradient
    "c4": dict(N=2000, L=50_000, K=100, beta_a=0.5, switch=1e-3, flip=1e-4,
               mu=1e-4, d_mean=1e-3, T=0, seed=44),
    # large single-GPU case, FP32 only
    "c5": dict(N=100_000, L=10_000, K=5000, beta_a=0.5, switch=5e-4, flip=1e-4,
               mu=1e-4, d_mean=1e-3, T=5, seed=55),
}


def get_config(name: str) -> dict:
    if name not in CONFIGS:
        raise KeyError(f"unknown config {name!r}; known: {sorted(CONFIGS)}")
    return dict(CONFIGS[name])


def spec_of(cfg: dict) -> MosaicSpec:
    return MosaicSpec(n_haps=cfg["N"], n_variants=cfg["L"], n_founders=cfg["K"],
                      switch=cfg["switch"], flip=cfg["flip"], seed=cfg["seed"],
                      beta_a=cfg.get("beta_a", 0.5),
                      rare_fraction=cfg.get("rare_fraction"),
                      rare_maf=cfg.get("rare_maf", 0.01))


def make_inputs(cfg, unpacked: bool = False, use_cache: bool = True) -> dict:
    """Materialise a workload: packed haplotypes, rho, mu and targets.

    ``cfg`` is a config name or a dict with the keys used in ``CONFIGS``.
    Large matrices are cached on disk (``LSINPUTS_CACHE``, default
    /tmp/lsinputs_cache) keyed by the generator spec.
    """
    if isinstance(cfg, str):
        cfg = get_config(cfg)
    spec = spec_of(cfg)
    N, L = cfg["N"], cfg["L"]
    packed = h01 = None
    path = os.path.join(cache_dir(), f"mosaic_{spec.key()}.npy")
    if use_cache and not unpacked and os.path.exists(path):
        try:
            packed = np.load(path, allow_pickle=False)
        except (OSError, ValueError):
            packed = None
    if packed is None:
        packed, h01 = mosaic_haplotypes(spec, unpacked=unpacked)
        if use_cache and N * L >= 10_000_000:
            tmp = path + f".{os.getpid()}.tmp.npy"
            np.save(tmp, packed)
            os.replace(tmp, path)
    d = spacings(L - 1, cfg["d_mean"], cfg["seed"] + 1_000_003)
    rho = rho_from_spacings(d)
    T = cfg.get("T", 0)
    targets = evenly_spaced_targets(L, T).astype(np.int32) if T else np.zeros(0, np.int32)
    return dict(N=N, L=L, H=packed, stride=int(packed.shape[1]), rho=rho,
                mu=float(cfg["mu"]), targets=targets, h01=h01, cfg=cfg)
