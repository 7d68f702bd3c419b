"""Configurations of the benchmark workloads (encoding, network, optimizer, run length).

c1: one 64^3 block, L=4, T=2^12, F=2, base 4, growth 2, 1x16 MLP, batch 4096, lr 1e-2, 200 steps.
c2: one 256^3 block, L=16, T=2^19, F=2, base 16, finest 256, 2x64 MLP, batch 2^18, 5000 steps.
c3: 64 uneven blocks (U{96..160} per axis, ghost 1), L=16, T=2^17, F=2, base 16, finest 160,
    2x64 MLP, 2^20 samples per step, 2000 steps.
c4: the c2 model on a 40-step 256^3 advected-blob series, warm-started, 500 steps per timestep.
c5: 512 blocks of 128^3 (ghost 1), L=16, T=2^19, F=2, base 16, finest 128, 2x64, 2^21 samples per step.
gradcheck: 8^3 block, L=3, base 2, growth 2, T=2^6, F=2, 1x16 MLP.
"""
from __future__ import annotations

from .dvnr import EncodingCfg, MlpCfg, OptimCfg

PRESETS = {
    "c1": dict(enc=EncodingCfg(4, 2, 12, 4, 2.0), mlp=MlpCfg(1, 16), optim=OptimCfg(lr=1e-2),
               batch=4096, steps=200),
    "c2": dict(enc=EncodingCfg(16, 2, 19, 16, 0.0, 256), mlp=MlpCfg(2, 64), optim=OptimCfg(lr=1e-2),
               batch=1 << 18, steps=5000),
    "c3": dict(enc=EncodingCfg(16, 2, 17, 16, 0.0, 160), mlp=MlpCfg(2, 64), optim=OptimCfg(lr=1e-2),
               batch=1 << 20, steps=2000),
    "c4": dict(enc=EncodingCfg(16, 2, 19, 16, 0.0, 256), mlp=MlpCfg(2, 64), optim=OptimCfg(lr=1e-2),
               batch=1 << 18, steps=500),
    "c5": dict(enc=EncodingCfg(16, 2, 19, 16, 0.0, 128), mlp=MlpCfg(2, 64), optim=OptimCfg(lr=1e-2),
               batch=1 << 21, steps=3000),
    "gradcheck": dict(enc=EncodingCfg(3, 2, 6, 2, 2.0), mlp=MlpCfg(1, 16), optim=OptimCfg(lr=1e-2),
                      batch=32, steps=1),
}


def get(name: str) -> dict:
    return PRESETS[name]
