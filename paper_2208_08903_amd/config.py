"""Run configuration in the layout of the paper's example parameter file
(example2d.toml: [device], [training], [physical], [model] groups, Sec. 2.1 and
its listing), read from TOML into dataclasses, validated, and turned into a
Flow and a Trainer.

Field meanings follow the listing:
  [device]    device_id         GPU ordinal (-1, the CPU, is not supported here)
  [training]  seed              Philox key of the prior draws
              batchsize, epochs, iterations, base_lr
              opt               "Adam"
              prior             a standard normal ("Normal{Float32}(0.f0, 1.f0)")
              lr_scheduler      "" (constant), "step:<gamma>:<every>" or "exp:<gamma>"
              pretrained        "" or the path of a checkpoint written by train.py
  [physical]  L, Nd (2 or 3), M2 (m^2), lam (lambda)
  [model]     seed              seed of the weight initialisation
              n_layers, hidden_sizes, kernel_size, inC (1), outC (2),
              use_final_tanh, use_bn
The listing's [config] version entry is accepted and ignored.  Precision
("bf16" or "fp32", default "bf16") and the initial weight scale (init_std,
default 0.1: weights N(0, init_std^2), biases 0, batch-norm gamma 1, beta 0) sit
in [model] as extensions.
"""
from __future__ import annotations

import re
from dataclasses import dataclass, field, fields

import numpy as np

from . import lfs


class ConfigError(ValueError):
    pass


@dataclass
class DeviceParams:
    device_id: int = 0


@dataclass
class TrainingParams:
    seed: int = 12345
    batchsize: int = 64
    epochs: int = 200
    iterations: int = 100
    base_lr: float = 1e-3
    opt: str = "Adam"
    prior: str = "Normal{Float32}(0.f0, 1.f0)"
    lr_scheduler: str = ""
    pretrained: str = ""


@dataclass
class PhysicalParams:
    L: int = 8
    Nd: int = 2
    M2: float = -4.0
    lam: float = 8.0


@dataclass
class ModelParams:
    seed: int = 2021
    n_layers: int = 16
    hidden_sizes: list = field(default_factory=lambda: [8, 8])
    kernel_size: int = 3
    inC: int = 1
    outC: int = 2
    use_final_tanh: bool = True
    use_bn: bool = False
    precision: str = "bf16"
    init_std: float = 0.1


@dataclass
class RunConfig:
    device: DeviceParams = field(default_factory=DeviceParams)
    training: TrainingParams = field(default_factory=TrainingParams)
    physical: PhysicalParams = field(default_factory=PhysicalParams)
    model: ModelParams = field(default_factory=ModelParams)


_GROUPS = {"device": DeviceParams, "training": TrainingParams, "physical": PhysicalParams,
           "model": ModelParams}
_NORMAL = re.compile(r"^\s*Normal(\{Float(32|64)\})?\(\s*0(\.0*)?(f0)?\s*,\s*1(\.0*)?(f0)?\s*\)\s*$")


def from_dict(d: dict, device_id: int | None = None) -> RunConfig:
    """RunConfig from the parsed TOML tables (device_id, if given, replaces the file's);
    unknown groups or keys are errors."""
    cfg = RunConfig()
    for group, table in d.items():
        if group == "config":
            continue
        if group not in _GROUPS:
            raise ConfigError(f"unknown group [{group}]")
        obj = getattr(cfg, group)
        names = {f.name for f in fields(obj)}
        for k, v in table.items():
            if k not in names:
                raise ConfigError(f"unknown key {k} in [{group}]")
            setattr(obj, k, v)
    if device_id is not None:
        cfg.device.device_id = device_id
    validate(cfg)
    return cfg


def load(path: str, device_id: int | None = None) -> RunConfig:
    try:
        import tomllib as toml
    except ImportError:          # Python < 3.11
        import tomli as toml
    with open(path, "rb") as fh:
        return from_dict(toml.load(fh), device_id)


def lr_schedule(spec: str):
    """None (constant rate) or the trainer's schedule function for lr_scheduler."""
    from .flow import exp_lr, step_lr
    if spec == "":
        return None
    parts = spec.split(":")
    try:
        if parts[0] == "step" and len(parts) == 3:
            return step_lr(float(parts[1]), int(parts[2]))
        if parts[0] == "exp" and len(parts) == 2:
            return exp_lr(float(parts[1]))
    except ValueError as e:
        raise ConfigError(f"bad lr_scheduler {spec!r}: {e}") from None
    raise ConfigError(f"lr_scheduler must be '', 'step:<gamma>:<every>' or 'exp:<gamma>', got {spec!r}")


def validate(cfg: RunConfig) -> None:
    t, p, m = cfg.training, cfg.physical, cfg.model
    if cfg.device.device_id < 0:
        raise ConfigError("device_id = -1 selects the CPU; this implementation runs on the GPU (device_id >= 0)")
    if t.opt != "Adam":
        raise ConfigError(f"opt must be Adam, got {t.opt!r}")
    if not _NORMAL.match(t.prior):
        raise ConfigError(f"prior must be a standard normal, got {t.prior!r}")
    if min(t.batchsize, t.epochs, t.iterations) < 1 or not t.base_lr > 0:
        raise ConfigError("batchsize, epochs, iterations must be >= 1 and base_lr > 0")
    lr_schedule(t.lr_scheduler)
    if p.Nd not in (2, 3) or p.L < 2 or p.L % 2:
        raise ConfigError("Nd must be 2 or 3 and L even and >= 2")
    if m.inC != 1 or m.outC != 2:
        raise ConfigError("the coupling network maps 1 input channel to 2 outputs (s, t)")
    hs = list(m.hidden_sizes)
    if not 1 <= len(hs) <= lfs.MAX_HIDDEN or any(int(h) < 1 or int(h) > 64 for h in hs):
        raise ConfigError(f"hidden_sizes needs 1..{lfs.MAX_HIDDEN} widths in 1..64, got {hs}")
    if m.kernel_size not in (1, 3, 5, 7):
        raise ConfigError("kernel_size must be odd, 1..7")
    if m.precision not in ("bf16", "fp32"):
        raise ConfigError("precision must be bf16 or fp32")
    if m.n_layers < 1:
        raise ConfigError("n_layers must be >= 1")


def layer_blocks(cfg: RunConfig) -> list:
    """(kind, shape) of one layer's packed blocks: W [cout, cin, K^Nd] and b [cout] per
    convolution, with gamma and beta after a hidden convolution's bias under batch norm."""
    m, T = cfg.model, cfg.model.kernel_size ** cfg.physical.Nd
    w = [int(h) for h in m.hidden_sizes]
    out = []
    for i, (ci, co) in enumerate(zip([1] + w, w + [2])):
        out += [("W", (co, ci, T)), ("b", (co,))]
        if m.use_bn and i < len(w):
            out += [("gamma", (co,)), ("beta", (co,))]
    return out


def init_params(cfg: RunConfig) -> np.ndarray:
    """Packed FP32 parameters: weights N(0, init_std^2) from the model seed, biases and
    betas 0, gammas 1."""
    rng = np.random.default_rng(cfg.model.seed)
    parts = []
    for _ in range(cfg.model.n_layers):
        for kind, shape in layer_blocks(cfg):
            n = int(np.prod(shape))
            if kind == "W":
                parts.append(rng.normal(0.0, cfg.model.init_std, n))
            else:
                parts.append(np.full(n, 1.0 if kind == "gamma" else 0.0))
    return np.concatenate(parts).astype(np.float32)


def make_flow(cfg: RunConfig, params=None):
    from .flow import Flow
    m, p = cfg.model, cfg.physical
    prec = lfs.LFS_BF16_CONV if m.precision == "bf16" else lfs.LFS_PLAIN_FP32
    return Flow(p.Nd, p.L, m.n_layers, 0, prec, final_tanh=m.use_final_tanh,
                params=init_params(cfg) if params is None else params,
                device=f"cuda:{cfg.device.device_id}", kernel=m.kernel_size,
                hidden_sizes=[int(h) for h in m.hidden_sizes], batch_norm=m.use_bn)


def make_trainer(cfg: RunConfig, flow, graph: bool = False):
    from .flow import Trainer
    t, p = cfg.training, cfg.physical
    return Trainer(flow, t.batchsize, p.M2, p.lam, lr=t.base_lr, key=t.seed,
                   lr_schedule=lr_schedule(t.lr_scheduler), graph=graph)
