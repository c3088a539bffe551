"""Inputs of the learned cap corrector: the network's weight layout, seeded
initial weights, the counter-based uniforms that training candidates are
drawn from, and the training recipe.  No arithmetic of the method here."""
import numpy as np

HIDDEN = 128
# flat weight layout (row = output unit): W1[128][6] b1[128] W2[128][128] b2[128] W3[3][128] b3[3]
OFFSETS = {"W1": (0, (HIDDEN, 6)), "b1": (768, (HIDDEN,)), "W2": (896, (HIDDEN, HIDDEN)),
           "b2": (17280, (HIDDEN,)), "W3": (17408, (3, HIDDEN)), "b3": (17792, (3,))}
N_WEIGHTS = 17795

_G = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_at(seed, idx):
    """Outputs number idx (0-based, any integer array) of the SplitMix64 stream
    of `seed` as doubles in [0,1): the same values as splitmix64_uniform."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (idx + np.uint64(1)) * _G
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def cap_uniforms(seed, first, n):
    """The ten uniforms of training candidates first .. first+n-1: candidate c
    takes stream outputs 10c .. 10c+9."""
    idx = (np.arange(first, first + n, dtype=np.uint64)[:, None] * np.uint64(10) +
           np.arange(10, dtype=np.uint64)[None, :])
    return splitmix64_at(seed, idx)


def mlp_init(seed, bias_scale=0.0):
    """Uniform initial weights, bound sqrt(6/fan_in) (W3: sqrt(1/fan_in)),
    biases uniform in +-bias_scale; float32 in the flat layout."""
    u = splitmix64_at(seed, np.arange(N_WEIGHTS)) * 2.0 - 1.0
    w = np.zeros(N_WEIGHTS)
    for name, (off, shape) in OFFSETS.items():
        n = int(np.prod(shape))
        if name.startswith("W"):
            fan_in = shape[1]
            bound = np.sqrt((1.0 if name == "W3" else 6.0) / fan_in)
        else:
            bound = bias_scale
        w[off:off + n] = u[off:off + n] * bound
    return w.astype(np.float32)


# training recipe of the learned workload: partial items of the h = delta/8
# family (legs 1/8 in units of delta, +-0.1 h jitter, both diagonals, random
# cyclic vertex order) outside the 0.02 delta fallback band
TRAIN = dict(samples=4_000_000, seed=20052, L=0.125, jitter=0.1, band=0.02, cap_edges=8,
             epochs=20, batch=4096, lr=1e-3)
