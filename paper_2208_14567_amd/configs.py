"""The measured configurations in one place: workloads, sizes, seeds, steps and
the escalation bands, read by bench.py (its command-line flags override them).

Workloads name gen.workload generators (synthetic inputs with the paper's
shapes: "Generating Valid Topologies", "Finding Valid Initial Positions").  The
bands are the library's defaults (links_sim_opts_default): the discriminant
band eps_disc on disc = K / (4 scale^2) in units of scale^2, the branch band
eps_branch on the branch distance in units of scale, and the drift tolerance
tau_drift in units of scale.
"""

T = 200  # actuator positions per turn ("Dataset Features & Statistics")

BANDS = {"eps_disc": 1e-6, "eps_branch": 1e-5, "tau_drift": 1e-4}

CONFIGS = {
    "cfg1": {"workload": "fourbar", "candidates": 10_000, "seed": 1, "T": T,
             "what": "crank-rocker four-bars with a coupler point; GPU FP64 and FP32 with hand-over against the "
                     "oracle"},
    "cfg2": {"workload": "dyad_6_20", "candidates": 1_000_000, "seed": 2, "T": T,
             "what": "the headline: dyad-built candidates, n ~ U{6..20}, FP32 with FP64 hand-over against plain "
                     "FP64, valid paths compacted and PCA-normalised"},
    "cfg2_rules": {"workload": "dyad_rules_6_20", "candidates": 1_000_000, "seed": 11, "T": T,
                   "what": "cfg2 with the paper's topology rules, generated on the device"},
    "cfg3": {"workload": "dyad_skewed", "candidates": 4_000_000, "seed": 3, "T": T,
             "what": "skewed joint counts (60% U{6..8}, 30% U{9..14}, 10% U{15..20})"},
    "cfg4": {"workload": "dyad_4_20", "pool": 500_000, "seed": 4, "requests": 2000, "sizes": (1, 200_000),
             "offsets_seed": 44, "T": T, "tick_max": 1 << 20, "ring_bytes": 2 << 30, "loads": (0.5, 0.8),
             "what": "serving: log-uniform request sizes, saturated and Poisson arrivals at fractions of the "
                     "saturated rate"},
    "cfg5": {"workload": "dyad (device generator)", "chunk": 4_000_000, "chunks": 25, "seed": 5, "T": T,
             "cap": 1_000_000,
             "what": "100M candidates streamed in chunks, valid paths normalised and copied to host memory"},
}
