"""Listed-candidate evaluation (dagbound_eval_listed), the GPU input generator
of explicit candidate bytes, and model checkpoints (dagbound_model_save /
dagbound_model_load) on the GPU.  Listed bounds are compared with the CPU
oracle on the same candidate bytes; a resumed model must continue training
bit for bit like the uninterrupted one."""
import os
import struct

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_20826_amd as db

    db.load_library()
    return torch, db


def say(*a):
    print(*a, flush=True)


def dev_inputs(torch, batch):
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    return [t(batch.node_off), t(batch.edge_off), t(batch.src), t(batch.dst), t(batch.wcet), t(batch.par)]


@pytest.mark.parametrize("wk,count,K", [(1, 50, 16), (3, 40, 256), (5, 3, 64)])
def test_device_bytes_equal_host_bytes(env, wk, count, K):
    torch, db = env
    wl = W.WORKLOADS[wk]
    batch = W.generate_workload(wk, count=count)
    ins = dev_inputs(torch, batch)
    say("device candidate bytes", wl.name.split(":")[0], count, K)
    out = torch.full((int(batch.node_off[-1]) * K,), 0xAB, dtype=torch.uint8, device="cuda:0")
    W.alloc_bytes_device(ins[0], ins[5], count, int(np.diff(batch.node_off).max()), wl.num_cus, K, wl.seed, out)
    torch.cuda.synchronize()
    want = W.alloc_bytes(batch, wl.num_cus, K, seed=wl.seed)
    assert np.array_equal(out.cpu().numpy(), want)


def test_device_bytes_of_a_later_range(env):
    # DAGs first..first+count-1 of a stream: the DAG index enters the hash
    torch, db = env
    wl = W.WORKLOADS[2]
    batch = W.generate_workload(2, count=30, first=500)
    ins = dev_inputs(torch, batch)
    out = torch.empty(int(batch.node_off[-1]) * 8, dtype=torch.uint8, device="cuda:0")
    W.alloc_bytes_device(ins[0], ins[5], 30, int(np.diff(batch.node_off).max()), 256, 8, 77, out, first=500)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), W.alloc_bytes(batch, 256, 8, seed=77, first=500))


@pytest.mark.parametrize("seeded", [False, True])
def test_listed_bounds_match_oracle(env, seeded):
    torch, db = env
    # every size class: small-er, batched-layered, persistent-mixed (up to 502 nodes), two large DAGs
    parts = [W.generate_workload(1, count=20), W.generate_workload(2, count=20),
             W.generate_workload(3, count=30), W.generate_workload(5, count=2)]
    batch = W.from_dags([p.dag(d) for p in parts for d in range(p.num_dags)])
    D, M, K, L = batch.num_dags, 256, 70, 9
    rng = np.random.default_rng(4)
    cand = rng.integers(0, K, (D, L)).astype(np.int32)
    cand[:, 0] = 0
    cand[:, 3] = cand[:, 2]  # repeats allowed
    ins = dev_inputs(torch, batch)
    b = db.create_batch(*ins, M)
    alloc = W.alloc_bytes(batch, M, K, seed=21)
    if seeded:
        db.set_allocations(b, K, db.ALLOC_SEEDED, None, 21)
    else:
        a_dev = torch.from_numpy(alloc).to("cuda:0")
        db.set_allocations(b, K, db.ALLOC_EXPLICIT, a_dev)
    say("eval_listed", D, "DAGs", L, "entries, seeded" if seeded else "explicit")
    c_dev = torch.from_numpy(cand.ravel().copy()).to("cuda:0")
    got = torch.empty(D * L, dtype=torch.int64, device="cuda:0")
    cp = torch.empty_like(got)
    it = torch.empty_like(got)
    db.eval_listed(b, c_dev, got, cp, it)
    got, cp, it = (x.cpu().numpy().reshape(D, L) for x in (got, cp, it))
    lb = W.alloc_bytes_list(batch, M, cand, seed=21)
    want, wcp, wit = oracle.bounds_batch(batch, M, L, lb, threads=8)
    assert np.array_equal(got, want)
    assert np.array_equal(cp, wcp) and np.array_equal(it, wit)
    # the same through host pointers, and equal to the gathered full evaluation
    host = np.zeros(D * L, np.int64)
    db.eval_listed(b, cand.ravel().copy(), host)
    assert np.array_equal(host.reshape(D, L), want)
    full = torch.empty(D * K, dtype=torch.int64, device="cuda:0")
    db.eval_bounds(b, full)
    full = full.cpu().numpy().reshape(D, K)
    assert np.array_equal(np.take_along_axis(full, cand.astype(np.int64), 1), want)
    b.close()


def test_listed_ids_out_of_range_are_rejected(env):
    torch, db = env
    batch = W.generate_workload(1, count=5)
    b = db.create_batch(*dev_inputs(torch, batch), 8)
    db.set_allocations(b, 16, db.ALLOC_SEEDED, None, 3)
    out = torch.zeros(5 * 2, dtype=torch.int64, device="cuda:0")
    for bad in (16, -1):
        cand = torch.zeros(10, dtype=torch.int32, device="cuda:0")
        cand[7] = bad
        with pytest.raises(db.DagboundError) as e:
            db.eval_listed(b, cand, out)
        assert e.value.code == -1 and "outside" in e.value.message
        assert not out.any()  # nothing evaluated
        with pytest.raises(db.DagboundError):
            db.eval_listed(b, cand.cpu().numpy(), np.zeros(10, np.int64))
    b.close()


def _train_steps(torch, db, model, shards, steps):
    losses = []
    for i in range(steps):
        sh = shards[i % len(shards)]
        losses.append(db.model_train_step(model, sh[0], sh[1], sh[2], sh[3], 1e-3))
    return losses


def test_checkpoint_resumes_training_bit_for_bit(env, tmp_path):
    torch, db = env
    from paper_2602_20826_amd import proposal as P

    M = 256
    dags = W.generate_workload(4, count=60, first=10**6)
    shards = [(s.batch, s.K, s.seed, s.bounds) for s in P.label_shards(torch, dags, M, 64, seed=11, per_shard=20)]
    say("checkpoint: train 4 steps, save, train 3 more; resume from the file")
    a = db.Model(9)
    _train_steps(torch, db, a, shards, 4)
    path = str(tmp_path / "model.dbm")
    a.save(path)
    assert not os.path.exists(path + ".tmp")
    saved = a.params()
    la = _train_steps(torch, db, a, shards, 3)
    pa = a.params()
    b = db.Model(123)  # different initial weights
    b.load(path)
    assert b.step() == 4
    assert np.array_equal(b.params(), saved)
    lb = _train_steps(torch, db, b, shards, 3)
    assert la == lb
    assert np.array_equal(b.params(), pa)
    assert b.step() == 7
    # the file: header fields and the checksum over parameters and both moments
    raw = open(path, "rb").read()
    magic, version, hbytes, nparams, step, fin, hid, layers, out, checksum = struct.unpack("<8sIIqqiiiiQ", raw[:56])
    assert magic == b"DAGBMDL\0" and version == 1 and hbytes == 56
    assert nparams == db.dagbound.MODEL_PARAMS and step == 4 and (fin, hid, layers, out) == (8, 128, 3, 4)
    body = np.frombuffer(raw[56:], np.uint8)
    assert body.size == 3 * 4 * nparams
    h = 0xCBF29CE484222325
    for x in body.tobytes():
        h = ((h ^ x) * 0x100000001B3) & (2**64 - 1)
    assert h == checksum
    assert np.array_equal(np.frombuffer(raw[56:56 + 4 * nparams], np.float32), saved)
    # a model without moments (fresh) restarts Adam; the loaded one does not
    c = db.Model(9)
    c.set_params(saved)
    lc = _train_steps(torch, db, c, shards, 3)
    assert lc[0] == la[0] and not np.array_equal(c.params(), pa)
    for m in (a, b, c):
        m.close()
    for s in shards:
        s[0].close()


def test_checkpoint_rejects_bad_files(env, tmp_path):
    torch, db = env
    m = db.Model(1)
    p0 = m.params()
    path = str(tmp_path / "m.dbm")
    m.save(path)
    raw = bytearray(open(path, "rb").read())
    cases = {
        "missing": None,
        "magic": bytes(b"XAGBMDL\0") + raw[8:],
        "version": raw[:8] + struct.pack("<I", 2) + raw[12:],
        "short": raw[:-4],
        "long": raw + b"\0",
        "checksum": raw[:100] + bytes([raw[100] ^ 1]) + raw[101:],
        "arch": raw[:32] + struct.pack("<i", 16) + raw[36:],
    }
    for name, data in cases.items():
        f = str(tmp_path / f"bad_{name}.dbm")
        if data is not None:
            open(f, "wb").write(bytes(data))
        with pytest.raises(db.DagboundError) as e:
            m.load(f)
        assert e.value.code == db.dagbound.E_IO, name
    assert np.array_equal(m.params(), p0)  # a failed load leaves the model as it was
    with pytest.raises(db.DagboundError) as e:
        m.save(str(tmp_path / "no_such_dir" / "m.dbm"))
    assert e.value.code == db.dagbound.E_IO
    m.close()
