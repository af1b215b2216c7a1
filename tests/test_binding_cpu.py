"""The Python binding checks every tensor's size against n, P, k and n_perms
before it calls the library, so a mismatched tensor raises PstatError instead
of becoming an out-of-bounds device read or write.  The checks run before any
device call, so they are tested here on CPU tensors."""
import pytest
import torch

ps = pytest.importorskip("paper_2505_04556_amd")

f32, f64, i32 = torch.float32, torch.float64, torch.int32


def einval(fn, *args, **kw):
    with pytest.raises(ps.PstatError) as e:
        fn(*args, **kw)
    assert e.value.code == ps.PSTAT_EINVAL, str(e.value)
    return str(e.value)


def test_sW_shapes():
    D = torch.zeros(10, 10, dtype=f32)
    g = torch.zeros(3, 10, dtype=i32)
    w = torch.ones(2, dtype=f64)
    assert "groupings" in einval(ps.pstat_sW, D, torch.zeros(3, 9, dtype=i32), w)
    assert "out" in einval(ps.pstat_sW, D, g, w, torch.zeros(2, dtype=f64))
    assert "inv_group_sizes" in einval(ps.pstat_sW, D, g, torch.zeros(0, dtype=f64))
    assert "mat" in einval(ps.pstat_sW, torch.zeros(10, 9, dtype=f32), g, w)
    assert "inv_group_sizes" in einval(ps.pstat_sW_k, D, g, 3, w)
    assert "out" in einval(ps.pstat_sW_k, D, g, 2, w, torch.zeros(2, dtype=f64))
    assert "groupings" in einval(ps.pstat_sW_k, D, torch.zeros(30, dtype=i32), 2, w)
    # packed layout: 45 floats are n = 10; 44 are no n at all
    assert "out" in einval(ps.pstat_sW_k, torch.zeros(45, dtype=f32), g, 2, w,
                           torch.zeros(1, dtype=f64))
    einval(ps.pstat_sW_k, torch.zeros(44, dtype=f32), g, 2, w)


def test_registered_handle_shapes():
    assert "unknown handle" in einval(ps.pstat_sW_registered, 987654, torch.zeros(1, 5, dtype=i32),
                                      2, torch.ones(2, dtype=f64))


def test_steps_around_the_statistic():
    s = torch.zeros(5, dtype=f64)
    einval(ps.pstat_sT, torch.zeros(4, 4, dtype=f32), torch.zeros(0, dtype=f64))
    assert "s_T" in einval(ps.pstat_F, s, torch.zeros(0, dtype=f64), 10, 2)
    assert "F" in einval(ps.pstat_F, s, torch.zeros(1, dtype=f64), 10, 2, torch.zeros(4, dtype=f64))
    assert "s_W_obs" in einval(ps.pstat_pvalue, torch.zeros(0, dtype=f64), s)
    assert "p" in einval(ps.pstat_pvalue, s[:1], s, torch.zeros(0, dtype=f64))
    assert "inv" in einval(ps.pstat_group_weights, torch.zeros(8, dtype=i32), 3,
                           torch.zeros(2, dtype=f64))
    assert "groupings" in einval(ps.pstat_permute, torch.zeros(8, dtype=i32), 4, 1,
                                 torch.zeros(3, 8, dtype=i32))


def test_whole_test_shapes():
    D = torch.zeros(10, 10, dtype=f32)
    assert "grouping" in einval(ps.pstat_permanova, D, torch.zeros(9, dtype=i32), 2, 5, 1)
    assert "grouping" in einval(ps.pstat_permanova, D, torch.zeros(11, dtype=i32), 2, 5, 1)
    assert "result" in einval(ps.pstat_permanova, D, torch.zeros(10, dtype=i32), 2, 5, 1,
                              result=torch.zeros(3, dtype=f64))
    assert "sW_all" in einval(ps.pstat_permanova, D, torch.zeros(10, dtype=i32), 2, 5, 1,
                              sW_all=torch.zeros(5, dtype=f64))


def test_serving_shapes():
    D = torch.zeros(10, 10, dtype=f32)
    assert "grouping" in einval(ps.pstat_job_create, 1, D, torch.zeros(9, dtype=i32), 2, 5, 1,
                                torch.zeros(8, dtype=torch.uint8))
    assert "unknown job" in einval(ps.pstat_job_finish, 1, 424242, torch.zeros(6, dtype=f64))
